// Continuous-batching UQ server: a request loop on its own host thread that
// admits jobs of different lattices and sample counts by device-memory
// footprint, keeps their populations resident, and advances every sample of
// every live job together (the non-intrusive UQ algorithm of OpenLB-UQ,
// Algorithm alg:uq_openlb, with the per-sample solve loop of all concurrent
// requests batched). Periodic vortex lattices and channels with node-local
// boundary rules run temporally blocked: N steps per launch over whole rows,
// one batched launch per kernel instance for all jobs that share it; other
// jobs advance one step per launch in one batched launch per step. A "plain"
// mode runs the same arithmetic one job at a time and one sample per launch,
// for comparison.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "uq_job.h"

namespace uqi {

// ------------------------------------------------------------------ arena
// One device allocation made at server start, carved first-fit into 256-byte
// aligned blocks; freed blocks coalesce with their neighbours. Serving never
// calls hipMalloc or hipFree (hipFree would synchronise the device).
class Arena {
   public:
    // from the caller's allocator if it has one, else hipMalloc
    uq_status init(size_t bytes, const uq_device &dev) {
        cap_ = (bytes + 255) / 256 * 256;
        dev_ = dev;
        if (dev_.alloc) {
            base_ = (char *)dev_.alloc(cap_, dev_.ctx);
        } else if (hipMalloc(&base_, cap_) != hipSuccess) {
            (void)hipGetLastError();
            base_ = nullptr;
        }
        if (!base_) return fail(UQ_ENOMEM, "server arena of " + std::to_string(cap_) + " B does not fit on the device");
        free_[0] = cap_;
        return UQ_OK;
    }
    // (the caller makes sure no work on the arena is pending)
    ~Arena() {
        if (!base_) return;
        if (dev_.alloc) {
            if (dev_.free) dev_.free(base_, dev_.ctx);
        } else {
            (void)hipFree(base_);
        }
    }
    void *alloc(size_t n) {
        std::lock_guard<std::mutex> lk(mu_);
        n = (n + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, sz = it->second;
            free_.erase(it);
            if (sz > n) free_[off + n] = sz - n;
            used_[off] = n;
            in_use_ += n;
            peak_ = std::max(peak_, in_use_);
            return base_ + off;
        }
        return nullptr;
    }
    void release(void *p) {
        std::lock_guard<std::mutex> lk(mu_);
        const size_t off = (size_t)((char *)p - base_);
        auto u = used_.find(off);
        if (u == used_.end()) return;
        size_t sz = u->second, start = off;
        used_.erase(u);
        in_use_ -= sz;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && next->first == off + sz) {
            sz += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                sz += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = sz;
    }
    size_t capacity() const { return cap_; }
    size_t in_use() {
        std::lock_guard<std::mutex> lk(mu_);
        return in_use_;
    }
    size_t peak() {
        std::lock_guard<std::mutex> lk(mu_);
        return peak_;
    }
    size_t largest_free() {
        std::lock_guard<std::mutex> lk(mu_);
        size_t m = 0;
        for (auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }

   private:
    char *base_ = nullptr;
    uq_device dev_{};
    size_t cap_ = 0, in_use_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_, used_;
    std::mutex mu_;
};

static void *arena_alloc_cb(size_t n, void *ctx) { return ((Arena *)ctx)->alloc(n); }
static void arena_free_cb(void *p, void *ctx) { ((Arena *)ctx)->release(p); }

static size_t up256(size_t n) { return (n + 255) / 256 * 256; }

// The batched instance that carries a job: periodic vortex lattices (kind
// 0) and channels whose boundary rules are node-local (kind 1: half-way
// walls and cylinder, Zou-He or wall or periodic ends) advance N steps per
// launch over whole rows of H-row chunks in the AB layout; vortex lattices
// too wide for whole rows, 4 steps per launch in strips (kind 2); kind -1:
// one step per launch in the AA layout (the batched single-step kernel). A shape the
// launch-shape tuner measured for the job's class is taken when it is a
// batched instance; otherwise N is the largest of the instance's choices
// whose LDS rings fit the row width (vortex 8, 6, 4, or 6, 8, 4 up to 128
// columns; channel 4, 3, 2), the vortex takes equal chunks of at most 256
// rows, and the channel cuts its rows into
// chunks so that its samples fill the GPU (at most 8, as the tuner tries).
struct ServeShape {
    int kind = -1, N = 0, K = 0, M = 0, H = 0;
    int W = 0, strips = 1;
};

int64_t job_footprint(const uq_problem &p, int64_t S, int K, bool ab);

static ServeShape serve_shape(const uq_problem &p, int64_t S, int K, size_t arena) {
    ServeShape sh;
    if (p.precision == UQ_FP64) return sh;
    const int64_t b = storage_bytes(p.precision);
    const int64_t plane = (int64_t)p.ny * row_pitch(p.nx) + 64;
    if (9 * plane * b >= ((int64_t)1 << 31) || plane * 4 >= ((int64_t)1 << 31)) return sh;
    int kind = -1;
    if (p.geometry == UQ_GEOM_TGV) kind = 0;
    else if (p.geometry == UQ_GEOM_CHANNEL && !needs_ab(p) && p.cyl_bc == UQ_CYL_HALFWAY) kind = 1;
    if (kind < 0) return sh;
    sh.W = p.nx;
    // vortex lattices of at most 128 columns (one column per lane) run
    // fastest at 6 steps per launch, wider ones at 8 (measured per width on
    // the serving mix); channels take the deepest pipeline that fits
    const bool narrow = p.nx <= 128;
    const int pref[2][3] = {{narrow ? 6 : 8, narrow ? 8 : 6, 4}, {4, 3, 2}};
    StepShape tuned;
    const bool have = tuned_shape(p, S, &tuned) && tuned.fwin == 2 && tuned.fuse >= 2;
    for (int c = -1; c < 3; ++c) {
        const int n = c < 0 ? (have ? tuned.fuse : 0) : pref[kind][c];
        int K = 0, M = 0;
        if (n < 2 || !rows_instance(kind, p.precision, n, p.nx, &K, &M) ||
            !fused_multi_supported(kind, p.precision, n, K, M))
            continue;
        sh.kind = kind;
        sh.N = n;
        sh.K = K;
        sh.M = M;
        if (c < 0) {
            sh.H = std::max(8, std::min(tuned.fty, p.ny));
        } else if (kind == 0) {
            // chunks of at most 256 rows, all of one height (a short last
            // chunk would hold its work item's CU for a full pipeline fill)
            const int chunks = (p.ny + 255) / 256;
            sh.H = std::max(8, (p.ny + chunks - 1) / chunks);
        } else {
            const int chunks = (int)std::min<int64_t>(8, std::max<int64_t>(1, (256 + S - 1) / S));
            sh.H = std::max(8, (p.ny + chunks - 1) / chunks);
        }
        return sh;
    }
    // vortex rows too wide for any whole-row instance: 4 steps per launch
    // in strips of 32-row chunks, if the job's two slabs take at most two
    // fifths of the arena (a larger job would hold back every other
    // admission; it runs in AA). (32 rows ran the serving mix's strip jobs
    // 4 % faster than 64: more, shorter work items.)
    if (kind == 0 && (size_t)job_footprint(p, S, K, true) <= arena * 2 / 5) {
        sh.kind = 2;
        sh.N = 4;
        sh.H = std::max(8, std::min(32, p.ny));
        window_strips(p.nx, sh.N, &sh.W, &sh.strips);
    }
    return sh;
}

// Device bytes a job takes in the server (scalar moments): slab (two in the
// AB layout), per-sample records, step counter, boundary mask, basis table,
// QoI buffers and the non-finite flag.
int64_t job_footprint(const uq_problem &p, int64_t S, int K, bool ab) {
    const int64_t pitch = row_pitch(p.nx);
    const int64_t plane = (int64_t)p.ny * pitch + 64;
    size_t b = up256((size_t)(S * 9 * plane * storage_bytes(p.precision))) * (ab ? 2 : 1);
    b += up256(sizeof(SampleDev) * S) + 256;
    if (p.geometry == UQ_GEOM_CHANNEL) b += up256(sizeof(uint32_t) * p.ny * pitch);
    if (K > 0) b += up256(sizeof(double) * S * K) + up256(sizeof(double) * S);
    b += up256(sizeof(double) * 4 * S) + up256(sizeof(double) * S) + up256(sizeof(double) * (K + 3)) + 256;
    return (int64_t)b;
}

struct Request {
    uint64_t ticket = 0;
    uq_problem p{};
    int64_t steps = 0;
    int32_t qoi = 0;
    int64_t S = 0;
    int K = 0;
    ServeShape shape;  // kind -1 in PLAIN mode
    int64_t footprint = 0;
    double t_submit = 0.0;
};

struct Live {
    Request r;
    uq_job *job = nullptr;
    double t_admit = 0.0;
    int tiles_x = 0, tiles_y = 0;
    int mult = 1;  // ticks advance this job mult times the tick's steps
};

// Jobs of the live set that share one batched instance; their table entries
// are fused[first .. first + count).
struct Group {
    int kind = 0, N = 0, K = 0, M = 0, mult = 1;
    int first = 0, count = 0;
    int64_t nwork = 0;
};

// Consecutive single-step jobs of one multiple of the tick: their entries
// end at jobs_end in the table and their tiles at tiles_end.
struct SingleRun {
    int mult = 1, jobs_end = 0;
    int64_t tiles_end = 0;
};

// Steps per tick of the batched mode: a multiple of 48, which holds a whole
// number of launch pairs of every instance (2N divides 48 for N = 2, 3, 4,
// 6, 8), so that every job's state is in the slab of its step's parity
// between ticks and one captured graph serves every tick while the live set
// is unchanged.
static int64_t batched_tick(int64_t steps_per_tick) {
    return std::max<int64_t>(48, (steps_per_tick + 24) / 48 * 48);
}

struct Server {
    uq_server_config cfg{};
    uq_device dev{};
    int device = 0;
    Arena arena;
    hipStream_t stream = nullptr;  // the loop's stream
    hipEvent_t ev = nullptr;
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> pending;
    std::vector<Live> live;
    std::map<uint64_t, uq_result> done;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::string fatal;
    std::thread th;

    // statistics (under mu)
    int64_t submitted = 0, completed = 0, failed = 0;
    double node_updates = 0.0, busy_s = 0.0;
    std::vector<double> latencies;

    // batching tables of the live set (device copies in d_tables, one block
    // the size of max_jobs entries of each kind): single-step jobs, the
    // batched fused instances, and every job's step counter
    void *d_tables = nullptr;
    MultiJob *d_table = nullptr;
    FusedJob *d_fused = nullptr;
    int64_t **d_tptrs = nullptr;
    int table_cap = 0;
    int n_single = 0, n_fused = 0, n_all = 0;
    std::vector<Group> groups;
    std::vector<SingleRun> single_runs;  // single-step jobs by multiple, largest first
    bool dirty = true;
    int64_t total_tiles = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    void loop();
    void admit();
    uq_status rebuild_table();
    uq_status enqueue_tick(int64_t T);
    uq_status tick(int64_t K);
    void finish(Live &l);
    void release_graph() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
    }
};

void Server::admit() {
    std::vector<Request> take;
    {
        std::lock_guard<std::mutex> lk(mu);
        const size_t max_live = cfg.mode == UQ_SERVE_PLAIN ? 1 : (size_t)cfg.max_jobs;
        size_t room = arena.largest_free();
        while (!pending.empty() && live.size() + take.size() < max_live) {
            const Request &r = pending.front();
            if ((size_t)r.footprint > room) break;  // first come, first served
            room -= (size_t)r.footprint;
            take.push_back(r);
            pending.pop_front();
        }
    }
    for (Request &r : take) {
        uq_device dv{};
        dv.device = device;
        dv.stream = stream;
        dv.alloc = arena_alloc_cb;
        dv.free = arena_free_cb;
        dv.ctx = &arena;
        StepShape sh;
        sh.cpt = 1;
        sh.pad = 64;
        sh.nt = 0;
        if (r.shape.kind >= 0) {
            sh.layout = UQ_LAYOUT_AB;
            sh.fuse = r.shape.N;
            sh.fwin = r.shape.kind == 2 ? 1 : 2;
            sh.fty = r.shape.H;
        } else {
            sh.layout = UQ_LAYOUT_AA;
        }
        uq_job *j = nullptr;
        uq_status st = create_job(r.p, &dv, &sh, &j);
        if (st == UQ_ENOMEM) {  // fragmentation: retry when memory frees up
            std::lock_guard<std::mutex> lk(mu);
            pending.push_front(r);
            continue;
        }
        if (st == UQ_OK && hipStreamSynchronize(j->stream) != hipSuccess) st = UQ_EDEVICE;
        if (st == UQ_OK && r.shape.kind >= 0 && j->fused_n() != r.shape.N)
            st = fail(UQ_ESTATE, "server job did not take its batched shape");
        if (st != UQ_OK) {
            uq_result res{};
            res.ticket = r.ticket;
            res.status = st;
            res.qoi = r.qoi;
            res.t_submit = r.t_submit;
            res.t_admit = res.t_done = now();
            if (j) delete j;
            std::lock_guard<std::mutex> lk(mu);
            done[r.ticket] = res;
            ++failed;
            cv_done.notify_all();
            continue;
        }
        j->use_graph = false;
        Live l;
        l.r = r;
        l.job = j;
        l.t_admit = now();
        tile_counts(j->jd, 1, &l.tiles_x, &l.tiles_y);
        std::lock_guard<std::mutex> lk(mu);
        live.push_back(l);
        dirty = true;
    }
}

// Tables of the jobs in `live` that take part in the next ticks.
uq_status Server::rebuild_table() {
    std::vector<MultiJob> single;
    std::vector<FusedJob> fused;
    std::vector<int64_t *> tptrs;
    int64_t tile = 0;
    // batched instances: jobs sorted by instance, each instance contiguous
    std::vector<size_t> order;
    for (size_t q = 0; q < live.size(); ++q)
        if (live[q].r.shape.kind >= 0) order.push_back(q);
    // Work-fair ticks: a tick advances every job by the same number of
    // steps, so a cheap job with many steps (few samples, a small lattice)
    // would need as many ticks as its steps allow, each as long as the
    // whole live set's work, and finish long after the rest. The cheapest
    // jobs take 8, 4 or 2 times the tick's steps (batched instances: in
    // launches of their own instance group; single steps: in the first
    // launches of the tick, which cover the jobs in order of multiple), as
    // long as the extra work stays within a quarter of the live set's work
    // per tick and within the job's remaining steps. A single step moves
    // about four times the bytes of a node update of a temporally blocked
    // launch and is weighted so.
    const int64_t T = batched_tick(cfg.steps_per_tick);
    {
        auto work = [&](size_t q) {
            return (double)live[q].job->S * live[q].r.p.nx * live[q].r.p.ny * (live[q].r.shape.kind < 0 ? 4.0 : 1.0);
        };
        double wtot = 0.0;
        std::vector<size_t> cheap;
        for (size_t q = 0; q < live.size(); ++q) {
            wtot += work(q);
            cheap.push_back(q);
        }
        std::stable_sort(cheap.begin(), cheap.end(), [&](size_t x, size_t y) { return work(x) < work(y); });
        double budget = 0.25 * wtot;
        for (size_t q : cheap) {
            Live &l = live[q];
            l.mult = 1;
            const int64_t rem = l.r.steps - l.job->t;
            for (int m : {8, 4, 2})
                if (m * T <= rem && (m - 1) * work(q) <= budget) {
                    l.mult = m;
                    budget -= (m - 1) * work(q);
                    break;
                }
        }
    }
    auto key = [&](size_t q) {
        const ServeShape &h = live[q].r.shape;
        return std::make_tuple(h.kind, h.N, h.K, h.M, live[q].mult);
    };
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return key(x) < key(y); });
    groups.clear();
    for (size_t q : order) {
        const Live &l = live[q];
        const ServeShape &h = l.r.shape;
        if (groups.empty() || key(q) != std::make_tuple(groups.back().kind, groups.back().N, groups.back().K,
                                                        groups.back().M, groups.back().mult)) {
            Group g;
            g.kind = h.kind;
            g.N = h.N;
            g.K = h.K;
            g.M = h.M;
            g.mult = l.mult;
            g.first = (int)fused.size();
            groups.push_back(g);
        }
        Group &g = groups.back();
        FusedJob f;
        std::memset(&f, 0, sizeof f);
        f.j = l.job->jd;
        f.d_t = l.job->d_t;
        f.H = h.H;
        f.chunks = (l.r.p.ny + h.H - 1) / h.H;
        f.W = h.W;
        f.strips = h.strips;
        f.work0 = g.nwork;
        f.par = (int32_t)(l.job->t & 1);
        g.nwork += l.job->S * f.chunks * f.strips;
        ++g.count;
        fused.push_back(f);
        tptrs.push_back(l.job->d_t);
    }
    // an instance whose jobs give fewer work items than the GPU has CUs
    // takes shorter row chunks: more items, each a shorter pipeline (the
    // extra halo rows cost less than idle CUs). The chunking does not change
    // any node's arithmetic.
    constexpr int64_t kTargetItems = 256;
    for (Group &g : groups) {
        if (g.kind == 2 || g.nwork >= kTargetItems) continue;
        const int hmin = g.N >= 6 ? 32 : 16;
        int64_t w = 0;
        for (int q = g.first; q < g.first + g.count; ++q) {
            FusedJob &f = fused[(size_t)q];
            const int64_t want = (f.chunks * kTargetItems + g.nwork - 1) / g.nwork;
            const int H = std::min(f.H, std::max(hmin, (int)((f.j.ny + want - 1) / want)));
            f.chunks = (f.j.ny + H - 1) / H;
            f.H = std::max(8, (f.j.ny + f.chunks - 1) / f.chunks);  // equal chunks
            f.work0 = w;
            w += (int64_t)f.j.S * f.chunks * f.strips;
        }
        g.nwork = w;
    }
    // single-step jobs in order of multiple, largest first: launch k of a
    // tick covers the prefix of jobs that take more than k steps in it
    std::vector<size_t> sorder;
    for (size_t q = 0; q < live.size(); ++q)
        if (live[q].r.shape.kind < 0) sorder.push_back(q);
    std::stable_sort(sorder.begin(), sorder.end(), [&](size_t x, size_t y) { return live[x].mult > live[y].mult; });
    single_runs.clear();
    for (size_t q : sorder) {
        const Live &l = live[q];
        MultiJob m;
        std::memset(&m, 0, sizeof m);
        m.j = l.job->jd;
        m.t = l.job->t;
        m.n_steps = l.r.steps;
        m.tile0 = tile;
        m.adv = l.mult * T;
        m.tiles_x = l.tiles_x;
        m.tiles_y = l.tiles_y;
        tile += (int64_t)l.job->S * l.tiles_x * l.tiles_y;
        single.push_back(m);
        tptrs.push_back(l.job->d_t);
        if (single_runs.empty() || single_runs.back().mult != l.mult) single_runs.push_back({l.mult, 0, 0});
        single_runs.back().jobs_end = (int)single.size();
        single_runs.back().tiles_end = tile;
    }
    total_tiles = tile;
    if ((int)tptrs.size() > table_cap) return fail(UQ_ESTATE, "more live jobs than the table holds");
    n_single = (int)single.size();
    n_fused = (int)fused.size();
    n_all = (int)tptrs.size();
    if (n_single)
        UQ_HIP_TRY(hipMemcpyAsync(d_table, single.data(), sizeof(MultiJob) * single.size(), hipMemcpyHostToDevice,
                                  stream));
    if (n_fused)
        UQ_HIP_TRY(hipMemcpyAsync(d_fused, fused.data(), sizeof(FusedJob) * fused.size(), hipMemcpyHostToDevice,
                                  stream));
    if (n_all)
        UQ_HIP_TRY(hipMemcpyAsync(d_tptrs, tptrs.data(), sizeof(int64_t *) * tptrs.size(), hipMemcpyHostToDevice,
                                  stream));
    UQ_HIP_TRY(hipStreamSynchronize(stream));  // the host vectors go out of scope
    release_graph();
    dirty = false;
    return UQ_OK;
}

// T steps of every job in the tables (mult T for the jobs of a group with
// a multiplier): each batched instance group in mult T/N launches (launch k
// reads the slab of parity t ^ k of each of its jobs), the single-step jobs
// in T launches, then every job's step counter (a group's counters are
// d_tptrs[first .. first + count), the single-step jobs' follow them).
uq_status Server::enqueue_tick(int64_t T) {
    for (const Group &g : groups)
        for (int k = 0; k < (int)(g.mult * T / g.N); ++k)
            UQ_HIP_TRY(launch_fused_multi(g.kind, cfg.precision, g.N, g.K, g.M, d_fused + g.first, g.count, g.nwork,
                                          k, stream));
    if (n_single) {
        // runs of equal multiple, largest first: launch k covers the runs
        // whose jobs take more than k steps
        for (int k = 0; k < (int)(single_runs.front().mult * T); ++k) {
            size_t r = 0;
            while (r + 1 < single_runs.size() && single_runs[r + 1].mult * T > k) ++r;
            UQ_HIP_TRY(launch_step_multi(d_table, single_runs[r].jobs_end, single_runs[r].tiles_end, k, cfg.precision,
                                         stream));
        }
        UQ_HIP_TRY(launch_advance_multi(d_table, n_single, stream));
    }
    for (const Group &g : groups) UQ_HIP_TRY(launch_advance_ptrs(d_tptrs + g.first, g.count, g.mult * T, stream));
    int prev = 0;
    for (const SingleRun &r : single_runs) {
        UQ_HIP_TRY(launch_advance_ptrs(d_tptrs + n_fused + prev, r.jobs_end - prev, r.mult * T, stream));
        prev = r.jobs_end;
    }
    return UQ_OK;
}

// Advance every job of the tables by K steps (batched: K is the tick).
uq_status Server::tick(int64_t K) {
    if (cfg.mode == UQ_SERVE_PLAIN) {
        // one job, one sample per launch, no graph
        Live &l = live.front();
        Job *j = l.job;
        const int64_t bytes_sample = 9 * j->jd.plane * storage_bytes(j->p.precision);
        StepShape sh;
        sh.layout = UQ_LAYOUT_AA;
        sh.cpt = 1;
        for (int64_t k = 0; k < K; ++k)
            for (int64_t s = 0; s < j->S; ++s) {
                JobDev v = j->jd;
                v.S = 1;
                v.f = (char *)j->jd.f + s * bytes_sample;
                v.smp = j->jd.smp + s;
                UQ_HIP_TRY(launch_step(v, j->d_t, (int)k, (int)((j->t + k) & 1), sh, stream));
            }
        UQ_HIP_TRY(launch_advance(j->d_t, K, stream));
        UQ_HIP_TRY(hipStreamSynchronize(stream));
        j->t += K;
        return UQ_OK;
    }
    if (cfg.use_graph && !gexec) {
        UQ_HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        uq_status st = enqueue_tick(K);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(stream, &g);
        if (st != UQ_OK || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(UQ_EDEVICE, "server graph capture failed");
        }
        graph = g;
        UQ_HIP_TRY(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    }
    if (cfg.use_graph) {
        UQ_HIP_TRY(hipGraphLaunch(gexec, stream));
    } else {
        uq_status st = enqueue_tick(K);
        if (st != UQ_OK) return st;
    }
    UQ_HIP_TRY(hipStreamSynchronize(stream));
    for (Live &l : live) l.job->t += K * l.mult;
    return UQ_OK;
}

void Server::finish(Live &l) {
    Job *j = l.job;
    uq_result res{};
    res.ticket = l.r.ticket;
    res.qoi = l.r.qoi;
    res.S = j->S;
    res.K = j->K;
    res.t_submit = l.r.t_submit;
    res.t_admit = l.t_admit;
    const double *M;
    int64_t n, ld;
    uq_status st = j->sample_values(l.r.qoi, &M, &n, &ld);
    if (st == UQ_OK) {
        double *dm = j->d_out, *dv = j->d_out + 1, *da = j->d_out + 2, *dc = j->d_out + 3;
        hipError_t e = launch_scalar_moments(M, j->S, j->d_wphi, j->d_a, j->K, dc, dm, dv, da, j->stream);
        std::vector<double> h((size_t)(3 + j->K));
        if (e == hipSuccess)
            e = hipMemcpyAsync(h.data(), j->d_out, sizeof(double) * h.size(), hipMemcpyDeviceToHost, j->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(j->stream);
        if (e != hipSuccess) {
            st = fail(UQ_EDEVICE, hipGetErrorString(e));
        } else {
            res.mean = h[0];
            res.var = h[1];
            res.var_alt = h[2];
            const int nk = std::min(j->K, (int)UQ_RESULT_MAX_COEFFS);
            for (int k = 0; k < nk; ++k) res.coeffs[k] = h[(size_t)(3 + k)];
        }
    }
    res.status = st;
    res.node_updates = (double)j->S * j->p.nx * j->p.ny * (double)l.r.steps;
    res.t_done = now();
    (void)hipSetDevice(device);
    delete l.job;  // returns its blocks to the arena
    l.job = nullptr;
    std::lock_guard<std::mutex> lk(mu);
    done[res.ticket] = res;
    if (st == UQ_OK) {
        ++completed;
        latencies.push_back(res.t_done - res.t_submit);
        node_updates += res.node_updates;
    } else {
        ++failed;
    }
    cv_done.notify_all();
}

void Server::loop() {
    (void)hipSetDevice(device);
    auto die = [&](const std::string &msg) {
        std::lock_guard<std::mutex> lk(mu);
        fatal = msg;
        stop = true;
        cv_done.notify_all();
    };
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] { return stop || !pending.empty() || !live.empty(); });
            if (stop) return;  // destroy: outstanding work is abandoned
        }
        admit();
        if (live.empty()) {
            // nothing fits: wait for a change (pending jobs are larger than the arena can hold now)
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait_for(lk, std::chrono::milliseconds(5));
            continue;
        }
        const bool plain = cfg.mode == UQ_SERVE_PLAIN;
        int64_t K = plain ? std::min<int64_t>(cfg.steps_per_tick, live.front().r.steps - live.front().job->t)
                          : batched_tick(cfg.steps_per_tick);
        // batched: jobs with fewer steps left than a tick leave the tables
        // and take their last steps in launches of their own (the same
        // arithmetic: fused and single steps agree bit for bit)
        std::vector<Live> ending;
        if (!plain) {
            std::vector<Live> keep;
            for (Live &l : live) (l.r.steps - l.job->t < K ? ending : keep).push_back(l);
            if (!ending.empty()) {
                std::lock_guard<std::mutex> lk(mu);
                live.swap(keep);
                dirty = true;
            }
            // a job whose multiple of the tick no longer fits its remaining
            // steps gets a smaller one
            for (const Live &l : live)
                if (l.mult > 1 && l.r.steps - l.job->t < l.mult * K) dirty = true;
            if (dirty && !live.empty()) {
                uq_status st = rebuild_table();
                if (st != UQ_OK) return die(uq_last_error());
            }
        }
        const double tb = now();
        for (Live &l : ending) {
            Job *j = l.job;
            uq_status st = j->enter();
            if (st == UQ_OK) st = j->advance(l.r.steps - j->t);
            if (st != UQ_OK) return die(uq_last_error());
        }
        uq_status st = (!live.empty() && K > 0) ? tick(K) : UQ_OK;
        if (st != UQ_OK) return die(uq_last_error());
        for (Live &l : ending) finish(l);
        const double te = now();
        {
            std::lock_guard<std::mutex> lk(mu);
            busy_s += te - tb;
        }
        if (plain && live.front().job->t >= live.front().r.steps) {
            finish(live.front());
            std::lock_guard<std::mutex> lk(mu);
            live.clear();
        }
    }
}

}  // namespace uqi

using namespace uqi;

struct uq_server : public uqi::Server {};

extern "C" uq_status uq_server_create(const uq_server_config *cfg, const uq_device *dev, uq_server **out) {
    if (!cfg || !out) return fail(UQ_EINVAL, "null argument");
    *out = nullptr;
    if (cfg->memory_budget <= 0 || cfg->max_jobs < 1 || cfg->max_jobs > 4096 || cfg->steps_per_tick < 2 ||
        (cfg->mode != UQ_SERVE_BATCHED && cfg->mode != UQ_SERVE_PLAIN) || cfg->precision < UQ_FP64 ||
        cfg->precision > UQ_BF16S)
        return fail(UQ_EINVAL, "invalid server configuration");
    if (dev && ((dev->alloc == nullptr) != (dev->free == nullptr)))
        return fail(UQ_EINVAL, "uq_device needs both alloc and free, or neither");
    std::unique_ptr<uq_server> s(new uq_server());
    s->cfg = *cfg;
    s->cfg.steps_per_tick &= ~1;
    if (dev) s->dev = *dev;
    s->device = s->dev.device;
    UQ_HIP_TRY(hipSetDevice(s->device));
    UQ_HIP_TRY(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
    UQ_HIP_TRY(hipEventCreateWithFlags(&s->ev, hipEventDisableTiming));
    uq_status st = s->arena.init((size_t)cfg->memory_budget, s->dev);
    if (st != UQ_OK) return st;
    // the arena (from the caller's allocator on the caller's stream) is
    // ready for the loop once the caller's stream has reached this point
    UQ_HIP_TRY(hipEventRecord(s->ev, (hipStream_t)s->dev.stream));
    UQ_HIP_TRY(hipStreamWaitEvent(s->stream, s->ev, 0));
    s->table_cap = cfg->max_jobs;
    const size_t tb = up256(sizeof(MultiJob) * s->table_cap) + up256(sizeof(FusedJob) * s->table_cap) +
                      up256(sizeof(int64_t *) * s->table_cap);
    s->d_tables = s->arena.alloc(tb);
    if (!s->d_tables) return fail(UQ_ENOMEM, "server memory budget too small for its job tables");
    char *t = (char *)s->d_tables;
    s->d_table = (MultiJob *)t;
    s->d_fused = (FusedJob *)(t + up256(sizeof(MultiJob) * s->table_cap));
    s->d_tptrs = (int64_t **)(t + up256(sizeof(MultiJob) * s->table_cap) + up256(sizeof(FusedJob) * s->table_cap));
    s->t0 = std::chrono::steady_clock::now();
    uq_server *raw = s.get();
    s->th = std::thread([raw] { raw->loop(); });
    *out = s.release();
    return UQ_OK;
}

extern "C" uq_status uq_server_submit(uq_server *s, const uq_problem *p, int64_t steps, int32_t qoi,
                                      uint64_t *ticket) {
    if (!s || !p || !ticket) return fail(UQ_EINVAL, "null argument");
    if (steps < 0) return fail(UQ_EINVAL, "steps must be >= 0");
    if (qoi != UQ_QOI_KE && qoi != UQ_QOI_CD && qoi != UQ_QOI_CL)
        return fail(UQ_EINVAL, "the server returns scalar QoIs (KE, CD, CL)");
    if ((qoi == UQ_QOI_CD || qoi == UQ_QOI_CL) &&
        (p->geometry != UQ_GEOM_CHANNEL || (p->D <= 0 && p->cyl_bc != UQ_CYL_BOUZIDI)))
        return fail(UQ_EINVAL, "drag/lift need a channel with a cylinder");
    if (p->precision != s->cfg.precision) return fail(UQ_EINVAL, "job precision differs from the server's");
    if (needs_ab(*p))
        return fail(UQ_EINVAL, "the server's kernels take node-local boundary rules; interpolated boundaries need a job of their own");
    Rule r;
    uq_status st = build_rule(*p, r);
    if (st != UQ_OK) return st;
    Request q;
    q.p = *p;
    q.steps = steps;
    q.qoi = qoi;
    q.S = r.S;
    q.K = r.K;
    if (s->cfg.mode == UQ_SERVE_BATCHED) q.shape = serve_shape(*p, r.S, r.K, s->arena.capacity());
    q.footprint = job_footprint(*p, r.S, r.K, q.shape.kind >= 0);
    if ((size_t)q.footprint > s->arena.capacity())
        return fail(UQ_ENOMEM, "job needs " + std::to_string(q.footprint) + " B, more than the server's memory budget");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(UQ_ESTATE, s->fatal.empty() ? "server is stopping" : s->fatal);
    q.ticket = s->next_ticket++;
    q.t_submit = s->now();
    s->pending.push_back(q);
    ++s->submitted;
    *ticket = q.ticket;
    s->cv_work.notify_one();
    return UQ_OK;
}

static uq_status take_result(uq_server *s, uint64_t ticket, uq_result *out) {
    auto it = s->done.find(ticket);
    if (it == s->done.end()) return UQ_EAGAIN;
    *out = it->second;
    s->done.erase(it);
    return UQ_OK;
}

extern "C" uq_status uq_server_poll(uq_server *s, uint64_t ticket, uq_result *out) {
    if (!s || !out) return fail(UQ_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    if (ticket == 0 || ticket >= s->next_ticket) return fail(UQ_EINVAL, "unknown ticket");
    uq_status st = take_result(s, ticket, out);
    if (st == UQ_EAGAIN && s->stop && !s->fatal.empty()) return fail(UQ_EDEVICE, s->fatal);
    return st;
}

extern "C" uq_status uq_server_wait(uq_server *s, uint64_t ticket, double timeout_s, uq_result *out) {
    if (!s || !out) return fail(UQ_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    if (ticket == 0 || ticket >= s->next_ticket) return fail(UQ_EINVAL, "unknown ticket");
    auto ready = [&] { return s->done.count(ticket) || (s->stop && !s->fatal.empty()); };
    if (timeout_s < 0)
        s->cv_done.wait(lk, ready);
    else
        s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
    uq_status st = take_result(s, ticket, out);
    if (st == UQ_EAGAIN && !s->fatal.empty()) return fail(UQ_EDEVICE, s->fatal);
    return st;
}

extern "C" uq_status uq_server_get_stats(uq_server *s, uq_server_stats *o) {
    if (!s || !o) return fail(UQ_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(o, 0, sizeof *o);
    o->submitted = s->submitted;
    o->completed = s->completed;
    o->failed = s->failed;
    o->pending = (int64_t)s->pending.size();
    o->live = (int64_t)s->live.size();
    o->elapsed_s = s->now();
    o->busy_s = s->busy_s;
    o->node_updates = s->node_updates;
    o->solves_per_hour = o->elapsed_s > 0 ? 3600.0 * (double)s->completed / o->elapsed_s : 0.0;
    o->mlups = o->elapsed_s > 0 ? s->node_updates / o->elapsed_s / 1e6 : 0.0;
    if (!s->latencies.empty()) {
        std::vector<double> v = s->latencies;
        std::sort(v.begin(), v.end());
        auto rank = [&](double q) {
            size_t i = (size_t)std::ceil(q * (double)v.size());
            return v[std::min(v.size(), std::max<size_t>(i, 1)) - 1];
        };
        o->latency_p50_s = rank(0.50);
        o->latency_p99_s = rank(0.99);
        double sum = 0.0;
        for (double x : v) sum += x;
        o->latency_mean_s = sum / (double)v.size();
    }
    o->arena_bytes = (int64_t)s->arena.capacity();
    o->arena_peak_bytes = (int64_t)s->arena.peak();
    return UQ_OK;
}

extern "C" void uq_server_destroy(uq_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->pending.clear();
        s->cv_work.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    (void)hipSetDevice(s->device);
    for (Live &l : s->live)
        if (l.job) delete l.job;
    s->live.clear();
    s->release_graph();
    if (s->stream) {
        // the caller's stream waits for the loop's work before the arena
        // goes back to the caller's allocator
        (void)hipStreamSynchronize(s->stream);
        if (s->ev && hipEventRecord(s->ev, s->stream) == hipSuccess)
            (void)hipStreamWaitEvent((hipStream_t)s->dev.stream, s->ev, 0);
    }
    if (s->d_tables) s->arena.release(s->d_tables);
    if (s->ev) (void)hipEventDestroy(s->ev);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;  // the arena's memory goes back
}
