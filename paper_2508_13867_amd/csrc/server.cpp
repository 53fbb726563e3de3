// Continuous-batching UQ server: a request loop on its own host thread that
// admits jobs of different lattices and sample counts by device-memory
// footprint, keeps their populations resident, and advances every sample of
// every live job in one fused launch per step (the non-intrusive UQ algorithm
// of OpenLB-UQ, Algorithm alg:uq_openlb, with the per-sample solve loop of
// all concurrent requests batched). A "plain" mode runs the same kernels one
// job at a time and one sample per launch, for comparison.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "uq_job.h"

namespace uqi {

// ------------------------------------------------------------------ arena
// One device allocation made at server start, carved first-fit into 256-byte
// aligned blocks; freed blocks coalesce with their neighbours. Serving never
// calls hipMalloc or hipFree (hipFree would synchronise the device).
class Arena {
   public:
    uq_status init(size_t bytes) {
        cap_ = (bytes + 255) / 256 * 256;
        if (hipMalloc(&base_, cap_) != hipSuccess) {
            (void)hipGetLastError();
            base_ = nullptr;
            return fail(UQ_ENOMEM, "server arena of " + std::to_string(cap_) + " B does not fit on the device");
        }
        free_[0] = cap_;
        return UQ_OK;
    }
    ~Arena() {
        if (base_) (void)hipFree(base_);
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
    size_t cap_ = 0, in_use_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_, used_;
    std::mutex mu_;
};

static void *arena_alloc_cb(size_t n, void *ctx) { return ((Arena *)ctx)->alloc(n); }
static void arena_free_cb(void *p, void *ctx) { ((Arena *)ctx)->release(p); }

static size_t up256(size_t n) { return (n + 255) / 256 * 256; }

// Device bytes a job takes in the server (AA layout, scalar moments): slab,
// per-sample records, step counter, boundary mask, basis table, QoI buffers
// and the non-finite flag.
int64_t job_footprint(const uq_problem &p, int64_t S, int K) {
    const int64_t pitch = row_pitch(p.nx);
    const int64_t plane = (int64_t)p.ny * pitch + 64;
    size_t b = up256((size_t)(S * 9 * plane * storage_bytes(p.precision)));
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
    int64_t footprint = 0;
    double t_submit = 0.0;
};

struct Live {
    Request r;
    uq_job *job = nullptr;
    double t_admit = 0.0;
    int tiles_x = 0, tiles_y = 0;
};

struct Server {
    uq_server_config cfg{};
    int device = 0;
    Arena arena;
    hipStream_t stream = nullptr;
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

    // continuous-batching table
    MultiJob *d_table = nullptr;
    int table_cap = 0;
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
        sh.layout = UQ_LAYOUT_AA;
        sh.cpt = 1;
        sh.pad = 64;
        sh.nt = 0;
        uq_job *j = nullptr;
        uq_status st = create_job(r.p, &dv, &sh, &j);
        if (st == UQ_ENOMEM) {  // fragmentation: retry when memory frees up
            std::lock_guard<std::mutex> lk(mu);
            pending.push_front(r);
            continue;
        }
        if (st == UQ_OK && hipStreamSynchronize(j->stream) != hipSuccess) st = UQ_EDEVICE;
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

uq_status Server::rebuild_table() {
    std::vector<MultiJob> h(live.size());
    int64_t tile = 0;
    for (size_t q = 0; q < live.size(); ++q) {
        Live &l = live[q];
        MultiJob &m = h[q];
        std::memset(&m, 0, sizeof m);
        m.j = l.job->jd;
        m.t = l.job->t;
        m.n_steps = l.r.steps;
        m.tile0 = tile;
        m.tiles_x = l.tiles_x;
        m.tiles_y = l.tiles_y;
        tile += (int64_t)l.job->S * l.tiles_x * l.tiles_y;
    }
    total_tiles = tile;
    if ((int)h.size() > table_cap) return fail(UQ_ESTATE, "more live jobs than the table holds");
    if (!h.empty()) {
        UQ_HIP_TRY(hipMemcpyAsync(d_table, h.data(), sizeof(MultiJob) * h.size(), hipMemcpyHostToDevice, stream));
        UQ_HIP_TRY(hipStreamSynchronize(stream));
    }
    release_graph();
    dirty = false;
    return UQ_OK;
}

// Advance every live job by K steps (jobs that reach their target stop).
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
    const int nj = (int)live.size();
    const int prec = cfg.precision;
    const bool graph_tick = cfg.use_graph && K == cfg.steps_per_tick;
    if (graph_tick && !gexec) {
        UQ_HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int k = 0; k < K && e == hipSuccess; ++k) e = launch_step_multi(d_table, nj, total_tiles, k, prec, stream);
        if (e == hipSuccess) e = launch_advance_multi(d_table, nj, K, stream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(UQ_EDEVICE, "server graph capture failed");
        }
        graph = g;
        UQ_HIP_TRY(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
    }
    if (graph_tick) {
        UQ_HIP_TRY(hipGraphLaunch(gexec, stream));
    } else {
        for (int k = 0; k < K; ++k) UQ_HIP_TRY(launch_step_multi(d_table, nj, total_tiles, k, prec, stream));
        UQ_HIP_TRY(launch_advance_multi(d_table, nj, K, stream));
    }
    UQ_HIP_TRY(hipStreamSynchronize(stream));
    for (Live &l : live) l.job->t = std::min<int64_t>(l.job->t + K, l.r.steps);
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
        hipError_t e = j->K > 0 ? launch_moments_sc(M, j->S, 1, 1, j->d_wphi, j->d_a, j->K, dc, dm, dv, da, j->stream)
                                : launch_moments_mc(M, j->S, 1, 1, dm, dv, da, j->stream);
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
        if (cfg.mode != UQ_SERVE_PLAIN && dirty) {
            uq_status st = rebuild_table();
            if (st != UQ_OK) {
                std::lock_guard<std::mutex> lk(mu);
                fatal = uq_last_error();
                stop = true;
                cv_done.notify_all();
                return;
            }
        }
        int64_t K = cfg.steps_per_tick;
        for (Live &l : live) K = std::min<int64_t>(K, l.r.steps - l.job->t);
        if (cfg.mode != UQ_SERVE_PLAIN && K < cfg.steps_per_tick && K > 0 && cfg.use_graph) {
            // a job ends inside this tick: run the full graph anyway if most
            // jobs have further to go; the finished job's tiles are skipped
            int64_t Kmax = 0;
            for (Live &l : live) Kmax = std::max<int64_t>(Kmax, l.r.steps - l.job->t);
            if (Kmax >= cfg.steps_per_tick) K = cfg.steps_per_tick;
        }
        const double tb = now();
        uq_status st = K > 0 ? tick(K) : UQ_OK;
        const double te = now();
        if (st != UQ_OK) {
            std::lock_guard<std::mutex> lk(mu);
            fatal = uq_last_error();
            stop = true;
            cv_done.notify_all();
            return;
        }
        {
            std::lock_guard<std::mutex> lk(mu);
            busy_s += te - tb;
        }
        std::vector<Live> keep;
        for (Live &l : live) {
            if (l.job->t >= l.r.steps) {
                finish(l);
                std::lock_guard<std::mutex> lk(mu);
                dirty = true;
            } else {
                keep.push_back(l);
            }
        }
        std::lock_guard<std::mutex> lk(mu);
        live.swap(keep);
    }
}

}  // namespace uqi

using namespace uqi;

struct uq_server : public uqi::Server {};

extern "C" uq_status uq_server_create(const uq_server_config *cfg, int32_t device, uq_server **out) {
    if (!cfg || !out) return fail(UQ_EINVAL, "null argument");
    *out = nullptr;
    if (cfg->memory_budget <= 0 || cfg->max_jobs < 1 || cfg->max_jobs > 4096 || cfg->steps_per_tick < 2 ||
        (cfg->mode != UQ_SERVE_BATCHED && cfg->mode != UQ_SERVE_PLAIN) || cfg->precision < UQ_FP64 ||
        cfg->precision > UQ_BF16S)
        return fail(UQ_EINVAL, "invalid server configuration");
    std::unique_ptr<uq_server> s(new uq_server());
    s->cfg = *cfg;
    s->cfg.steps_per_tick &= ~1;
    s->device = device;
    UQ_HIP_TRY(hipSetDevice(device));
    uq_status st = s->arena.init((size_t)cfg->memory_budget);
    if (st != UQ_OK) return st;
    UQ_HIP_TRY(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
    s->table_cap = cfg->max_jobs;
    UQ_HIP_TRY(hipMalloc(&s->d_table, sizeof(MultiJob) * s->table_cap));
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
        return fail(UQ_EINVAL, "the server runs the in-place AA layout; interpolated boundaries need a job of their own");
    Rule r;
    uq_status st = build_rule(*p, r);
    if (st != UQ_OK) return st;
    Request q;
    q.p = *p;
    q.steps = steps;
    q.qoi = qoi;
    q.S = r.S;
    q.K = r.K;
    q.footprint = job_footprint(*p, r.S, r.K);
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
    if (s->d_table) (void)hipFree(s->d_table);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}
