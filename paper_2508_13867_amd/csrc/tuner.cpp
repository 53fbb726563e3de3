// Launch-shape autotuner of the step kernel: times every candidate
// (layout AA / AB, rows per thread, non-temporal AB stores, plane padding) on
// the device with the problem's real lattice and sample count, and keeps the
// fastest per problem class for later jobs of this process. An optional
// cache file (UQ_TUNE_CACHE) carries results across processes.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "uq_job.h"

namespace uqi {

namespace {

// problem class: precision, geometry, lattice, samples, requested layout
// (interpolated-boundary problems count as a layout request of their own)
using Key = std::tuple<int, int, int, int, int64_t, int>;

struct Entry {
    StepShape shape;
    double gbs = 0.0;
};

std::mutex g_mu;
std::map<Key, Entry> g_cache;
bool g_loaded = false;

Key key_of(const uq_problem &p, int64_t S) {
    return Key(p.precision, p.geometry, p.nx, p.ny, S, needs_ab(p) ? 16 + p.layout : p.layout);
}

const char *cache_path() {
    const char *v = std::getenv("UQ_TUNE_CACHE");
    return (v && *v) ? v : nullptr;
}

void load_cache_locked() {
    if (g_loaded) return;
    g_loaded = true;
    const char *path = cache_path();
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    int prec, geom, nx, ny, lay_req, layout, cpt, nt, pad, bx, fuse, fty, fwin;
    long long S;
    double gbs;
    while (std::fscanf(f, "%d %d %d %d %lld %d %d %d %d %d %d %d %d %d %lf", &prec, &geom, &nx, &ny, &S, &lay_req,
                       &layout, &cpt, &nt, &pad, &bx, &fuse, &fty, &fwin, &gbs) == 15) {
        Entry e;
        e.shape.layout = layout;
        e.shape.cpt = cpt;
        e.shape.nt = nt;
        e.shape.pad = pad;
        e.shape.bx = bx;
        e.shape.fuse = fuse;
        e.shape.fty = fty;
        e.shape.fwin = fwin;
        e.gbs = gbs;
        g_cache[Key(prec, geom, nx, ny, (int64_t)S, lay_req)] = e;
    }
    std::fclose(f);
}

void store_locked(const Key &k, const Entry &e) {
    g_cache[k] = e;
    const char *path = cache_path();
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%d %d %d %d %lld %d %d %d %d %d %d %d %d %d %.3f\n", std::get<0>(k), std::get<1>(k),
                 std::get<2>(k), std::get<3>(k), (long long)std::get<4>(k), std::get<5>(k), e.shape.layout, e.shape.cpt,
                 e.shape.nt, e.shape.pad, e.shape.bx, e.shape.fuse, e.shape.fty, e.shape.fwin, e.gbs);
    std::fclose(f);
}

}  // namespace

bool tuned_shape(const uq_problem &p, int64_t S, StepShape *out) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache_locked();
    auto it = g_cache.find(key_of(p, S));
    if (it == g_cache.end()) return false;
    *out = it->second.shape;
    return true;
}

}  // namespace uqi

using namespace uqi;

extern "C" uq_status uq_autotune(const uq_problem *p, const uq_device *dev, int64_t steps, uq_tune_result *out) {
    if (!p || !out) return fail(UQ_EINVAL, "null argument");
    if (steps < 2) return fail(UQ_EINVAL, "steps must be >= 2");
    if (steps < 120) steps = 120;
    Rule r;
    uq_status st = build_rule(*p, r);
    if (st != UQ_OK) return st;

    std::vector<StepShape> cands;
    for (int layout : {UQ_LAYOUT_AA, UQ_LAYOUT_AB}) {
        if (p->layout != UQ_LAYOUT_AUTO && p->layout != layout) continue;
        if (needs_ab(*p) && layout != UQ_LAYOUT_AB) continue;
        for (int bx : {64, 128, 256})
            for (int cpt : {1, 2})
                for (int pad : {0, 64})
                    for (int nt : {0, 1}) {
                        if (layout == UQ_LAYOUT_AA && nt) continue;  // AA stores are in place
                        if (bx > 64 && bx / 2 >= p->nx) continue;      // mostly idle lanes
                        StepShape s;
                        s.layout = layout;
                        s.cpt = cpt;
                        s.pad = pad;
                        s.nt = nt;
                        s.bx = bx;
                        cands.push_back(s);
                    }
        // channels with half-way and Zou-He / wall / periodic ends (AB): the
        // full-row window, 2 to 4 steps per launch, the height cut into 1 to 8
        // balanced chunks (a workgroup per chunk and sample: few samples
        // need several chunks to fill the chip)
        if (layout == UQ_LAYOUT_AB && p->geometry == UQ_GEOM_CHANNEL && p->cyl_bc == UQ_CYL_HALFWAY &&
            p->xbc != UQ_XBC_INTERP) {
            std::vector<int> heights;
            for (int nch : {1, 2, 3, 4, 6, 8}) {
                const int h = (p->ny + nch - 1) / nch;
                if (h >= 8 && (heights.empty() || heights.back() != h)) heights.push_back(h);
            }
            for (int n : {2, 3, 4})
                for (int fty : heights) {
                    if (p->nx > channel_rows_max_nx(p->precision, n)) continue;
                    StepShape s;
                    s.layout = layout;
                    s.pad = 64;
                    s.nt = 0;
                    s.fuse = n;
                    s.fty = fty;
                    s.fwin = 2;
                    cands.push_back(s);
                }
        }
        // 2, 3 or 4 steps per launch (periodic lattices, AB): tiles of 64 x fty
        // nodes, and sliding windows down chunks of fty rows
        if (layout == UQ_LAYOUT_AB && p->geometry == UQ_GEOM_TGV) {
            for (int n : {2, 3, 4})
                for (int pad : {0, 64})
                    for (int fty : (p->precision == UQ_FP64 ? std::vector<int>{4, 8} : std::vector<int>{8, 16})) {
                        StepShape s;
                        s.layout = layout;
                        s.pad = pad;
                        s.nt = 1;
                        s.fuse = n;
                        s.fty = fty;
                        cands.push_back(s);
                    }
            for (int win : {1, 2})
                for (int n : {2, 3, 4, 5, 6, 7, 8})
                    for (int fty : (p->precision == UQ_FP64 ? std::vector<int>{32, 64} : std::vector<int>{64, 256})) {
                        if (win == 1 && n > 4) continue;  // strips: up to 4 steps
                        if (win == 2 && (n < 3 || p->nx > full_rows_max_nx(p->precision, n))) continue;
                        StepShape s;
                        s.layout = layout;
                        s.pad = 64;
                        s.nt = 0;
                        s.fuse = n;
                        s.fty = fty;
                        s.fwin = win;
                        cands.push_back(s);
                    }
        }
    }

    const double bytes_per_node = 18.0 * (double)storage_bytes(p->precision);
    Entry best;
    int tried = 0;
    double best_ms = 0.0;
    for (const StepShape &cand : cands) {
        uq_job *j = nullptr;
        st = create_job(*p, dev, &cand, &j);
        if (st == UQ_ENOMEM) continue;  // e.g. no room for the second AB slab
        if (st != UQ_OK) return st;
        j->use_graph = false;
        double ms = 0.0;
        hipEvent_t a = nullptr, b = nullptr;
        bool ok = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess;
        // each candidate times whole launch blocks (N steps, 2N for even N)
        const int64_t block = cand.fuse >= 2 ? ((cand.fuse & 1) ? cand.fuse : 2 * cand.fuse) : 1;
        const int64_t csteps = std::max(block, steps / block * block);
        ok = ok && j->advance(2 * block) == UQ_OK;  // warm-up
        ok = ok && hipEventRecord(a, j->stream) == hipSuccess;
        ok = ok && j->advance(csteps) == UQ_OK;
        ok = ok && hipEventRecord(b, j->stream) == hipSuccess;
        ok = ok && hipEventSynchronize(b) == hipSuccess;
        float f = 0.0f;
        ok = ok && hipEventElapsedTime(&f, a, b) == hipSuccess;
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        (void)hipSetDevice(j->dev.device);
        delete j;
        if (!ok) return fail(UQ_EDEVICE, "timing a tuning candidate failed");
        ms = (double)f / (double)csteps;
        ++tried;
        const double gbs = (double)r.S * p->nx * p->ny * bytes_per_node / (ms * 1e-3) / 1e9;
        if (tried == 1 || gbs > best.gbs) {
            best.shape = cand;
            best.gbs = gbs;
            best_ms = ms;
        }
    }
    if (tried == 0) return fail(UQ_ENOMEM, "no tuning candidate fits in device memory");
    {
        std::lock_guard<std::mutex> lk(g_mu);
        load_cache_locked();
        store_locked(key_of(*p, r.S), best);
    }
    out->layout = best.shape.layout;
    out->cpt = best.shape.cpt;
    out->nt_store = best.shape.nt;
    out->plane_pad = best.shape.pad;
    out->bx = best.shape.bx;
    out->fused = best.shape.fuse >= 2 ? best.shape.fuse : 0;
    out->fused_rows = best.shape.fuse >= 2 ? best.shape.fty : 0;
    out->fused_window = best.shape.fuse >= 2 ? best.shape.fwin : 0;
    out->gbs = best.gbs;
    out->ms_per_step = best_ms;
    out->n_candidates = tried;
    return UQ_OK;
}
