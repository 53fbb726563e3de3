// Time stepping of one job: eager launches or replays of a captured
// hipGraph of an even number of steps (the AA parity pattern inside the graph
// is then fixed, and the step count lives in device memory so the same graph
// serves every replay).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <string>

#include "uq_job.h"

namespace uqi {

static int env_int(const char *name, int dflt) {
    const char *v = std::getenv(name);
    if (!v || !*v) return dflt;
    return std::atoi(v);
}

// Launch shape and layout of a job. Order of precedence: a shape measured by
// uq_autotune for this problem class (when the problem leaves the layout to
// AUTO, or fixes the same layout), then the UQ_* environment overrides, then
// the defaults (AA, one row per thread, 64 elements of plane padding).
StepShape choose_shape(const uq_problem &p, int64_t S) {
    StepShape s;
    if (tuned_shape(p, S, &s)) {
        if (needs_ab(p)) s.layout = UQ_LAYOUT_AB;
        return s;
    }
    s.cpt = env_int("UQ_CPT", 1);
    s.persistent = env_int("UQ_PERSISTENT", 0);
    s.nt = env_int("UQ_NT_STORE", 1);
    s.pad = env_int("UQ_PLANE_PAD", 64);
    s.bx = env_int("UQ_BX", 64);
    s.fuse = env_int("UQ_FUSE", 0);
    s.fty = env_int("UQ_FUSE_TY", 8);
    s.fwin = env_int("UQ_FUSE_WINDOW", 0);
    if (s.fwin == 2 && p.nx > full_rows_max_nx(p.precision, s.fuse)) s.fwin = 1;  // rows too wide
    s.layout = UQ_LAYOUT_AA;
    if (p.layout == UQ_LAYOUT_AA || p.layout == UQ_LAYOUT_AB) {
        s.layout = p.layout;
    } else {
        const char *v = std::getenv("UQ_LAYOUT");
        if (v && (v[0] == 'a' || v[0] == 'A') && (v[1] == 'b' || v[1] == 'B')) s.layout = UQ_LAYOUT_AB;
    }
    if (needs_ab(p)) s.layout = UQ_LAYOUT_AB;
    return s;
}

// The job's own stream is non-blocking, so it is ordered against the
// caller's stream explicitly, also when that is the null stream.
uq_status Job::enter() {
    if (user_stream != stream) {
        UQ_HIP_TRY(hipEventRecord(ev_in, user_stream));
        UQ_HIP_TRY(hipStreamWaitEvent(stream, ev_in, 0));
    }
    return UQ_OK;
}

uq_status Job::leave() {
    if (user_stream != stream) {
        UQ_HIP_TRY(hipEventRecord(ev_out, stream));
        UQ_HIP_TRY(hipStreamWaitEvent(user_stream, ev_out, 0));
    }
    return UQ_OK;
}

void Job::release_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    graph_len = 0;
}

// steps per fused launch in effect (0: none)
int Job::fused_n() const {
    if (shape.fuse < 2) return 0;
    if (jd.geom == 1)  // channel: whole rows, up to 4 steps, where the LDS rows fit
        return (shape.fwin == 2 && shape.fuse <= 4 && channel_fusable(jd) &&
                jd.nx <= channel_rows_max_nx(jd.prec, shape.fuse))
                   ? shape.fuse
                   : 0;
    const int nmax = shape.fwin == 2 ? 8 : 4;  // whole rows: up to 8 steps
    return (shape.fuse <= nmax && fused_supported(jd)) ? shape.fuse : 0;
}

// Launches for `n` steps starting at step t + k0 of the host mirror. The
// state of step u lives in slab u & 1. A launch of N fused steps reads the
// current slab and writes the other one: for odd N that is the slab of step
// u + N; even N go in pairs (there and back), so that the invariant holds
// after each pair. Steps left over go in single fused launches of an odd
// number (3 or more, at most N) of steps, largest first, then one per launch.
hipError_t Job::enqueue_steps(int k0, int64_t n) {
    hipError_t e = hipSuccess;
    int64_t &enqueued = pending_launches;
    int64_t k = 0;
    const int N = fused_n();
    if (N) {
        const int64_t block = (N & 1) ? N : 2 * N;
        for (; k + block <= n && e == hipSuccess; k += block) {
            const bool odd = ((t + k0 + k) & 1) != 0;
            e = launch_fused(jd, N, odd, shape.fty, shape.fwin, shape.nt != 0, d_t, (int)(k0 + k), stream);
            ++enqueued;
            if (e == hipSuccess && !(N & 1)) {
                e = launch_fused(jd, N, !odd, shape.fty, shape.fwin, shape.nt != 0, d_t, (int)(k0 + k + N), stream);
                ++enqueued;
            }
        }
        // fewer steps than a block: a shape that runs N steps runs fewer
        for (int64_t r = n - k; r >= 3 && e == hipSuccess; r = n - k) {
            int m = (int)std::min<int64_t>(r, N);
            if (!(m & 1)) --m;
            if (m < 3) break;
            const bool odd = ((t + k0 + k) & 1) != 0;
            e = launch_fused(jd, m, odd, shape.fty, shape.fwin, shape.nt != 0, d_t, (int)(k0 + k), stream);
            ++enqueued;
            k += m;
        }
    }
    for (; k < n && e == hipSuccess; ++k) {
        e = launch_step(jd, d_t, (int)(k0 + k), (int)((t + k0 + k) & 1), shape, stream, &side);
        ++enqueued;
    }
    return e;
}

uq_status Job::advance(int64_t steps) {
    int L = env_int("UQ_GRAPH_STEPS", 64) & ~1;
    // whole fused blocks in a graph: multiples of 2N (N even) or 2N (N odd,
    // even length keeps every replay starting at an even step)
    if (const int N = fused_n()) L = L / (2 * N) * (2 * N);
    if (use_graph && L >= 2 && steps >= L + 1) {
        if (t & 1) {
            UQ_HIP_TRY(launch_step(jd, d_t, 0, 1, shape, stream, &side));
            ++launches;
            UQ_HIP_TRY(launch_advance(d_t, 1, stream));
            t += 1;
            steps -= 1;
        }
        if (!gexec || graph_len != L) {
            release_graph();
            UQ_HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
            pending_launches = 0;
            hipError_t e = enqueue_steps(0, L);
            graph_launches = pending_launches;
            pending_launches = 0;
            if (e == hipSuccess) e = launch_advance(d_t, L, stream);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(stream, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return fail(UQ_EDEVICE, std::string("graph capture failed: ") +
                                            hipGetErrorString(e != hipSuccess ? e : e2));
            }
            graph = g;
            UQ_HIP_TRY(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
            graph_len = L;
        }
        while (steps >= L) {
            UQ_HIP_TRY(hipGraphLaunch(gexec, stream));
            t += L;
            steps -= L;
            launches += graph_launches;
        }
    }
    if (steps > 0) {
        pending_launches = 0;
        UQ_HIP_TRY(enqueue_steps(0, steps));
        launches += pending_launches;
        UQ_HIP_TRY(launch_advance(d_t, steps, stream));
        t += steps;
    }
    return UQ_OK;
}

Job::~Job() {
    if (stream) (void)hipStreamSynchronize(stream);
    release_graph();
    dfree_all();
    if (side.stream) (void)hipStreamSynchronize(side.stream);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (side.fork) (void)hipEventDestroy(side.fork);
    if (side.join) (void)hipEventDestroy(side.join);
    if (side.stream) (void)hipStreamDestroy(side.stream);
    if (stream) (void)hipStreamDestroy(stream);
}

}  // namespace uqi
