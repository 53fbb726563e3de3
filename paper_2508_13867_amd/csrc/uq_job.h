// A UQ job: problem, sample set, device buffers and time-stepping state.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "uq_internal.h"

namespace uqi {

int64_t storage_bytes(int prec);
int64_t row_pitch(int nx);
void build_mask(const uq_problem &p, int64_t pitch, std::vector<uint32_t> &mask, std::vector<double> &q,
                std::vector<int32_t> &special, int &fluid);
StepShape choose_shape(const uq_problem &p, int64_t S);
// tuned shape for a problem class, if one was measured in this process
bool tuned_shape(const uq_problem &p, int64_t S, StepShape *out);

// Device buffers of one statistics evaluation (uq_qoi_samples, uq_moments
// and its allocation-free variant): per-sample scalar QoIs qoi[S][4], the
// selected scalar M[S], per-sample fields fields[S][4][ny][nx] (per-sample
// field values only; the moments of a field are formed from the populations
// without them), the outputs out[(K + 3) n_out] and one int64 flag.
struct StatBufs {
    double *qoi = nullptr, *M = nullptr, *fields = nullptr, *out = nullptr;
    int64_t *flag = nullptr;
};

// values per sample of a QoI (1, nx ny or 2 nx ny); 0 for an unknown QoI
int64_t qoi_width(const uq_problem &p, int qoi);

struct Job {
    uq_problem p{};
    uq_device dev{};
    Rule rule;
    int64_t S = 0;
    int K = 0;
    int64_t pitch = 0;
    int scale_exp = 0;
    int fluid = 0;
    int plane_pad = 0;

    hipStream_t user_stream = nullptr;  // caller's stream (ordering only)
    hipStream_t stream = nullptr;       // the job's own work stream
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    SideStream side;                    // boundary-node kernels (AB channel jobs)

    JobDev jd{};
    StepShape shape{};
    int64_t t = 0;            // steps done (host mirror)
    int64_t launches = 0;     // step-kernel launches issued (graph replays counted per launch)
    int64_t graph_launches = 0; // step-kernel launches in the captured graph
    int64_t pending_launches = 0; // counted by enqueue_steps
    int64_t *d_t = nullptr;   // steps done at the last base update (device)

    std::vector<void *> allocs;
    int64_t bytes_held = 0;
    double *d_qoi = nullptr, *d_M = nullptr, *d_out = nullptr, *d_fields = nullptr;
    double *d_wphi = nullptr, *d_a = nullptr, *d_export = nullptr;
    int64_t *d_flag = nullptr;
    int64_t out_cap = 0;

    // hipGraph of `graph_len` steps starting at an even step
    bool use_graph = true;
    int graph_len = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;

    ~Job();
    void *dalloc(size_t bytes);
    void dfree(void *p);  // release one block from dalloc
    void dfree_all();
    uq_status ensure_stats_buffers(int64_t n_out_max);
    uq_status ensure_fields();
    // the job's own statistics buffers for `qoi` (with the per-sample field
    // buffer if `fields`), allocated on first use
    uq_status own_stat_bufs(int qoi, bool fields, StatBufs *b);
    uq_status check_finite(const StatBufs &b);
    // per-sample values of `qoi` in b (M: value o of sample s at M[s*ld + o])
    uq_status sample_values_in(const StatBufs &b, int qoi, const double **M, int64_t *n_out, int64_t *ld);
    uq_status sample_values(int qoi, const double **M, int64_t *n_out, int64_t *ld);
    // statistics of `qoi` computed in b and copied to out (blocking)
    uq_status moments_in(const StatBufs &b, int qoi, uq_moments_out *out);
    uq_status advance(int64_t steps);
    hipError_t enqueue_steps(int k0, int64_t n);
    int fused_n() const;
    uq_status enter();  // order the job stream after the caller's stream
    uq_status leave();  // order the caller's stream after the job stream
    void release_graph();
};

}  // namespace uqi

struct uq_job : public uqi::Job {};

namespace uqi {
// Build a job; `forced` (may be null) fixes layout and launch shape.
uq_status create_job(const uq_problem &p, const uq_device *dev, const StepShape *forced, uq_job **out);
}  // namespace uqi
