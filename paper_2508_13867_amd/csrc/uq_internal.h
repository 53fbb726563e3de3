// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/uq.h"

namespace uqi {

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);
uq_status fail(uq_status st, const std::string &msg);

#define UQ_HIP_TRY(expr)                                                                          \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return ::uqi::fail(UQ_EDEVICE, std::string(#expr " failed: ") + hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------ host sampler
struct Rule {
    int64_t S = 0;
    int d = 0;
    int K = 0;                  // 0 for Monte Carlo
    std::vector<double> xi;     // [S][d]
    std::vector<double> a;      // [S]
    std::vector<int32_t> alpha; // [K][d]
    std::vector<double> phi;    // [S][K]
};

uq_status validate_problem(const uq_problem &p);
// interpolated boundaries (finite-difference inlet/outlet, interpolated
// cylinder) read neighbours' previous state: AB layout only
inline bool needs_ab(const uq_problem &p) {
    return p.geometry == UQ_GEOM_CHANNEL && (p.xbc == UQ_XBC_INTERP || p.cyl_bc == UQ_CYL_BOUZIDI);
}
uq_status build_rule(const uq_problem &p, Rule &r);

// Per-sample solver inputs after mapping the reference variables.
struct SampleInputs {
    double nu, u0, phase_x, phase_y, u_peak;  // u_peak: the channel's peak inflow
    double zeta[4];
};
void map_inputs(const uq_problem &p, const double *xi_row, SampleInputs &out);

// ------------------------------------------------------------------ device-side layout
// Per-sample parameters read by the kernels (one 128-byte record per sample).
struct alignas(64) SampleDev {
    double omega;   // 1/tau
    double u0;      // TGV amplitude
    double phase_x; // TGV phases
    double phase_y;
    double u_peak;  // channel peak inflow
    double zeta[4]; // harmonic perturbation amplitudes (UQ_INIT_TGV_HARMONIC)
    double pad[7];
};

// Per-node boundary mask of the channel (one 32-bit word per node).
//  bits 0..8   : the pull source x - c_i is a wall/solid -> bounce-back
//  bits 9..17  : the pull source x - c_i lies beyond an open column (Zou-He)
//  bit  18     : node is solid
//  bit  19     : node is on the inlet column, bit 20: outlet column
//  bits 21..29 : the link x -> x + c_i enters the cylinder (force links)
//  bit  30     : some bounce-back link of the node is interpolated (the link
//                fractions are in JobDev::q)
//  bit  31     : the node is stepped by a boundary-node kernel (interpolated
//                links, finite-difference open columns), not the bulk kernel
enum : uint32_t {
    M_BB = 0,
    M_OPEN = 9,
    M_SOLID = 1u << 18,
    M_INLET = 1u << 19,
    M_OUTLET = 1u << 20,
    M_CYL = 21,
    M_QLINK = 1u << 30,
    M_SPECIAL = 1u << 31,
};

// A job as the kernels see it.
struct JobDev {
    void *f;               // population slab [S][9][ny][pitch] (AB: state at even t)
    void *f2;              // AB: second slab (state at odd t); AA: null
    const SampleDev *smp;  // [S]
    const uint32_t *mask;  // [ny][pitch] or null (TGV)
    int64_t pitch;         // elements per row
    int64_t plane;         // ny * pitch
    int32_t nx, ny, S;
    int32_t geom;          // 0 TGV, 1 channel
    int32_t xbc;
    int32_t prec;
    float scale, inv_scale; // FP16S/BF16S storage scale
    double ramp;            // T_r (0: none)
    double ke_norm;         // 2/(nx ny u0^2)
    int32_t D;
    int32_t layout;         // UQ_LAYOUT_AA or UQ_LAYOUT_AB
    int32_t init;           // uq_init (vortex)
    int32_t pad1;
    const double *q;        // [9][ny][pitch] interpolated-link fraction of pull
                            // direction i (0: none); null without such links
    double dia;             // diameter in C_D, C_L
    double u_fac;           // their velocity: u_fac * u_peak of the sample
    const int32_t *special; // [n_special] nodes (y * pitch + x) with M_QLINK
    int32_t n_special;
    int32_t pad2;
};

// A job in the continuous-batching table (device memory).
struct alignas(16) MultiJob {
    JobDev j;
    int64_t t;        // steps done at the current base
    int64_t n_steps;  // the job's target; tiles of finished jobs are skipped
    int64_t tile0;    // first global tile of the job
    int64_t adv;      // steps of this job per tick (launches k >= adv skip it)
    int32_t tiles_x, tiles_y;
};

// A job of a batched fused launch (device table, continuous batching with
// temporal blocking): every chunk of every sample of every job in the table
// advances N steps per launch through one kernel instance. Jobs differ in
// lattice (up to the instance's row width), sample count and step parity.
struct alignas(16) FusedJob {
    JobDev j;
    const int64_t *d_t;  // the job's device step count (inflow ramp)
    int64_t work0;       // first work item: the job has S * chunks * strips
    int32_t H, chunks;   // rows per chunk, chunks per sample
    int32_t W, strips;   // strip window: columns per strip, strips per row
                         // (whole rows: W = nx, strips = 1)
    int32_t par;         // t & 1 of the job at the start of the tick
    int32_t pad;
};

// ------------------------------------------------------------------ kernel launchers
struct StepShape {
    int cpt = 1;        // rows per thread (1 or 2)
    int persistent = 0; // 0: one workgroup per tile; >0: workgroups per CU
    int nt = 1;         // AB layout: non-temporal (cache-bypassing) stores
    int layout = UQ_LAYOUT_AA;
    int pad = 64;       // elements of padding after each population plane
    int bx = 64;        // workgroup width along x (64, 128 or 256; height 256/bx)
    int fuse = 0;       // periodic AB jobs: steps per launch of k_stepN (2..4; 0, 1: k_step)
    int fty = 8;        // k_stepN tile height (rows of 64 output nodes); k_stepW chunk rows
    int fwin = 0;       // fused kernel: 0 tiles (k_stepN), 1 sliding window (k_stepW), 2 full rows (k_stepR)
};

// one stream-collide step for all samples at time t = *d_t + k; `parity`
// must equal t & 1 (the host keeps a mirror of t)
hipError_t launch_init(const JobDev &j, hipStream_t s);
// A second stream for the boundary-node kernels (interpolated links,
// finite-difference columns): they run beside k_step of the same step,
// forked from and joined back into the main stream with the two events.
struct SideStream {
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
hipError_t launch_step(const JobDev &j, const int64_t *d_t, int k, int parity, const StepShape &shape,
                       hipStream_t s, const SideStream *side = nullptr);
// n = 2..4 fused steps of a periodic AB job in one launch: the state is
// read from slab f2 if src2 else f and n steps later written to the other
// slab (the host keeps the slab of each step's state; see Job::enqueue_steps)
// (window 1: the sliding-window kernel with chunks of fty rows, its stores
// non-temporal if nt; 2: the same over whole rows; 0: the 64 x fty tile kernel)
// (channel jobs: window 2 only, advancing the steps t = *d_t + k ..; see
// channel_fusable)
hipError_t launch_fused(const JobDev &j, int n, bool src2, int fty, int window, bool nt, const int64_t *d_t, int k,
                        hipStream_t s);
// channel jobs the fused channel kernel takes: AB, half-way walls and
// cylinder, Zou-He / wall / periodic ends (no interpolated rule)
bool channel_fusable(const JobDev &j);
// widest channel the fused channel kernel takes at this precision and N
int channel_rows_max_nx(int prec, int n);
// widest lattice the full-row kernel takes at this precision and N (0: none)
int full_rows_max_nx(int prec, int n);
bool fused_supported(const JobDev &j);
// Batched fused launches (continuous batching with temporal blocking).
// kind 0: periodic lattice over whole rows, kind 1: channel over whole rows,
// kind 2: periodic lattice in strips of at most 64 - 2(N - 1) columns (any
// width). rows_instance gives the waves per level K and columns per lane M
// of the N-step whole-row instance for rows nx wide (0 if none fits);
// fused_multi_supported says whether the batched form of an instance exists
// (N in {4, 6, 8} periodic rows, {2, 3, 4} channel rows, 4 strips; single-
// precision storage formats). window_strips gives the strips per row and
// their width for N steps.
int rows_instance(int kind, int prec, int n, int nx, int *K, int *M);
bool fused_multi_supported(int kind, int prec, int n, int K, int M);
void window_strips(int nx, int n, int *W, int *strips);
// launch number `launch` of a tick: every work item of jobs[0..njobs)
hipError_t launch_fused_multi(int kind, int prec, int n, int K, int M, const FusedJob *jobs, int njobs,
                              int64_t nwork, int launch, hipStream_t s);
// *d_t[q] += n for q < njobs
hipError_t launch_advance_ptrs(int64_t *const *d_t, int njobs, int64_t n, hipStream_t s);
// one step of every job in a table (AA layout, one row per thread); all jobs
// must share precision `prec`
hipError_t launch_step_multi(const MultiJob *jobs, int njobs, int64_t ntiles, int k, int prec, hipStream_t s);
hipError_t launch_advance_multi(MultiJob *jobs, int njobs, hipStream_t s);  // t += adv
void tile_counts(const JobDev &j, int cpt, int *tiles_x, int *tiles_y);
// *d_t += n (one thread; keeps the device copy of the step count current)
hipError_t launch_advance(int64_t *d_t, int64_t n, hipStream_t s);
// per-sample scalar QoIs at time t: out[S][4] = {KE, Fx, Fy, nonfinite}
hipError_t launch_qoi_scalars(const JobDev &j, int64_t t, double *out, hipStream_t s);
// out[0] = the first sample s whose scalars above flag a non-finite value,
// or S if none (one workgroup; overwrites out[0], nothing to clear)
hipError_t launch_first_bad(const double *qoi, int64_t S, int64_t *out, hipStream_t s);
// M[s] = KE, C_D or C_L of sample s from the scalars above
hipError_t launch_select_scalar(const JobDev &j, const double *qoi, int which, double *M, hipStream_t s);
// per-sample fields at time t: out[S][4][ny][nx] = {ux, uy, rho, |u|}
hipError_t launch_fields(const JobDev &j, int64_t t, double *out, hipStream_t s);
// unshifted double populations of one sample in natural order
hipError_t launch_export(const JobDev &j, int64_t t, int64_t sample, double *out, hipStream_t s);

// Statistics of a field QoI (VEL, RHO, SPEED) at time t straight from the
// populations (no per-sample field buffer); the same results as the
// buffered path above. SC: K > 0 with wphi, a; MC: K = 0. coeffs[K][n_out].
hipError_t launch_field_moments(const JobDev &j, int64_t t, int qoi, const double *wphi, const double *a, int K,
                                double *coeffs, double *mean, double *var, double *var_alt, hipStream_t s);
// Statistics of a scalar QoI M[S], each sum split across a workgroup in a
// fixed order. SC: K > 0 with wphi, a; MC: K = 0.
hipError_t launch_scalar_moments(const double *M, int64_t S, const double *wphi, const double *a, int K,
                                 double *coeffs, double *mean, double *var, double *var_alt, hipStream_t s);

}  // namespace uqi
