/*
 * uq.h -- C-ABI of the MI355X batched lattice-Boltzmann UQ library.
 *
 * The library runs the non-intrusive uncertainty-quantification method of
 * OpenLB-UQ (arXiv 2508.13867): an ensemble of deterministic D2Q9 BGK solves,
 * one per sample of the uncertain inputs (Sec. "Uncertainty quantification
 * methods", Algorithm alg:uq_openlb), followed by Monte Carlo statistics
 * (Eqs. meanMCS, varMCS) or the stochastic-collocation gPC projection
 * (Eqs. coef_discrete, gpc_mean, gpc_std). All samples of a job advance
 * together on one GPU; every step of the path runs in the library's HIP
 * kernels for gfx950.
 *
 * Conventions for every call:
 *  - Functions return uq_status; on failure uq_last_error() returns a
 *    message for the calling thread. No C++ exception crosses the ABI.
 *  - Host pointers are caller-owned; the library never keeps them past the
 *    call. Device memory of a job is owned by the job and released by
 *    uq_destroy().
 *  - Calls on distinct jobs may be made from different threads. Calls on the
 *    same job must not overlap.
 *  - All quantities are in lattice units (dx = dt = 1).
 */
#ifndef UQ_LBM_H
#define UQ_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    UQ_OK = 0,
    UQ_EINVAL = 1,    /* invalid argument (tau <= 1/2, bad sizes, bad enum) */
    UQ_ENOMEM = 2,    /* device allocation failed / job can never fit       */
    UQ_EAGAIN = 3,    /* not finished yet (server polling)                  */
    UQ_EUNSTABLE = 4, /* a sample produced a non-finite value               */
    UQ_EDEVICE = 5,   /* a HIP runtime call failed                          */
    UQ_ESTATE = 6     /* call not valid in the object's current state       */
} uq_status;

/* Storage precision of the populations. Collision always runs on shifted
 * populations f_i - w_i; FP64 computes in double, the others in float. */
typedef enum {
    UQ_FP64 = 0,  /* double storage, double compute                        */
    UQ_FP32 = 1,  /* float storage, float compute                          */
    UQ_FP16S = 2, /* IEEE half storage scaled by 2^s per job, float compute */
    UQ_BF16S = 3  /* bfloat16 storage (unscaled), float compute           */
} uq_precision;

/* Memory layout of the populations (an execution choice; results agree to
 * rounding). AA: one slab updated in place (AA access pattern). AB: two slabs,
 * pull from one and write aligned to the other (twice the memory, higher
 * HBM rate on MI355X). AUTO: the launch-shape tuner's choice for the
 * problem class (AA unless a measured AB entry exists or UQ_LAYOUT is set). */
typedef enum { UQ_LAYOUT_AUTO = 0, UQ_LAYOUT_AA = 1, UQ_LAYOUT_AB = 2 } uq_layout;

/* Deterministic problem solved for every sample. */
typedef enum {
    /* Taylor-Green vortex on a fully periodic nx x ny lattice (Sec. "Taylor--
     * Green vortex flow with uncertain viscosity", Eqs. TGV_vel, TGV_press):
     * u = u0(-cos(kx+px) sin(ky+py), sin(kx+px) cos(ky+py)), k = 2 pi/n,
     * rho = 1 + 3p, equilibrium start. */
    UQ_GEOM_TGV = 0,
    /* Channel of nx x ny nodes with half-way bounce-back walls at y = -1/2
     * and y = ny - 1/2, an optional solid cylinder of diameter D centred on
     * node (cx, cy), and an x boundary chosen by `xbc` (Sec. "Flow past a
     * circular cylinder with uncertain inlet velocity"). */
    UQ_GEOM_CHANNEL = 1
} uq_geometry;

typedef enum {
    UQ_XBC_ZOUHE = 0,   /* Zou-He parabolic velocity inlet at x = 0 and Zou-He
                           pressure outlet (rho = 1) at x = nx-1            */
    UQ_XBC_WALLS = 1,   /* half-way bounce-back walls at x = -1/2, nx - 1/2 */
    UQ_XBC_PERIODIC = 2, /* periodic in x                                   */
    /* the paper's interpolated inlet and outlet (Sec. "Flow past a circular
     * cylinder with uncertain inlet velocity", after Latt et al., Phys. Rev.
     * E 77, 056703, 2008): every population of an open-column node is
     * rebuilt as equilibrium plus the first-order non-equilibrium part
     * -w_i rho tau/cs^2 Q_i : grad u, Q_i = c_i c_i - cs^2 I, with grad u by
     * second-order finite differences (one-sided into the fluid across the
     * column, central along it, one-sided at its two ends). Inlet: the
     * parabolic velocity, rho from the known populations; outlet: rho = 1,
     * u_y = 0, u_x from the known populations. Needs the AB layout, nx >= 4,
     * and the cylinder at least 3 nodes away from both columns. */
    UQ_XBC_INTERP = 3
} uq_xbc;

/* Cylinder wall treatment (channel). */
typedef enum {
    /* solid nodes 4((x-cx)^2 + (y-cy)^2) <= D^2 on the integer centre (cx,
     * cy); half-way bounce-back on every link into them */
    UQ_CYL_HALFWAY = 0,
    /* the exact circle of centre (cyl_x, cyl_y) and diameter cyl_d (solid
     * iff (x-cyl_x)^2 + (y-cyl_y)^2 <= (cyl_d/2)^2) with the linear
     * interpolated bounce-back of Bouzidi, Firdaouss and Lallemand (Phys.
     * Fluids 13, 3452, 2001), the paper's second-order curved wall: for the
     * link from fluid node x along c_k that meets the circle at fraction q,
     *   q <  1/2: f_opp(k)(x, t+1) = 2q f*_k(x) + (1-2q) f*_k(x - c_k)
     *   q >= 1/2: f_opp(k)(x, t+1) = f*_k(x)/(2q) + (1 - 1/(2q)) f*_opp(k)(x).
     * Forces by momentum exchange over the same links, F = sum c_k (f*_k(x)
     * + f_opp(k)(x, t+1)) (Mei et al., J. Comput. Phys. 175, 2002). Needs
     * the AB layout and the circle at least 2 nodes inside the walls and 3
     * nodes away from the x ends. */
    UQ_CYL_BOUZIDI = 1
} uq_cyl_bc;

/* Velocity that normalises C_D, C_L and that a Reynolds-number input uses
 * (nu = U D/Re with the nominal peak): */
typedef enum {
    UQ_FORCE_REF_PEAK = 0, /* U = the sample's peak inflow u_peak           */
    UQ_FORCE_REF_MEAN = 1  /* U = the mean of the parabola, 2/3 u_peak       */
} uq_force_ref;

/* Input that an uncertain variable drives. */
typedef enum {
    UQ_T_NU = 0,      /* kinematic viscosity; tau = 3 nu + 1/2             */
    UQ_T_U0 = 1,      /* TGV velocity amplitude                            */
    UQ_T_PHASE_X = 2, /* TGV phase shift in x (radians)                    */
    UQ_T_PHASE_Y = 3, /* TGV phase shift in y                              */
    UQ_T_RE = 4,      /* channel Reynolds number; nu = u_peak_nominal D/Re */
    UQ_T_U_PEAK = 5,  /* channel peak inflow velocity                      */
    /* amplitudes zeta_{ij} of the harmonic perturbation of the TGV with
     * init = UQ_INIT_TGV_HARMONIC (i, j in {0, 1}) */
    UQ_T_ZETA00 = 6,
    UQ_T_ZETA01 = 7,
    UQ_T_ZETA10 = 8,
    UQ_T_ZETA11 = 9
} uq_target;

/* Initial field of the vortex. */
typedef enum {
    /* u = u0(-cos(kx+px) sin(ky+py), sin(kx+px) cos(ky+py)), k = 2 pi/n */
    UQ_INIT_TGV = 0,
    /* the four-dimensional perturbed vortex (Sec. "Taylor--Green vortex flow
     * with four-dimensional uncertain initial velocity perturbation", Eq.
     * taylorGreen): two periods over the lattice, kappa = 4 pi/n,
     *   u = u0^R (-cos(kappa x) sin(kappa y), sin(kappa x) cos(kappa y)),
     *   p = -(u0^R)^2/4 (cos(2 kappa x) + cos(2 kappa y)), rho = 1 + 3p,
     *   u0^R = u0 (1 + eps), eps = 1/4 sum_{i,j in {0,1}} zeta_ij
     *          k_i(2 kappa x) k_j(2 kappa y), k_0 = sin, k_1 = cos
     * (the paper's physical amplitude is 1, so its additive perturbation is
     * relative to u0 here). */
    UQ_INIT_TGV_HARMONIC = 1
} uq_init;

/* One independent uniform input U(lo, hi) (Sec. "Distribution and
 * polynomial basis"); its reference variable xi on [-1, 1] maps to
 * lo + (hi - lo)(xi + 1)/2. */
typedef struct {
    int32_t target; /* uq_target */
    double lo, hi;
} uq_dist;

typedef enum {
    /* Tensor Gauss-Legendre collocation with n_per_dim nodes per input and
     * weights of the probability measure (sum 1), dimension 0 varying
     * slowest; gPC of total degree <= order in graded order (Sec. "Quadrature
     * and collocation", SC-gPC procedure). */
    UQ_RULE_GL_TENSOR = 0,
    /* Monte Carlo: mc_n i.i.d. draws from SplitMix64 seeded with `seed`; draw
     * number c = j*d + k + 1 feeds sample j, input k (Sec. "Monte Carlo and
     * quasi Monte Carlo sampling"). */
    UQ_RULE_MC = 1,
    /* Smolyak sparse grid of nested Clenshaw-Curtis rules (Sec. "Quadrature
     * and collocation": Clenshaw-Curtis, sparse Smolyak grids), sparse level
     * `level` >= 0 (1-D rules of 1, 3, 5, 9, 17, ... nodes); points are the
     * union of the tensor grids, ordered lexicographically (input 0 most
     * significant); weights of the probability measure, some negative; gPC
     * of total degree <= order, exact for order <= level when the response is
     * polynomial. In d = 4 the levels 0..4 have 1, 9, 41, 137, 401 points. */
    UQ_RULE_SMOLYAK_CC = 2,
    /* Quasi Monte Carlo: the first mc_n points of the Halton sequence (radical
     * inverses in the first d primes) starting at index 1; equal weights,
     * Monte Carlo statistics (Sec. "Monte Carlo and quasi Monte Carlo
     * sampling"). */
    UQ_RULE_HALTON = 3,
    /* Latin hypercube sampling of mc_n points: per input a random permutation
     * of the mc_n strata and a uniform position inside each, drawn from
     * SplitMix64 seeded with `seed` (Sec. "Sampling strategies"); equal
     * weights, Monte Carlo statistics. */
    UQ_RULE_LHS = 4
} uq_rule;

#define UQ_MAX_DIMS 8

typedef struct {
    int32_t geometry;  /* uq_geometry */
    int32_t precision; /* uq_precision */
    int32_t nx, ny;    /* lattice nodes, >= 2 (TGV) / nx >= 2, ny >= 3 (channel) */
    /* nominal (deterministic) inputs */
    double nu;               /* viscosity (both geometries unless driven)          */
    double u0;               /* TGV amplitude; also the energy normalisation       */
    double phase_x, phase_y; /* TGV phases                                        */
    double u_peak;           /* channel peak inflow velocity (also in Re -> nu)   */
    int32_t D, cx, cy;       /* cylinder diameter (0 = none) and centre node     */
    int32_t xbc;             /* uq_xbc                                           */
    int64_t ramp;            /* inflow ramp length T_r: s(t) = sin^2(pi t/(2T_r)) */
    /* uncertain inputs */
    int32_t n_dists;
    uq_dist dists[UQ_MAX_DIMS];
    /* sampling / collocation rule */
    int32_t rule;      /* uq_rule */
    int32_t n_per_dim; /* GL: nodes per input                               */
    int32_t order;     /* GL / SMOLYAK_CC: total gPC degree P (K = C(d+P, P)) */
    int64_t mc_n;      /* MC / HALTON / LHS: number of samples              */
    uint64_t seed;     /* MC / LHS: generator seed                          */
    int32_t layout;    /* uq_layout                                         */
    int32_t level;     /* SMOLYAK_CC: sparse-grid level                     */
    int32_t init;      /* uq_init (vortex only)                             */
    int32_t cyl_bc;    /* uq_cyl_bc (channel)                               */
    int32_t force_ref; /* uq_force_ref (channel)                            */
    double cyl_x, cyl_y, cyl_d; /* exact circle of UQ_CYL_BOUZIDI          */
} uq_problem;

/* Device context. `stream` is a hipStream_t (e.g. torch's current stream,
 * NULL = the null stream). When `alloc`/`free` are NULL the library uses
 * hipMalloc/hipFree; otherwise every device buffer of a job comes from
 * alloc(bytes, ctx) (256-byte aligned) and goes back through free(ptr, ctx). */
typedef void *(*uq_alloc_fn)(size_t bytes, void *ctx);
typedef void (*uq_free_fn)(void *ptr, void *ctx);
typedef struct {
    int32_t device;
    void *stream;
    uq_alloc_fn alloc;
    uq_free_fn free;
    void *ctx;
} uq_device;

typedef struct uq_job uq_job;

/* Quantities of interest. */
typedef enum {
    /* normalised total kinetic energy K = 2/(nx ny u0^2) sum (u^2 + v^2)
     * over fluid nodes, u0 the nominal amplitude (Eq. KineticEnergy).    */
    UQ_QOI_KE = 0,
    /* velocity field, n_out = 2 nx ny: all u_x in row-major [ny][nx], then
     * all u_y; 0 at solid nodes (Fig. velocity_stats statistics).        */
    UQ_QOI_VEL = 1,
    /* drag / lift coefficient 2F/(U^2 D) from momentum exchange on the
     * cylinder links of the final state (half-way: F = sum 2 c_i f*_i over
     * links into the cylinder; interpolated links as under uq_cyl_bc), U
     * the sample's peak inflow or its mean (uq_force_ref), D the diameter
     * (Eqs. dragForce, liftForce and the C_D, C_L definitions).         */
    UQ_QOI_CD = 2,
    UQ_QOI_CL = 3,
    /* density field [ny][nx], 0 at solid nodes */
    UQ_QOI_RHO = 4,
    /* speed field |u| [ny][nx], 0 at solid nodes */
    UQ_QOI_SPEED = 5
} uq_qoi;

/* Statistics of one QoI over the samples, caller-owned host buffers; any
 * pointer may be NULL to skip that output. n_out and K are filled in.
 *   mean[n_out]      MC: Eq. meanMCS; SC: coefficient 0 (Eq. gpc_mean)
 *   var[n_out]       MC: Eq. varMCS (1/(N-1)); SC: sum_{k>=1} c_k^2 (Eq. gpc_std)
 *   var_alt[n_out]   MC: the 1/N variance of Algorithm alg:uq_openlb;
 *                    SC: quadrature variance sum_j a_j (M_j - mean)^2
 *   coeffs[K*n_out]  SC only: c_k for k = 0..K-1, row k at coeffs + k*n_out
 *   alpha[K*d]       SC only: multi-index of term k at alpha + k*d          */
typedef struct {
    int64_t n_out;
    int32_t K;
    int32_t d;
    double *mean;
    double *var;
    double *var_alt;
    double *coeffs;
    int32_t *alpha;
} uq_moments_out;

typedef struct {
    int64_t S;          /* samples                                     */
    int32_t d;          /* uncertain inputs                            */
    int32_t K;          /* gPC terms (0 for MC)                        */
    int64_t steps_done; /* LBM steps taken so far                      */
    int64_t pitch;      /* row pitch of a population plane (elements)  */
    int64_t device_bytes; /* device memory held by the job            */
    int32_t scale_exp;  /* FP16S storage scale 2^scale_exp (else 0)    */
    int32_t fluid_nodes;
    int32_t layout;     /* uq_layout in use (AA or AB)                 */
    int32_t cpt;        /* rows per thread of the step kernel          */
    int32_t nt_store;   /* 1 if AB stores bypass the caches            */
    int32_t plane_pad;  /* padding elements after each population plane */
    int32_t bx;         /* step-kernel workgroup width (height 256/bx) */
    int32_t fused;      /* steps per launch of the fused AB kernel
                           (tiles and strips 2..4, whole periodic rows
                           2..8, whole channel rows 2..4), 0 if not
                           fused                                       */
    int32_t fused_rows; /* its tile height (rows of 64 nodes), or the
                           window kernel's chunk height               */
    int64_t step_launches; /* step-kernel launches so far (a fused launch
                              counts once: each launch reads and writes
                              every population of every sample once)  */
    int32_t fused_window; /* fused kernel: 0 tiles, 1 sliding window
                             down strips, 2 sliding window over whole
                             rows                                      */
    int32_t pad3;
} uq_job_info;

/* Set up a job: sample the inputs, map each sample to its solver parameters,
 * allocate the population slab and initialise every sample to equilibrium
 * (enqueued on dev->stream). The problem is copied. */
uq_status uq_create(const uq_problem *p, const uq_device *dev, uq_job **out);

/* Sample matrix and weights (getSamplingPoints of the paper's user API).
 * xi: [S*d] reference variables in [-1,1], a: [S] weights. Any pointer may
 * be NULL; S and d are returned through the pointers if not NULL. */
uq_status uq_samples(const uq_job *job, double *xi, double *a, int64_t *S, int32_t *d);

/* Advance all samples by `steps` LBM steps (stream + collide with the
 * boundaries inline). Every launch advances all samples: one step per launch,
 * or, in the fused shapes the tuner picks for periodic lattices and simple
 * channels in the AB layout, N = 2..8 steps per launch (temporal blocking).
 * Whole blocks of fused launches are replayed from a captured hipGraph; the
 * steps left over run as launches of an odd number (3 or more, at most N) of
 * fused steps, largest first, and the last one or two as single steps, so
 * the state after `steps` steps does not depend on N. Asynchronous on the
 * job's stream; steps >= 0. */
uq_status uq_run(uq_job *job, int64_t steps);

/* uq_run followed by a wait, with the elapsed device time of the step
 * launches measured by HIP events on the job's stream: *ms receives the
 * total over the `steps` steps (divide by steps for the average launch
 * duration of the step kernel). Blocking. */
uq_status uq_run_timed(uq_job *job, int64_t steps, double *ms);

/* Wait for all work of the job. */
uq_status uq_sync(uq_job *job);

/* Per-sample QoI values at the current step, computed on the device and
 * copied to out[S * n_out] (sample-major). *n_out receives values per
 * sample. out may be NULL to query n_out. Blocking. */
uq_status uq_qoi_samples(uq_job *job, int32_t qoi, double *out, int64_t *n_out);

/* Statistics of a QoI at the current step: per-sample reduction, then the
 * cross-sample moments / gPC projection in compensated FP64, all on the
 * device; results copied to the caller's buffers. Blocking. Returns
 * UQ_EUNSTABLE if any sample holds a non-finite value. */
uq_status uq_moments(uq_job *job, int32_t qoi, uq_moments_out *out);

/* uq_moments without any device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels and the same results
 * (bit for bit) as uq_moments, with their intermediates -- per-sample scalar
 * QoIs, the moment outputs and a flag -- in a fixed array of
 * UQ_NOALLOC_SCRATCH_BYTES that the library keeps on every GPU it runs on
 * until the process ends, instead of buffers the job would allocate on its
 * first statistics call. The job's own device memory is untouched
 * (uq_job_info.device_bytes stays the same). The need is the sum of
 *   8 * 4 S, 8 * S, 8 and 8 * (K + 3) n_out bytes, each rounded up to 256
 * (field moments are formed from the populations, with no per-sample field
 * buffer);
 * larger requests fail with UQ_EINVAL and a message naming both sizes (use
 * uq_moments then). Calls on one GPU share its array: the library runs them
 * one at a time (each holds the GPU's lock until its results are on the
 * host), so calls from several threads are safe but do not overlap. Same
 * arguments, outputs, errors and blocking behaviour as uq_moments. */
#define UQ_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
uq_status uq_moments_noalloc(uq_job *job, int32_t qoi, uq_moments_out *out);

/* Populations f_i(x, t) of one sample in natural order [9][ny][nx], unshifted
 * and in double, for inspection and tests (solid nodes hold 0). Blocking. */
uq_status uq_populations(uq_job *job, int64_t sample, double *out);

uq_status uq_job_get_info(const uq_job *job, uq_job_info *info);

/* Release every device buffer of the job (after its stream is idle). */
void uq_destroy(uq_job *job);

/* Message of the last failure on the calling thread ("" if none). */
const char *uq_last_error(void);

/* Launch-shape autotuning. Times the step kernel of the problem (its real
 * lattice and sample count) for every candidate shape -- layout AA or AB
 * (only the problem's layout unless it is UQ_LAYOUT_AUTO), workgroups of
 * 64 x 4, 128 x 2 or 256 x 1 threads, 1 or 2 rows per thread, plane padding
 * 0 or 64 elements, cached or non-temporal AB stores, and for periodic
 * lattices in AB the fused kernels (2, 3 or 4 steps per launch: on tiles of
 * 64 x rows nodes kept in LDS between the steps, with a ring of one node per
 * extra step, rows 8 or 16, FP64 4 or 8; or as a sliding window, one wave
 * per step, down strips of at most 64 - 2(N - 1) columns or down whole rows
 * of up to 256 columns (K waves per step, one or two columns per lane,
 * N K <= 16, 3 to 8 steps where (N - 1) 21 rows fit in the LDS), in chunks of 64 or
 * 256 rows, FP64 32 or 64), and for channels in AB with half-way walls and
 * cylinder and Zou-He, wall or periodic ends the fused kernel over whole rows
 * (2 to 4 steps per launch where the LDS rows fit: FP32 N = 3 at 440
 * columns; the height cut into 1 to 8 balanced chunks) --
 * over `steps` steps each (at least 120; rounded down to whole launches of a
 * fused kernel: N steps, 2N for even N), on
 * dev's device with temporary jobs. The fastest becomes the shape of every later job of the
 * same class (precision, geometry, nx, ny, S, layout field) in this process,
 * and is appended to the file named by UQ_TUNE_CACHE if set. Candidates that
 * do not fit in device memory are skipped. Blocking. */
typedef struct {
    int32_t layout;
    int32_t cpt;
    int32_t nt_store;
    int32_t plane_pad;
    int32_t bx;         /* workgroup width along x: 64, 128 or 256          */
    double gbs;         /* GB/s of the best at 18 b per node and step (a ranking
                           figure: a fused launch moves 18 b per node for all of
                           its steps, so for those it exceeds the traffic)      */
    double ms_per_step; /* its average step duration                           */
    int32_t n_candidates;
    int32_t fused;      /* steps per launch of the best if fused (2..8), else 0 */
    int32_t fused_rows; /* its tile height (window: chunk height)              */
    int32_t fused_window; /* 0 tiles, 1 window strips, 2 window over whole rows */
} uq_tune_result;
uq_status uq_autotune(const uq_problem *p, const uq_device *dev, int64_t steps, uq_tune_result *out);

/* ------------------------------------------------------------------------
 * Serving: a request loop on its own host thread. Jobs are admitted first
 * come, first served while their device footprint fits in the server's
 * memory arena (allocated once at creation; serving itself never calls
 * hipMalloc/hipFree) and fewer than max_jobs are live. In BATCHED mode every
 * sample of every live job advances together, in ticks of a multiple of 48
 * steps (steps_per_tick rounded to the nearest, at least 48) replayed from
 * one captured hipGraph while the live set is unchanged: periodic vortex
 * lattices and channels with half-way walls, cylinder and Zou-He, wall or
 * periodic ends in single-precision storage run in the AB layout, N steps
 * per launch over whole rows (N from the launch-shape tuner's measurement of
 * the job's class when it has one, else the largest that fits: vortex 8, 6
 * or 4, channel 4, 3 or 2), one launch for all jobs that share a kernel
 * instance; vortex lattices too wide for whole rows run 4 steps per launch
 * in column strips when their two slabs take at most a quarter of the
 * arena; the other jobs (FP64, wide channels, very large vortex jobs) run in
 * the AA layout, one launch per step for all of them. Jobs of different lattices, geometries,
 * sample counts and step parities share launches. A job with fewer steps
 * left than a tick takes its last steps in launches of its own. PLAIN mode
 * runs one job at a time and one sample per launch per step (AA), with no
 * graph. Fused and single steps give bit for bit the same populations, so a
 * job's result is the same in either mode, alone or in any mix. All jobs of
 * a server share its precision. Results are one scalar QoI per job (KE, CD
 * or CL): its statistics as in uq_moments. */
typedef enum { UQ_SERVE_BATCHED = 0, UQ_SERVE_PLAIN = 1 } uq_serve_mode;

typedef struct {
    int64_t memory_budget;  /* bytes of device memory for resident jobs        */
    int32_t max_jobs;       /* live jobs at once (1..4096)                     */
    int32_t steps_per_tick; /* steps between admission checks (>= 2; BATCHED:
                               rounded to a multiple of 48)                   */
    int32_t mode;           /* uq_serve_mode                                   */
    int32_t use_graph;      /* capture each tick of the batched mode           */
    int32_t precision;      /* uq_precision of every job                       */
} uq_server_config;

#define UQ_RESULT_MAX_COEFFS 256
typedef struct {
    uint64_t ticket;
    int32_t status; /* UQ_OK, UQ_EUNSTABLE, ...                              */
    int32_t qoi;
    int64_t S;
    int32_t K;      /* gPC terms (0 for MC); coeffs holds the first 256       */
    int32_t pad0;
    double mean, var, var_alt;
    double coeffs[UQ_RESULT_MAX_COEFFS];
    double t_submit, t_admit, t_done; /* seconds since server creation       */
    double node_updates;              /* S * nx * ny * steps                 */
} uq_result;

typedef struct {
    int64_t submitted, completed, failed, pending, live;
    double elapsed_s;       /* since creation                                  */
    double busy_s;          /* host time spent in step ticks                   */
    double node_updates;    /* of completed jobs                               */
    double solves_per_hour; /* completed / elapsed                             */
    double mlups;           /* node_updates / elapsed / 1e6                    */
    double latency_p50_s, latency_p99_s, latency_mean_s; /* done - submit      */
    int64_t arena_bytes, arena_peak_bytes;
} uq_server_stats;

typedef struct uq_server uq_server;

/* Start a server on dev->device (dev may be NULL: device 0, hipMalloc,
 * the null stream). Its arena of cfg->memory_budget bytes is allocated here,
 * through dev->alloc when the caller gives allocator callbacks (e.g. torch's
 * caching allocator, as the job API does) and else with hipMalloc; it holds
 * every resident job and the batching tables, and goes back through
 * dev->free at uq_server_destroy. dev->stream orders the server against the
 * caller: the loop's first work waits for what the caller had queued on it
 * (the arena's allocation), and uq_server_destroy makes it wait for the
 * loop's last work before the arena is freed. The loop itself runs on a
 * stream of its own. */
uq_status uq_server_create(const uq_server_config *cfg, const uq_device *dev, uq_server **out);
/* Queue a job; never blocks. UQ_ENOMEM if it can never fit the arena. The
 * problem is copied. *ticket identifies the result. */
uq_status uq_server_submit(uq_server *s, const uq_problem *p, int64_t steps, int32_t qoi, uint64_t *ticket);
/* Result of a finished job (copied out and forgotten), else UQ_EAGAIN. */
uq_status uq_server_poll(uq_server *s, uint64_t ticket, uq_result *out);
/* Wait up to timeout_s (< 0: forever) for a result; UQ_EAGAIN on timeout. */
uq_status uq_server_wait(uq_server *s, uint64_t ticket, double timeout_s, uq_result *out);
uq_status uq_server_get_stats(uq_server *s, uq_server_stats *out);
/* Stop the loop, abandon queued and live jobs, release all device memory. */
void uq_server_destroy(uq_server *s);

/* 1-Wasserstein distance between the numerical statistical solutions of two
 * jobs at their current steps (Sec. "Taylor--Green vortex flow with
 * four-dimensional uncertain initial velocity perturbation", Eq. of W_1):
 * the law of a field QoI of job a (every value of every sample, value o of
 * sample j carrying weight a_j / n_out, each value multiplied by scale_a)
 * against the same for job b, W_1 = integral |F_a - F_b|. Both jobs must be
 * on the same device; the result is computed there (sort, prefix sums,
 * quantile overlap, compensated sum) on job a's stream. qoi must be a field
 * (VEL, RHO or SPEED). Blocking. */
uq_status uq_wasserstein1(uq_job *a, uq_job *b, int32_t qoi, double scale_a, double scale_b, double *w1);

/* Lattice units of the paper's four-dimensional vortex case (Table
 * tab:simulation_parameters): for n nodes per side, Mach number Ma and
 * Reynolds number Re (physical velocity 1, viscosity 1/Re, domain 2 pi):
 * dx = 2 pi/(n-1), u_lat = Ma/sqrt(3), dt = dx u_lat, nu_lat = dt/(Re dx^2),
 * tau = 3 nu_lat + 1/2. Host only. */
uq_status uq_tgv_units(int32_t n, double Ma, double Re, double *nu_lat, double *u_lat, double *dx, double *dt,
                       double *tau);

/* Host-only helpers (no device needed): the job's sample set and basis,
 * for callers that want the rule without creating a job.
 *   uq_rule_size: S and K of a problem.
 *   uq_rule_points: xi [S*d], a [S], alpha [K*d], phi [S*K]; any may be NULL. */
uq_status uq_rule_size(const uq_problem *p, int64_t *S, int32_t *K);
uq_status uq_rule_points(const uq_problem *p, double *xi, double *a, int32_t *alpha, double *phi);

#ifdef __cplusplus
}
#endif
#endif /* UQ_LBM_H */
