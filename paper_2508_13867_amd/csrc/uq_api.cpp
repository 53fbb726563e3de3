// C-ABI of the batched LBM-UQ library: job set-up, time stepping, per-sample
// QoIs and cross-sample statistics (Algorithm alg:uq_openlb of OpenLB-UQ,
// arXiv 2508.13867, with the solve loop replaced by one batched launch per
// step over all samples).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "uq_internal.h"
#include "uq_job.h"

namespace uqi {

// ------------------------------------------------------------------ device memory
void *Job::dalloc(size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (dev.alloc) {
        p = dev.alloc(bytes, dev.ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    if (p) {
        allocs.push_back(p);
        bytes_held += (int64_t)bytes;
    }
    return p;
}

void Job::dfree(void *p) {
    for (size_t i = 0; i < allocs.size(); ++i)
        if (allocs[i] == p) {
            if (dev.free)
                dev.free(p, dev.ctx);
            else
                (void)hipFree(p);
            allocs.erase(allocs.begin() + (long)i);
            return;
        }
}

void Job::dfree_all() {
    for (void *p : allocs) {
        if (dev.free)
            dev.free(p, dev.ctx);
        else
            (void)hipFree(p);
    }
    allocs.clear();
    bytes_held = 0;
}

int64_t storage_bytes(int prec) { return prec == UQ_FP64 ? 8 : (prec == UQ_FP32 ? 4 : 2); }

int64_t row_pitch(int nx) { return ((int64_t)nx + 63) / 64 * 64; }

// Channel node classification (see M_* bits in uq_internal.h). The pull
// source of direction i at node x is x - c_i: beyond the walls y = -1/2,
// ny - 1/2 -> bounce-back; beyond x = -1/2 or nx - 1/2 -> per xbc; a solid
// cylinder node -> bounce-back (interpolated for UQ_CYL_BOUZIDI, with the
// link fraction in q[i][y][pitch]).
static bool cyl_solid(const uq_problem &p, int x, int y) {
    if (p.cyl_bc == UQ_CYL_BOUZIDI) {
        const double dx = x - p.cyl_x, dy = y - p.cyl_y, r = 0.5 * p.cyl_d;
        return dx * dx + dy * dy <= r * r;
    }
    if (p.D <= 0) return false;
    const int64_t dx = x - p.cx, dy = y - p.cy;
    return 4 * (dx * dx + dy * dy) <= (int64_t)p.D * p.D;
}

static const int HCX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int HCY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

// Fraction t in (0, 1] of the link from fluid node (x, y) towards
// (x, y) - c_i at which it enters the circle: the smaller root of
// |d - t c_i|^2 = r^2, d = (x, y) - centre, in the cancellation-free form
// t = (|d|^2 - r^2) / (h + sqrt(h^2 - |c_i|^2 (|d|^2 - r^2))), h = c_i . d.
static double circle_fraction(const uq_problem &p, int x, int y, int i) {
    const double dx = x - p.cyl_x, dy = y - p.cyl_y, r = 0.5 * p.cyl_d;
    const double a = (double)(HCX[i] * HCX[i] + HCY[i] * HCY[i]);
    const double h = HCX[i] * dx + HCY[i] * dy;
    const double g = dx * dx + dy * dy - r * r;
    const double t = g / (h + std::sqrt(std::max(0.0, h * h - a * g)));
    return std::min(1.0, std::max(t, 1e-12));
}

void build_mask(const uq_problem &p, int64_t pitch, std::vector<uint32_t> &mask, std::vector<double> &q,
                std::vector<int32_t> &special, int &fluid) {
    const int nx = p.nx, ny = p.ny;
    const bool interp_cyl = p.cyl_bc == UQ_CYL_BOUZIDI;
    const bool open_x = p.xbc == UQ_XBC_ZOUHE || p.xbc == UQ_XBC_INTERP;
    mask.assign((size_t)ny * pitch, M_SOLID);
    q.clear();
    special.clear();
    if (interp_cyl) q.assign((size_t)9 * ny * pitch, 0.0);
    fluid = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            uint32_t m = 0;
            if (cyl_solid(p, x, y)) {
                mask[(size_t)y * pitch + x] = M_SOLID;
                continue;
            }
            ++fluid;
            for (int i = 1; i < 9; ++i) {
                int sx = x - HCX[i], sy = y - HCY[i];
                bool bb = false, open = false, cyl = false;
                if (sy < 0 || sy >= ny) {
                    bb = true;
                } else if (sx < 0 || sx >= nx) {
                    if (p.xbc == UQ_XBC_PERIODIC) {
                        sx = (sx + nx) % nx;
                        bb = cyl = cyl_solid(p, sx, sy);
                    } else if (p.xbc == UQ_XBC_WALLS) {
                        bb = true;
                    } else {
                        open = true;
                    }
                } else {
                    bb = cyl = cyl_solid(p, sx, sy);
                }
                if (bb) m |= 1u << (M_BB + i);
                if (open) m |= 1u << (M_OPEN + i);
                if (cyl && interp_cyl) {
                    m |= M_QLINK;
                    q[((size_t)i * ny + y) * pitch + x] = circle_fraction(p, x, y, i);
                }
                const int dx = x + HCX[i], dy = y + HCY[i];
                if (dx >= 0 && dx < nx && dy >= 0 && dy < ny && cyl_solid(p, dx, dy)) m |= 1u << (M_CYL + i);
            }
            if (open_x && x == 0) m |= M_INLET;
            if (open_x && x == nx - 1) m |= M_OUTLET;
            // boundary nodes stepped by their own kernels: interpolated links
            // (listed) and finite-difference open columns (whole columns)
            if (m & M_QLINK) special.push_back((int32_t)((int64_t)y * pitch + x));
            if ((m & M_QLINK) || (p.xbc == UQ_XBC_INTERP && (m & (M_INLET | M_OUTLET)))) m |= M_SPECIAL;
            mask[(size_t)y * pitch + x] = m;
        }
}

uq_status Job::ensure_stats_buffers(int64_t n_out_max) {
    if (!d_qoi) {
        d_qoi = (double *)dalloc(sizeof(double) * 4 * S);
        d_M = (double *)dalloc(sizeof(double) * S);
        d_flag = (int64_t *)dalloc(sizeof(int64_t));
        if (!d_qoi || !d_M || !d_flag) return fail(UQ_ENOMEM, "out of device memory for QoI buffers");
    }
    if (n_out_max > out_cap) {
        const int64_t per = (int64_t)(K > 0 ? K : 0) + 3;
        d_out = (double *)dalloc(sizeof(double) * per * n_out_max);
        if (!d_out) return fail(UQ_ENOMEM, "out of device memory for moment outputs");
        out_cap = n_out_max;
    }
    return UQ_OK;
}

uq_status Job::ensure_fields() {
    if (!d_fields) {
        const int64_t cells = (int64_t)p.nx * p.ny;
        d_fields = (double *)dalloc(sizeof(double) * 4 * cells * S);
        if (!d_fields) return fail(UQ_ENOMEM, "out of device memory for per-sample fields");
    }
    return UQ_OK;
}

int64_t qoi_width(const uq_problem &p, int qoi) {
    const int64_t cells = (int64_t)p.nx * p.ny;
    switch (qoi) {
        case UQ_QOI_KE:
        case UQ_QOI_CD:
        case UQ_QOI_CL: return 1;
        case UQ_QOI_VEL: return 2 * cells;
        case UQ_QOI_RHO:
        case UQ_QOI_SPEED: return cells;
        default: return 0;
    }
}

uq_status Job::own_stat_bufs(int qoi, bool fields, StatBufs *b) {
    uq_status st = ensure_stats_buffers(qoi_width(p, qoi));
    if (st != UQ_OK) return st;
    if (fields && qoi_width(p, qoi) > 1) {
        st = ensure_fields();
        if (st != UQ_OK) return st;
    }
    b->qoi = d_qoi;
    b->M = d_M;
    b->fields = d_fields;
    b->out = d_out;
    b->flag = d_flag;
    return UQ_OK;
}

}  // namespace uqi

namespace uqi {

uq_status create_job(const uq_problem &prob, const uq_device *dev, const StepShape *forced, uq_job **out) {
    const uq_problem *p = &prob;
    *out = nullptr;
    std::unique_ptr<uq_job> j(new uq_job());
    j->p = *p;
    if (dev) j->dev = *dev;
    uq_status st = build_rule(j->p, j->rule);
    if (st != UQ_OK) return st;
    const uq_problem &P = j->p;
    j->S = j->rule.S;
    j->K = j->rule.K;
    j->pitch = row_pitch(P.nx);
    if (9 * ((int64_t)P.ny * j->pitch + 4096) >= ((int64_t)1 << 31))
        return fail(UQ_EINVAL, "lattice too large for one sample");
    j->user_stream = (hipStream_t)j->dev.stream;
    UQ_HIP_TRY(hipSetDevice(j->dev.device));
    UQ_HIP_TRY(hipStreamCreateWithFlags(&j->stream, hipStreamNonBlocking));
    UQ_HIP_TRY(hipEventCreateWithFlags(&j->ev_in, hipEventDisableTiming));
    UQ_HIP_TRY(hipEventCreateWithFlags(&j->ev_out, hipEventDisableTiming));
    if (needs_ab(P)) {
        UQ_HIP_TRY(hipStreamCreateWithFlags(&j->side.stream, hipStreamNonBlocking));
        UQ_HIP_TRY(hipEventCreateWithFlags(&j->side.fork, hipEventDisableTiming));
        UQ_HIP_TRY(hipEventCreateWithFlags(&j->side.join, hipEventDisableTiming));
    }
    {
        uq_status e = j->enter();
        if (e != UQ_OK) return e;
    }

    // per-sample solver parameters
    std::vector<SampleDev> smp((size_t)j->S);
    double umax = 0.0;
    for (int64_t s = 0; s < j->S; ++s) {
        SampleInputs in;
        map_inputs(P, &j->rule.xi[(size_t)s * j->rule.d], in);
        const double tau = 3.0 * in.nu + 0.5;
        if (!(in.nu > 0.0) || !std::isfinite(tau))
            return fail(UQ_EINVAL, "sample " + std::to_string(s) + " has tau <= 1/2 (nu must be > 0)");
        SampleDev d;
        std::memset(&d, 0, sizeof d);
        d.omega = 1.0 / tau;
        d.u0 = in.u0;
        d.phase_x = in.phase_x;
        d.phase_y = in.phase_y;
        d.u_peak = in.u_peak;
        for (int k = 0; k < 4; ++k) d.zeta[k] = in.zeta[k];
        smp[(size_t)s] = d;
        const double uc = P.geometry == UQ_GEOM_TGV ? std::fabs(in.u0) : 1.5 * std::fabs(in.u_peak);
        umax = std::max(umax, uc);
    }
    // storage scale 2^s for FP16 (bfloat16 has float's exponent range and is
    // stored unscaled): the largest shifted population is about u/3, so
    // 2^12 / (u/2) keeps stored magnitudes near 2^11
    j->scale_exp = 0;
    if (P.precision == UQ_FP16S) {
        const double B = 0.5 * umax + 1e-4;
        j->scale_exp = (int)std::floor(std::log2(4096.0 / B));
        j->scale_exp = std::max(0, std::min(j->scale_exp, 24));
    }

    std::vector<uint32_t> mask;
    std::vector<double> qlink;
    std::vector<int32_t> special;
    j->fluid = P.nx * P.ny;
    if (P.geometry == UQ_GEOM_CHANNEL) build_mask(P, j->pitch, mask, qlink, special, j->fluid);

    // device buffers
    j->shape = forced ? *forced : choose_shape(P, j->S);
    if (needs_ab(P) && j->shape.layout != UQ_LAYOUT_AB)
        return fail(UQ_EINVAL, "interpolated boundaries need the AB layout");
    // padding after each population plane (elements, multiple of 64): spreads
    // the nine plane streams of a wavefront over HBM channels
    const int64_t pad = std::max(0, j->shape.pad) / 64 * 64;
    const int64_t plane = (int64_t)P.ny * j->pitch + pad;
    const int64_t slab_bytes = j->S * 9 * plane * storage_bytes(P.precision);
    void *slab = j->dalloc((size_t)slab_bytes);
    void *slab2 = nullptr;
    if (j->shape.layout == UQ_LAYOUT_AB) {
        slab2 = j->dalloc((size_t)slab_bytes);
        if (!slab2) {
            j->dfree_all();
            return fail(UQ_ENOMEM, "out of device memory for the second slab (" + std::to_string(slab_bytes) + " B)");
        }
    }
    SampleDev *d_smp = (SampleDev *)j->dalloc(sizeof(SampleDev) * j->S);
    j->d_t = (int64_t *)j->dalloc(sizeof(int64_t));
    uint32_t *d_mask = nullptr;
    if (!slab || !d_smp || !j->d_t) {
        j->dfree_all();
        return fail(UQ_ENOMEM, "out of device memory for the population slab (" + std::to_string(slab_bytes) + " B)");
    }
    double *d_q = nullptr;
    int32_t *d_special = nullptr;
    if (!mask.empty()) {
        d_mask = (uint32_t *)j->dalloc(sizeof(uint32_t) * mask.size());
        if (!qlink.empty()) d_q = (double *)j->dalloc(sizeof(double) * qlink.size());
        if (!special.empty()) d_special = (int32_t *)j->dalloc(sizeof(int32_t) * special.size());
        if (!d_mask || (!qlink.empty() && !d_q) || (!special.empty() && !d_special)) {
            j->dfree_all();
            return fail(UQ_ENOMEM, "out of device memory for the boundary mask");
        }
    }
    if (j->K > 0) {
        j->d_wphi = (double *)j->dalloc(sizeof(double) * j->S * j->K);
        j->d_a = (double *)j->dalloc(sizeof(double) * j->S);
        if (!j->d_wphi || !j->d_a) {
            j->dfree_all();
            return fail(UQ_ENOMEM, "out of device memory for the basis table");
        }
        std::vector<double> wphi((size_t)(j->S * j->K));
        for (int64_t s = 0; s < j->S; ++s)
            for (int k = 0; k < j->K; ++k)
                wphi[(size_t)(s * j->K + k)] = j->rule.a[(size_t)s] * j->rule.phi[(size_t)(s * j->K + k)];
        UQ_HIP_TRY(hipMemcpyAsync(j->d_wphi, wphi.data(), sizeof(double) * wphi.size(), hipMemcpyHostToDevice, j->stream));
        UQ_HIP_TRY(hipMemcpyAsync(j->d_a, j->rule.a.data(), sizeof(double) * j->S, hipMemcpyHostToDevice, j->stream));
        UQ_HIP_TRY(hipStreamSynchronize(j->stream));
    }
    const int64_t zero = 0;
    UQ_HIP_TRY(hipMemcpyAsync(j->d_t, &zero, sizeof(int64_t), hipMemcpyHostToDevice, j->stream));
    UQ_HIP_TRY(hipMemcpyAsync(d_smp, smp.data(), sizeof(SampleDev) * j->S, hipMemcpyHostToDevice, j->stream));
    if (d_mask)
        UQ_HIP_TRY(hipMemcpyAsync(d_mask, mask.data(), sizeof(uint32_t) * mask.size(), hipMemcpyHostToDevice, j->stream));
    if (d_q) UQ_HIP_TRY(hipMemcpyAsync(d_q, qlink.data(), sizeof(double) * qlink.size(), hipMemcpyHostToDevice, j->stream));
    if (d_special)
        UQ_HIP_TRY(hipMemcpyAsync(d_special, special.data(), sizeof(int32_t) * special.size(), hipMemcpyHostToDevice,
                                  j->stream));
    // host vectors above go out of scope: make the copies complete first
    UQ_HIP_TRY(hipStreamSynchronize(j->stream));

    JobDev &jd = j->jd;
    std::memset(&jd, 0, sizeof jd);
    jd.f = slab;
    jd.f2 = slab2;
    jd.layout = j->shape.layout;
    jd.smp = d_smp;
    jd.mask = d_mask;
    jd.pitch = j->pitch;
    jd.plane = plane;
    jd.nx = P.nx;
    jd.ny = P.ny;
    jd.S = (int32_t)j->S;
    jd.geom = P.geometry;
    jd.xbc = P.xbc;
    jd.prec = P.precision;
    jd.scale = std::ldexp(1.0f, j->scale_exp);
    jd.inv_scale = std::ldexp(1.0f, -j->scale_exp);
    jd.ramp = (double)P.ramp;
    const double uref = P.geometry == UQ_GEOM_TGV ? P.u0 : P.u_peak;
    jd.ke_norm = uref != 0.0 ? 2.0 / ((double)P.nx * P.ny * uref * uref) : 1.0;
    jd.D = P.D;
    jd.init = P.init;
    jd.q = d_q;
    jd.dia = P.cyl_bc == UQ_CYL_BOUZIDI ? P.cyl_d : (double)P.D;
    jd.u_fac = P.force_ref == UQ_FORCE_REF_MEAN ? 2.0 / 3.0 : 1.0;
    jd.special = d_special;
    jd.n_special = (int32_t)special.size();
    j->plane_pad = (int)pad;

    UQ_HIP_TRY(launch_init(jd, j->stream));
    {
        uq_status e = j->leave();
        if (e != UQ_OK) return e;
    }
    *out = j.release();
    return UQ_OK;
}

}  // namespace uqi

using namespace uqi;

extern "C" uq_status uq_create(const uq_problem *p, const uq_device *dev, uq_job **out) {
    if (!p || !out) return fail(UQ_EINVAL, "null argument");
    return create_job(*p, dev, nullptr, out);
}

extern "C" uq_status uq_samples(const uq_job *j, double *xi, double *a, int64_t *S, int32_t *d) {
    if (!j) return fail(UQ_EINVAL, "null job");
    if (xi) std::memcpy(xi, j->rule.xi.data(), sizeof(double) * j->rule.xi.size());
    if (a) std::memcpy(a, j->rule.a.data(), sizeof(double) * j->rule.a.size());
    if (S) *S = j->S;
    if (d) *d = j->rule.d;
    return UQ_OK;
}

extern "C" uq_status uq_run(uq_job *j, int64_t steps) {
    if (!j) return fail(UQ_EINVAL, "null job");
    if (steps < 0) return fail(UQ_EINVAL, "steps must be >= 0");
    UQ_HIP_TRY(hipSetDevice(j->dev.device));
    uq_status st = j->enter();
    if (st != UQ_OK) return st;
    st = j->advance(steps);
    if (st != UQ_OK) return st;
    return j->leave();
}

extern "C" uq_status uq_run_timed(uq_job *j, int64_t steps, double *ms) {
    if (!j || !ms) return fail(UQ_EINVAL, "null argument");
    if (steps < 0) return fail(UQ_EINVAL, "steps must be >= 0");
    UQ_HIP_TRY(hipSetDevice(j->dev.device));
    uq_status st = j->enter();
    if (st != UQ_OK) return st;
    hipEvent_t a, b;
    UQ_HIP_TRY(hipEventCreate(&a));
    UQ_HIP_TRY(hipEventCreate(&b));
    UQ_HIP_TRY(hipEventRecord(a, j->stream));
    st = j->advance(steps);
    UQ_HIP_TRY(hipEventRecord(b, j->stream));
    UQ_HIP_TRY(hipEventSynchronize(b));
    float f = 0.0f;
    UQ_HIP_TRY(hipEventElapsedTime(&f, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *ms = (double)f;
    if (st != UQ_OK) return st;
    return j->leave();
}

extern "C" uq_status uq_sync(uq_job *j) {
    if (!j) return fail(UQ_EINVAL, "null job");
    UQ_HIP_TRY(hipSetDevice(j->dev.device));
    UQ_HIP_TRY(hipStreamSynchronize(j->stream));
    UQ_HIP_TRY(hipStreamSynchronize(j->user_stream));
    return UQ_OK;
}

namespace uqi {

// Per-sample scalar QoIs into b.qoi, and UQ_EUNSTABLE if any sample holds a
// non-finite value. Blocking (one flag read).
uq_status Job::check_finite(const StatBufs &b) {
    UQ_HIP_TRY(launch_qoi_scalars(jd, t, b.qoi, stream));
    UQ_HIP_TRY(launch_first_bad(b.qoi, S, b.flag, stream));
    int64_t bad = S;
    UQ_HIP_TRY(hipMemcpyAsync(&bad, b.flag, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    UQ_HIP_TRY(hipStreamSynchronize(stream));
    if (bad < S)
        return fail(UQ_EUNSTABLE, "sample " + std::to_string(bad) + " holds a non-finite value at step " + std::to_string(t));
    return UQ_OK;
}

// Per-sample values of one QoI in the buffers b. Returns the device pointer,
// number of values per sample and the row stride. Blocking (one flag read).
uq_status Job::sample_values_in(const StatBufs &b, int qoi, const double **M, int64_t *n_out, int64_t *ld) {
    const uq_problem &P = p;
    const int64_t cells = (int64_t)P.nx * P.ny;
    if (qoi_width(P, qoi) == 0) return fail(UQ_EINVAL, "unknown QoI");
    if ((qoi == UQ_QOI_CD || qoi == UQ_QOI_CL) && (P.geometry != UQ_GEOM_CHANNEL || (P.D <= 0 && P.cyl_bc != UQ_CYL_BOUZIDI)))
        return fail(UQ_EINVAL, "drag/lift need a channel with a cylinder");
    uq_status st = check_finite(b);
    if (st != UQ_OK) return st;
    if (qoi_width(P, qoi) == 1) {
        UQ_HIP_TRY(launch_select_scalar(jd, b.qoi, qoi, b.M, stream));
        *M = b.M;
        *n_out = 1;
        *ld = 1;
        return UQ_OK;
    }
    UQ_HIP_TRY(launch_fields(jd, t, b.fields, stream));
    *M = qoi == UQ_QOI_VEL ? b.fields : b.fields + (qoi == UQ_QOI_RHO ? 2 : 3) * cells;
    *n_out = qoi_width(P, qoi);
    *ld = 4 * cells;
    return UQ_OK;
}

uq_status Job::sample_values(int qoi, const double **M, int64_t *n_out, int64_t *ld) {
    if (qoi_width(p, qoi) == 0) return fail(UQ_EINVAL, "unknown QoI");
    StatBufs b;
    uq_status st = own_stat_bufs(qoi, true, &b);
    if (st != UQ_OK) return st;
    return sample_values_in(b, qoi, M, n_out, ld);
}

// Scalar QoIs: per-sample values, then the sums over samples spread across a
// workgroup. Field QoIs: after the per-sample non-finite check, straight
// from the populations (no per-sample field buffer: b.fields is not used).
uq_status Job::moments_in(const StatBufs &b, int qoi, uq_moments_out *out) {
    const int64_t n = qoi_width(p, qoi);
    uq_status st = enter();
    if (st != UQ_OK) return st;
    double *d_mean = b.out, *d_var = b.out + n, *d_alt = b.out + 2 * n, *d_coef = b.out + 3 * n;
    if (n == 1) {
        const double *M;
        int64_t n1, ld;
        st = sample_values_in(b, qoi, &M, &n1, &ld);
        if (st != UQ_OK) return st;
        UQ_HIP_TRY(launch_scalar_moments(M, S, d_wphi, d_a, K, d_coef, d_mean, d_var, d_alt, stream));
    } else {
        StatBufs scalars = b;
        scalars.fields = nullptr;
        st = check_finite(scalars);
        if (st != UQ_OK) return st;
        UQ_HIP_TRY(launch_field_moments(jd, t, qoi, d_wphi, d_a, K, d_coef, d_mean, d_var, d_alt, stream));
    }
    out->n_out = n;
    out->K = K;
    out->d = rule.d;
    if (out->mean) UQ_HIP_TRY(hipMemcpyAsync(out->mean, d_mean, sizeof(double) * n, hipMemcpyDeviceToHost, stream));
    if (out->var) UQ_HIP_TRY(hipMemcpyAsync(out->var, d_var, sizeof(double) * n, hipMemcpyDeviceToHost, stream));
    if (out->var_alt) UQ_HIP_TRY(hipMemcpyAsync(out->var_alt, d_alt, sizeof(double) * n, hipMemcpyDeviceToHost, stream));
    if (out->coeffs && K > 0)
        UQ_HIP_TRY(hipMemcpyAsync(out->coeffs, d_coef, sizeof(double) * n * K, hipMemcpyDeviceToHost, stream));
    UQ_HIP_TRY(hipStreamSynchronize(stream));
    if (out->alpha && K > 0) std::memcpy(out->alpha, rule.alpha.data(), sizeof(int32_t) * rule.alpha.size());
    return UQ_OK;
}

}  // namespace uqi

extern "C" uq_status uq_qoi_samples(uq_job *j, int32_t qoi, double *out, int64_t *n_out) {
    if (!j) return fail(UQ_EINVAL, "null job");
    UQ_HIP_TRY(hipSetDevice(j->dev.device));
    int64_t n = qoi_width(j->p, qoi);
    if (n == 0) return fail(UQ_EINVAL, "unknown QoI");
    if (n_out) *n_out = n;
    if (!out) return UQ_OK;
    const double *M;
    int64_t ld;
    uq_status st = j->enter();
    if (st != UQ_OK) return st;
    st = j->sample_values(qoi, &M, &n, &ld);
    if (st != UQ_OK) return st;
    UQ_HIP_TRY(hipMemcpy2DAsync(out, sizeof(double) * n, M, sizeof(double) * ld, sizeof(double) * n, (size_t)j->S,
                                hipMemcpyDeviceToHost, j->stream));
    UQ_HIP_TRY(hipStreamSynchronize(j->stream));
    return UQ_OK;
}

extern "C" uq_status uq_moments(uq_job *j, int32_t qoi, uq_moments_out *out) {
    if (!j || !out) return fail(UQ_EINVAL, "null argument");
    UQ_HIP_TRY(hipSetDevice(j->dev.device));
    if (qoi_width(j->p, qoi) == 0) return fail(UQ_EINVAL, "unknown QoI");
    StatBufs b;
    uq_status st = j->own_stat_bufs(qoi, false, &b);
    if (st != UQ_OK) return st;
    return j->moments_in(b, qoi, out);
}

extern "C" uq_status uq_populations(uq_job *j, int64_t sample, double *out) {
    if (!j || !out) return fail(UQ_EINVAL, "null argument");
    if (sample < 0 || sample >= j->S) return fail(UQ_EINVAL, "sample out of range");
    UQ_HIP_TRY(hipSetDevice(j->dev.device));
    const int64_t cells = (int64_t)j->p.nx * j->p.ny;
    if (!j->d_export) {
        j->d_export = (double *)j->dalloc(sizeof(double) * 9 * cells);
        if (!j->d_export) return fail(UQ_ENOMEM, "out of device memory");
    }
    uq_status st = j->enter();
    if (st != UQ_OK) return st;
    UQ_HIP_TRY(launch_export(j->jd, j->t, sample, j->d_export, j->stream));
    UQ_HIP_TRY(hipMemcpyAsync(out, j->d_export, sizeof(double) * 9 * cells, hipMemcpyDeviceToHost, j->stream));
    UQ_HIP_TRY(hipStreamSynchronize(j->stream));
    return UQ_OK;
}

extern "C" uq_status uq_job_get_info(const uq_job *j, uq_job_info *info) {
    if (!j || !info) return fail(UQ_EINVAL, "null argument");
    info->S = j->S;
    info->d = j->rule.d;
    info->K = j->K;
    info->steps_done = j->t;
    info->pitch = j->pitch;
    info->device_bytes = j->bytes_held;
    info->scale_exp = j->scale_exp;
    info->fluid_nodes = j->fluid;
    info->layout = j->shape.layout;
    info->cpt = j->shape.cpt;
    info->nt_store = j->shape.nt;
    info->plane_pad = j->plane_pad;
    info->bx = j->shape.bx;
    info->fused = j->fused_n();
    info->fused_rows = info->fused ? j->shape.fty : 0;
    info->fused_window = info->fused ? j->shape.fwin : 0;
    info->step_launches = j->launches;
    return UQ_OK;
}

extern "C" void uq_destroy(uq_job *j) {
    if (!j) return;
    (void)hipSetDevice(j->dev.device);
    delete j;  // waits for the job stream, then releases graph, buffers, stream
}
