// HIP kernels (gfx950) of the batched D2Q9 BGK ensemble and its
// statistics: OpenLB-UQ (arXiv 2508.13867), Sec. "Lattice Boltzmann
// methods" (Eqs. deterministicLBE, bgkCollision, equilibrium, the D2Q9 set
// and weights, the collide/stream split) and Sec. "Uncertainty
// quantification methods" (Eqs. meanMCS, varMCS, coef_discrete, gpc_mean,
// gpc_std).
//
// Storage: shifted populations f~_i = f_i - w_i in slabs [S][9][ny][pitch]
// (x fastest, pitch a multiple of 64 elements). Two layouts:
//
// AA (one slab, in place; Bailey et al. 2009):
//   even step t: node x reads its own slots i, collides, and writes f*_i to
//                its own slot opp(i);
//   odd step t:  node x reads f_i(x,t) = f*_i(x - c_i, t-1) from slot opp(i)
//                of node x - c_i, collides, and writes f*_i to slot i of
//                node x + c_i, leaving the natural layout for step t+1.
//   Each node reads and writes exactly the same nine locations in either
//   parity, so one launch per step needs no second lattice and no barrier.
//
// AB (two slabs, pull): slab t&1 holds g_i(x) = f*_i(x, t-1), the
//   post-collision populations of the previous step; step t reads
//   f_i(x,t) = g_i(x - c_i) (bounce-back: g_opp(i)(x)), collides and writes
//   f*_i(x,t) to slot i of node x in the other slab: every store is aligned
//   and can bypass the caches. Twice the memory of AA; on MI355X a
//   two-buffer stream reaches a higher HBM rate than an in-place one.
//
// Direction order i = 0..8: (0,0), (1,0), (0,1), (-1,0), (0,-1), (1,1),
// (-1,1), (-1,-1), (1,-1); opposite pairs (1,3), (2,4), (5,7), (6,8).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "uq_internal.h"

// Every fused multiply-add in these kernels is written out (fma_c). Implicit
// contraction is off so that the compiler cannot fuse the last fma of the
// collision with the conversion to a 16-bit storage format (one rounding
// where the storage model has two), which it would do in some kernels and
// not in others: with it off, every kernel rounds the same operations the
// same way and their results agree bit for bit in every format.
#pragma clang fp contract(off)

namespace uqi {

// ------------------------------------------------------------------ storage types
template <int P>
struct Prec;

template <>
struct Prec<UQ_FP64> {
    using T = double;
    using C = double;
    __device__ static inline C ld(const T *p, float) { return *p; }
    __device__ static inline void st(T *p, C v, float) { *p = v; }
    __device__ static inline void st_nt(T *p, C v, float) { __builtin_nontemporal_store(v, p); }
    // the value a store and a reload would give back
    __device__ static inline C rt(C v, float, float) { return v; }
};
template <>
struct Prec<UQ_FP32> {
    using T = float;
    using C = float;
    __device__ static inline C ld(const T *p, float) { return *p; }
    __device__ static inline void st(T *p, C v, float) { *p = v; }
    __device__ static inline void st_nt(T *p, C v, float) { __builtin_nontemporal_store(v, p); }
    __device__ static inline C rt(C v, float, float) { return v; }
};
template <>
struct Prec<UQ_FP16S> {
    using T = _Float16;
    using C = float;
    // stored value = f~ * 2^s (power-of-two scale, exact); rounding to half is
    // round-to-nearest-even (v_cvt_f16_f32 in the default mode). Back to
    // float as h * 2^-s + 0: one mixed-precision fma (v_fma_mix_f32) where a
    // product would take a conversion and a multiply; the same value, except
    // that -0 comes back as +0.
    __device__ static inline C up(_Float16 h, float inv) { return __builtin_fmaf((float)h, inv, 0.0f); }
    __device__ static inline C ld(const T *p, float inv) { return up(*p, inv); }
    __device__ static inline void st(T *p, C v, float sc) { *p = (_Float16)(v * sc); }
    __device__ static inline void st_nt(T *p, C v, float sc) { __builtin_nontemporal_store((_Float16)(v * sc), p); }
    __device__ static inline C rt(C v, float sc, float inv) { return up((_Float16)(v * sc), inv); }
};
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
template <>
struct Prec<UQ_BF16S> {
    // bfloat16 has float's exponent range: stored unscaled (the job's scale
    // exponent is 0 and sc, inv are not used)
    using T = uint16_t;
    using C = float;
    __device__ static inline C ld(const T *p, float) { return __uint_as_float((uint32_t)(*p) << 16); }
    // round to nearest, ties to even (the conversion instruction of gfx950)
    __device__ static inline uint16_t rne(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
    __device__ static inline void st(T *p, C v, float) { *p = rne(v); }
    __device__ static inline void st_nt(T *p, C v, float) { __builtin_nontemporal_store(rne(v), p); }
    // the rounded value in the upper half of a word whose lower half is +0:
    // that word is the float itself, from one conversion instruction
    __device__ static inline C rt(C v, float, float) {
        return __builtin_bit_cast(float, __builtin_convertvector((f32x2_t){0.0f, v}, bf16x2_t));
    }
};

// ------------------------------------------------------------------ lattice
__device__ constexpr int CXd[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int CYd[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int OPPd[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
// index of a direction among the three that share its c_y
__device__ constexpr int GJd[9] = {0, 1, 0, 2, 0, 1, 2, 1, 2};

template <typename C>
__device__ inline C wgt(int i) {
    return i == 0 ? C(4) / C(9) : (i < 5 ? C(1) / C(9) : C(1) / C(36));
}

// BGK relaxation of shifted populations toward the second-order equilibrium
// (Eqs. bgkCollision, equilibrium with c_s^2 = 1/3). With j = rho u, the
// equilibrium minus the weight is
//   f_eq,i - w_i = w_i (drho - 3/2 j.u + 9/2 (c_i.j)(c_i.u)) + 3 w_i (c_i.j),
// which equals the textbook form in exact arithmetic. It is evaluated this way
// so that single-precision rounding does not bias the flow:
//  - the first-order term uses j itself, not rho * (j / rho);
//  - the first-order term omega 3 w_i (c_i.j) is one rounded product per
//    direction pair, a1 (c_i.j) on the axes and a2 (c_i.j) on the diagonals,
//    with coefficients whose momentum sum 2 a1 + 4 a2 is omega exactly, so
//    that the collision conserves momentum to rounding. In double precision
//    a1 = omega/3 is carried as a two-term split (hi + lo, one fused
//    multiply-add per term) and a2 = a1/4. In single precision a1 =
//    fl(omega fl(1/3)) and a2 = (omega - 2 a1)/4, whose subtraction is exact
//    (Sterbenz: omega and 2 a1 are within a factor of two), one multiply per
//    term; a2 then differs from omega/12 by O(1e-7), which touches only a
//    third moment of the equilibrium (Q_xyy), not mass, momentum or stress.
//    Multiplying both by a rounded omega/3 instead scales these terms by a
//    fixed 1 + O(1e-8) every step: the collision then does not conserve
//    momentum, and in single precision the decay of the kinetic energy
//    drifts by ~1e-5..1e-4 over a few thousand steps (measured), against
//    ~1e-7 in this form.
// Returns rho - 1 and u.
template <typename C>
struct Third;
template <>
struct Third<float> {
    static constexpr float hi = 0x1.555556p-2f, lo = -0x1.555556p-27f;  // hi + lo = 1/3 to ~2^-48
};
template <>
struct Third<double> {
    static constexpr double hi = 0x1.5555555555555p-2, lo = 0x1.5555555555555p-56;
};
__device__ inline float fma_c(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fma_c(double a, double b, double c) { return __builtin_fma(a, b, c); }
// 1/x from the hardware reciprocal estimate refined by Newton steps (one in
// single, two in double precision): within an ulp of the quotient, a third of
// the instructions of the IEEE division sequence
__device__ inline float recip(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
}
__device__ inline double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

// 1/(1 + drho) inside the collision. The velocity it gives enters only the
// second-order terms of the equilibrium (the first-order term uses j), so
// in single precision the hardware estimate (within an ulp) is used as it
// is; double precision refines it to full accuracy.
__device__ inline float coll_recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double coll_recip(double x) { return recip(x); }

template <typename C>
__device__ inline void bgk(C f[9], C omega, C &drho_o, C &ux_o, C &uy_o) {
    // moments from the sums of the c_y = +1 and c_y = -1 populations (j_y is
    // their difference), with the c_y = -1 terms last: the fused kernels
    // read the others a row ahead, so most of this runs while those loads
    // are in flight
    const C cs = f[2] + (f[5] + f[6]), as = f[4] + (f[7] + f[8]);
    const C drho = ((f[0] + (f[1] + f[3])) + cs) + as;
    const C jx = ((f[1] - f[3]) + (f[5] - f[6])) + (f[8] - f[7]);
    const C jy = cs - as;
    const C ir = coll_recip(C(1) + drho);
    const C ux = jx * ir, uy = jy * ir;
    // second-order terms from the products j_x u_x, j_y u_y and j_x u_y
    // (= j_y u_x): (c.j)(c.u) is j_x u_x or j_y u_y on the axes and
    // j_x u_x + j_y u_y +- 2 j_x u_y on the diagonals
    const C px = jx * ux, py = jy * uy, pp = px + py;
    const C db = fma_c(C(-1.5), pp, drho);
    // omega folded into the constants (per sample: the compiler hoists them
    // out of the node loops): omega w_i, and omega / 3 as an unevaluated sum
    // hi + lo (exact product of omega with the split of 1/3, rounded once to
    // the pair; unused in single precision), so that the first-order term is
    // still formed with a single rounding. Every multiply-add is an explicit
    // fma.
    const C ow0 = omega * (C(4) / C(9)), ow1 = omega * (C(1) / C(9)), ow2 = omega * (C(1) / C(36));
    const C o3h = omega * Third<C>::hi;
    const C o3l = fma_c(omega, Third<C>::lo, fma_c(omega, Third<C>::hi, -o3h));
    // diagonal coefficient: in single precision the exact remainder of omega
    // after the two axis terms, so that 2 o3h + 4 o12h = omega
    const C o12h = std::is_same<C, float>::value ? (omega - C(2) * o3h) * C(0.25) : o3h * C(0.25);
    const C o12l = o3l * C(0.25);
    // the first-order term, rounded once (single precision: one multiply)
    auto first = [&](C cj, C h, C l) -> C {
        if constexpr (std::is_same<C, float>::value) return cj * h;
        else return fma_c(cj, h, cj * l);
    };
    const C om1 = C(1) - omega;
    f[0] = fma_c(om1, f[0], ow0 * db);
    {
        const C q = fma_c(C(4.5), px, db), l = first(jx, o3h, o3l);
        f[1] = fma_c(om1, f[1], fma_c(q, ow1, l));
        f[3] = fma_c(om1, f[3], fma_c(q, ow1, -l));
    }
    {
        const C q = fma_c(C(4.5), py, db), l = first(jy, o3h, o3l);
        f[2] = fma_c(om1, f[2], fma_c(q, ow1, l));
        f[4] = fma_c(om1, f[4], fma_c(q, ow1, -l));
    }
    const C t = fma_c(C(4.5), pp, db), jx9 = C(9) * jx;
    {
        const C cj = jx + jy;
        const C q = fma_c(jx9, uy, t), l = first(cj, o12h, o12l);
        f[5] = fma_c(om1, f[5], fma_c(q, ow2, l));
        f[7] = fma_c(om1, f[7], fma_c(q, ow2, -l));
    }
    {
        const C cj = jy - jx;
        const C q = fma_c(-jx9, uy, t), l = first(cj, o12h, o12l);
        f[6] = fma_c(om1, f[6], fma_c(q, ow2, l));
        f[8] = fma_c(om1, f[8], fma_c(q, ow2, -l));
    }
    drho_o = drho;
    ux_o = ux;
    uy_o = uy;
}

// moments only
template <typename C>
__device__ inline void moments(const C f[9], C &drho, C &ux, C &uy) {
    drho = ((f[0] + (f[1] + f[3])) + (f[2] + f[4])) + ((f[5] + f[7]) + (f[6] + f[8]));
    const C jx = ((f[1] - f[3]) + (f[5] - f[7])) + (f[8] - f[6]);
    const C jy = ((f[2] - f[4]) + (f[5] - f[7])) + (f[6] - f[8]);
    const C ir = recip(C(1) + drho);
    ux = jx * ir;
    uy = jy * ir;
}

// inflow ramp s(t) = sin^2(pi t / (2 T_r)) for t < T_r, else 1
__device__ inline double ramp_factor(int64_t t, double T) {
    if (T <= 0.0 || (double)t >= T) return 1.0;
    double s = sin(M_PI * (double)t / (2.0 * T));
    return s * s;
}

// inflow profile u_x at row y, time t: s(t) 4 u_peak (y+1/2)(H-y-1/2)/H^2,
// from a = s(t) 4 u_peak
__device__ inline double inflow_u_a(double a, int ny, int y) {
    // 1/H^2 depends on the lattice only: the compiler hoists its division
    // out of the row loops, leaving three multiplies per row
    const double H = (double)ny, yy = (double)y + 0.5, inv_h2 = 1.0 / (H * H);
    return a * yy * (H - yy) * inv_h2;
}
__device__ inline double inflow_u(int ny, double ramp, int y, int64_t t, double u_peak) {
    return inflow_u_a(ramp_factor(t, ramp) * 4.0 * u_peak, ny, y);
}

// Zou-He (1997) completion of the unknown populations on the open columns,
// written for shifted populations (the weights cancel in every relation):
// the inlet with the imposed velocity u, the outlet at rho = 1.
// (explicit fmas, as in the collision: the same result in every kernel)
template <typename C>
__device__ inline void zou_he_u(C f[9], bool inlet, C u) {
    const C h = C(0.5) * (f[2] - f[4]);
    if (inlet) {
        const C S = fma_c(C(2), (f[3] + f[6]) + f[7], (f[0] + f[2]) + f[4]);
        const C drho = (S + u) / (C(1) - u);
        const C ru = (C(1) + drho) * u;
        f[1] = fma_c(C(2) / C(3), ru, f[3]);
        f[5] = fma_c(C(1) / C(6), ru, f[7] - h);
        f[8] = fma_c(C(1) / C(6), ru, f[6] + h);
    } else {
        const C v = fma_c(C(2), (f[1] + f[5]) + f[8], (f[0] + f[2]) + f[4]);
        f[3] = fma_c(-(C(2) / C(3)), v, f[1]);
        f[7] = fma_c(-(C(1) / C(6)), v, f[5] + h);
        f[6] = fma_c(-(C(1) / C(6)), v, f[8] - h);
    }
}

template <typename C>
__device__ inline void zou_he(C f[9], const JobDev &j, int x, int y, int64_t t, double u_peak) {
    zou_he_u(f, x == 0, x == 0 ? (C)inflow_u(j.ny, j.ramp, y, t, u_peak) : C(0));
}

// Addressing inside one sample's slab.
struct Site {
    int x, y, xm, xp, ym, yp;
};

__device__ inline Site site(const JobDev &j, int x, int y) {
    Site s;
    s.x = x;
    s.y = y;
    s.xm = x == 0 ? j.nx - 1 : x - 1;
    s.xp = x == j.nx - 1 ? 0 : x + 1;
    s.ym = y == 0 ? j.ny - 1 : y - 1;
    s.yp = y == j.ny - 1 ? 0 : y + 1;
    return s;
}

__device__ inline int sx_of(const Site &s, int dx) { return dx == 0 ? s.x : (dx > 0 ? s.xp : s.xm); }
__device__ inline int sy_of(const Site &s, int dy) { return dy == 0 ? s.y : (dy > 0 ? s.yp : s.ym); }

// Access modes of a step / QoI read.
enum : int { AA_EVEN = 0, AA_ODD = 1, AB_PULL = 2 };

template <int LAYOUT, int PARITY>
struct ModeOf {
    static constexpr int value = LAYOUT == UQ_LAYOUT_AB ? AB_PULL : (PARITY ? AA_ODD : AA_EVEN);
};

// Interpolated bounce-back (Bouzidi, Firdaouss & Lallemand 2001) for pull
// direction i of a node whose link x -> x - c_i meets the cylinder at
// fraction q; AB layout, where the source slab holds every node's f* of the
// previous step. With k = opp(i):
//   q <  1/2: f_i(x) = 2q f*_k(x) + (1 - 2q) f*_k(x + c_i)
//   q >= 1/2: f_i(x) = f*_k(x)/(2q) + (1 - 1/(2q)) f*_i(x)
// (x + c_i is fluid: the circle keeps clear of the walls, and by convexity
// the node behind a fluid node on a link into the circle is outside it). The
// weights of the shifted populations cancel (the coefficients sum to 1).
template <int P>
__device__ inline typename Prec<P>::C wall_return(const JobDev &j, const typename Prec<P>::T *base, const Site &s,
                                                  int64_t own, int i) {
    using PR = Prec<P>;
    using C = typename PR::C;
    const int k = OPPd[i];
    const C fk = PR::ld(base + k * j.plane + own, j.inv_scale);
    const double q = j.q[(int64_t)i * j.ny * j.pitch + own];
    if (!(q > 0.0)) return fk;  // a half-way link (channel wall)
    if (q >= 0.5) {
        const C fi = PR::ld(base + i * j.plane + own, j.inv_scale);
        const double a = 1.0 / (2.0 * q);
        return (C)a * fk + (C)(1.0 - a) * fi;
    }
    const int xb = sx_of(s, CXd[i]), yb = sy_of(s, CYd[i]);
    const C fb = PR::ld(base + k * j.plane + (int64_t)yb * j.pitch + xb, j.inv_scale);
    return (C)(2.0 * q) * fk + (C)(1.0 - 2.0 * q) * fb;
}

template <int P, bool CHANNEL, int MODE, bool FD = true, bool QL = true>
__device__ inline void gather(const JobDev &j, const typename Prec<P>::T *base, const Site &s, uint32_t m,
                              int64_t t, double u_peak, double omega, typename Prec<P>::C f[9]);

__device__ inline double inlet_ux(const JobDev &j, int y, int64_t t, double u_peak) {
    return inflow_u(j.ny, j.ramp, y, t, u_peak);
}

// velocity of an outlet-column node from its known populations (rho = 1)
template <int P>
__device__ inline double outlet_ux(const JobDev &j, const typename Prec<P>::T *base, int x, int y, int64_t t,
                                   double u_peak, double omega) {
    typename Prec<P>::C g[9];
    gather<P, true, AB_PULL, false>(j, base, site(j, x, y), j.mask[(int64_t)y * j.pitch + x], t, u_peak, omega, g);
    return (double)((g[0] + g[2] + g[4]) + (g[1] + g[5] + g[8]) + (g[1] + g[5] + g[8]));
}

// velocity of an interior node from its streamed populations
template <int P>
__device__ inline void node_u(const JobDev &j, const typename Prec<P>::T *base, int x, int y, int64_t t,
                              double u_peak, double omega, double &ux, double &uy) {
    using C = typename Prec<P>::C;
    C g[9], drho, gx, gy;
    gather<P, true, AB_PULL, false>(j, base, site(j, x, y), j.mask[(int64_t)y * j.pitch + x], t, u_peak, omega, g);
    moments(g, drho, gx, gy);
    ux = (double)gx;
    uy = (double)gy;
}

// Finite-difference reconstruction of an open-column node (the paper's
// interpolated inlet / outlet after Latt et al. 2008): f_i = f_i^eq(rho, u)
// + f_i^neq, f_i^neq = -3 w_i rho tau Q_i : grad u, Q_i = c_i c_i - I/3.
// grad u: across the column the one-sided second-order difference
// (-3 u_0 + 4 u_1 - u_2)/2 into the fluid; along it the central difference,
// one-sided at the two end rows. Inlet: u prescribed, rho from the known
// populations; outlet: rho = 1, u_y = 0, u_x from the known populations.

// imposed state of an open-column node from its streamed populations
// (unknown ones unset)
template <typename C>
__device__ inline void fd_state(const JobDev &j, const C f[9], bool inlet, int y, int64_t t, double u_peak,
                                double &rho, double &ux) {
    if (inlet) {
        ux = inlet_ux(j, y, t, u_peak);
        const double S = (double)((f[0] + f[2] + f[4]) + (f[3] + f[6] + f[7]) + (f[3] + f[6] + f[7]));
        rho = 1.0 + (S + ux) / (1.0 - ux);
    } else {
        rho = 1.0;
        ux = (double)((f[0] + f[2] + f[4]) + (f[1] + f[5] + f[8]) + (f[1] + f[5] + f[8]));
    }
}

// d(u_x)/dy along the column from the column values at y-2 .. y+2
// (um2, um1, u0, up1, up2; only those inside the column are read)
__device__ inline double fd_dy(int y, int ny, double um2, double um1, double u0, double up1, double up2) {
    if (y == 0) return (-3.0 * u0 + 4.0 * up1 - up2) * 0.5;
    if (y == ny - 1) return (3.0 * u0 - 4.0 * um1 + um2) * 0.5;
    return (up1 - um1) * 0.5;
}

// f = f^eq + f^neq from the imposed state and the gradient (u_y = 0)
template <typename C>
__device__ inline void fd_rebuild(C f[9], double rho, double ux, double dxux, double dxuy, double dyux, double omega) {
    const double uy = 0.0, dyuy = 0.0;
    const double tau = 1.0 / omega, drho = rho - 1.0, uu = ux * ux + uy * uy;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double cx = CXd[i], cy = CYd[i], w = wgt<double>(i);
        const double cu = cx * ux + cy * uy;
        const double QS = (cx * cx - 1.0 / 3.0) * dxux + (cy * cy - 1.0 / 3.0) * dyuy + cx * cy * (dxuy + dyux);
        f[i] = (C)(w * (drho + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu)) - 3.0 * w * rho * tau * QS);
    }
}

// the whole reconstruction for one node, neighbours gathered here (QoI and
// export kernels; the step uses k_fd_columns, which shares them in LDS)
template <int P>
__device__ inline void fd_column(const JobDev &j, const typename Prec<P>::T *base, const Site &s, int64_t t,
                                 double u_peak, double omega, typename Prec<P>::C f[9]) {
    const int x = s.x, y = s.y, ny = j.ny;
    const bool inlet = x == 0;
    const int sd = inlet ? 1 : -1;
    double rho, ux;
    fd_state(j, f, inlet, y, t, u_peak, rho, ux);
    double u1x, u1y, u2x, u2y;
    node_u<P>(j, base, x + sd, y, t, u_peak, omega, u1x, u1y);
    node_u<P>(j, base, x + 2 * sd, y, t, u_peak, omega, u2x, u2y);
    const double dxux = sd * (-3.0 * ux + 4.0 * u1x - u2x) * 0.5;
    const double dxuy = sd * (-3.0 * 0.0 + 4.0 * u1y - u2y) * 0.5;
    auto col_ux = [&](int yy) {
        return inlet ? inlet_ux(j, yy, t, u_peak) : outlet_ux<P>(j, base, x, yy, t, u_peak, omega);
    };
    double dyux;
    if (y == 0)
        dyux = fd_dy(y, ny, 0.0, 0.0, ux, col_ux(1), col_ux(2));
    else if (y == ny - 1)
        dyux = fd_dy(y, ny, col_ux(ny - 3), col_ux(ny - 2), ux, 0.0, 0.0);
    else
        dyux = fd_dy(y, ny, 0.0, col_ux(y - 1), ux, col_ux(y + 1), 0.0);
    fd_rebuild(f, rho, ux, dxux, dxuy, dyux, omega);
}

// Gather f~(x, t) of one node, with the wall rules and the open columns
// (FD = false leaves the open-column populations of a finite-difference job
// unset: the reconstruction reads its neighbours that way; QL = false omits
// the interpolated links: the bulk step kernel never meets those nodes).
template <int P, bool CHANNEL, int MODE, bool FD, bool QL>
__device__ inline void gather(const JobDev &j, const typename Prec<P>::T *base, const Site &s, uint32_t m,
                              int64_t t, double u_peak, double omega, typename Prec<P>::C f[9]) {
    using PR = Prec<P>;
    using C = typename PR::C;
    const float inv = j.inv_scale;
    const int64_t pitch = j.pitch, plane = j.plane;
    const int64_t own = (int64_t)s.y * pitch + s.x;
    // Every direction issues its one load unconditionally, the wall rule only
    // selecting the address: with no branches between them all nine loads
    // are in flight together (per-direction branches made the compiler wait
    // for each load at the block boundaries).
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if (MODE == AA_EVEN) {
            f[i] = PR::ld(base + i * plane + own, inv);
            continue;
        }
        // pull: f_i(x,t) = f*_i(x - c_i, t-1) (AA odd: slot opp(i) there;
        // AB: slot i); bounce-back: f*_opp(i)(x, t-1) at this node (AA odd:
        // slot i; AB: slot opp(i))
        const int xs = sx_of(s, -CXd[i]), ys = sy_of(s, -CYd[i]);
        int64_t off = (int64_t)(MODE == AA_ODD ? OPPd[i] : i) * plane + (int64_t)ys * pitch + xs;
        bool bb = false;
        if (CHANNEL) {
            bb = (m >> (M_BB + i)) & 1u;
            const int64_t off_bb = (int64_t)(MODE == AA_ODD ? i : OPPd[i]) * plane + own;
            off = bb ? off_bb : off;
        }
        C v = PR::ld(base + off, inv);
        if (CHANNEL) {
            // interpolated links (AB only) combine it with a second value
            if (MODE == AB_PULL && QL && bb && (m & M_QLINK)) v = wall_return<P>(j, base, s, own, i);
            // beyond an open column: rest state at t = 0, else filled below
            // (the wrapped pull address is in bounds; its value is unused)
            v = ((m >> (M_OPEN + i)) & 1u) ? C(0) : v;
        }
        f[i] = v;
    }
    if (CHANNEL && (m & (0x1FFu << M_OPEN)) && t > 0) {
        if (j.xbc != UQ_XBC_INTERP)
            zou_he(f, j, s.x, s.y, t, u_peak);
        else if (MODE == AB_PULL && FD)
            fd_column<P>(j, base, s, t, u_peak, omega, f);
    }
}

// Scatter post-collision f*(x, t) to where step t+1 reads it.
template <int P, bool CHANNEL, int MODE, bool NT>
__device__ inline void scatter(const JobDev &j, typename Prec<P>::T *base, const Site &s, uint32_t m,
                               const typename Prec<P>::C f[9]) {
    using PR = Prec<P>;
    const float sc = j.scale;
    const int64_t pitch = j.pitch, plane = j.plane;
    const int64_t own = (int64_t)s.y * pitch + s.x;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        if (MODE == AB_PULL) {
            if (NT)
                PR::st_nt(base + i * plane + own, f[i], sc);
            else
                PR::st(base + i * plane + own, f[i], sc);
        } else if (MODE == AA_EVEN) {
            PR::st(base + OPPd[i] * plane + own, f[i], sc);
        } else {
            // AA odd: f*_i goes to slot i of x + c_i; if that is a wall it
            // returns to this node as f_opp(i) (slot opp(i) here). A value
            // leaving through an open column is parked in that same own slot,
            // which nothing else writes and the next gather overrides (no
            // branch: the stores stay back to back).
            const int o = OPPd[i];
            const int xd = sx_of(s, CXd[i]), yd = sy_of(s, CYd[i]);
            int64_t off = (int64_t)i * plane + (int64_t)yd * pitch + xd;
            if (CHANNEL) {
                const bool back = ((m >> (M_BB + o)) | (m >> (M_OPEN + o))) & 1u;
                off = back ? (int64_t)o * plane + own : off;
            }
            PR::st(base + off, f[i], sc);
        }
    }
}

// Slab holding the state at step t (AA: the only one; AB: slab t & 1).
template <int LAYOUT>
__device__ inline void *state_slab(const JobDev &j, int64_t t) {
    return (LAYOUT == UQ_LAYOUT_AB && (t & 1)) ? j.f2 : j.f;
}

// ------------------------------------------------------------------ tile walk
// Blocks are dealt round-robin to the 8 XCDs; renumber them so that each XCD
// gets a contiguous run of tiles (neighbouring rows share its L2).
__device__ inline int64_t xcd_logical(int64_t b, int64_t G) {
    const int64_t xcd = b & 7, k = b >> 3;
    const int64_t q = G >> 3, r = G & 7;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

constexpr int BX = 64;  // default workgroup shape: 64 nodes along x (one
constexpr int BY = 4;   // wavefront) by 4 rows; the step kernel takes any
                        // 256-thread shape bx x (256/bx) from its launch

// One tile of one sample: blockDim.x nodes along x by blockDim.y*CPT rows;
// each thread takes CPT rows blockDim.y apart. All CPT nodes of a thread are gathered before any is
// written back: in the AA pattern a node reads and writes only its own nine
// locations (and in AB reads and writes different slabs), so the nodes are
// independent and the loads of all CPT rows can be in flight together.
template <int P, bool CHANNEL, int PARITY, int CPT, int LAYOUT, bool NT>
__device__ inline void tile_update(const JobDev &j, int64_t t, int64_t smp, int tx, int ty) {
    using PR = Prec<P>;
    using C = typename PR::C;
    using T = typename PR::T;
    constexpr int MODE = ModeOf<LAYOUT, PARITY>::value;
    const int x = tx * (int)blockDim.x + threadIdx.x;
    if (x >= j.nx) return;
    T *src_all = (T *)(LAYOUT == UQ_LAYOUT_AB && PARITY ? j.f2 : j.f);
    T *dst_all = (T *)(LAYOUT == UQ_LAYOUT_AB && !PARITY ? j.f2 : j.f);
    const double omega_d = j.smp[smp].omega;
    const C omega = (C)omega_d;
    const double u_peak = CHANNEL ? j.smp[smp].u_peak : 0.0;
    const T *src = src_all + smp * 9 * j.plane;
    T *dst = dst_all + smp * 9 * j.plane;
    const int by = (int)blockDim.y;
    const int y0 = ty * by * CPT + threadIdx.y;
    C f[CPT][9];
    uint32_t m[CPT];
    bool live[CPT];
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
        const int y = y0 + r * by;
        live[r] = y < j.ny;
        m[r] = 0;
        if (CHANNEL && live[r]) {
            m[r] = j.mask[(int64_t)y * j.pitch + x];
            // solid nodes, and the boundary nodes that k_qlinks and
            // k_fd_columns update (interpolated links, finite-difference
            // open columns), are not stepped here
            live[r] = !(m[r] & (M_SOLID | M_SPECIAL));
        }
        if (live[r]) gather<P, CHANNEL, MODE, false, false>(j, src, site(j, x, y), m[r], t, u_peak, omega_d, f[r]);
    }
#pragma unroll
    for (int r = 0; r < CPT; ++r) {
        if (!live[r]) continue;
        C drho, ux, uy;
        bgk(f[r], omega, drho, ux, uy);
        scatter<P, CHANNEL, MODE, NT>(j, dst, site(j, x, y0 + r * by), m[r], f[r]);
    }
}

// One step for every live node of every sample of one job.
template <int P, bool CHANNEL, int PARITY, int CPT, int LAYOUT, bool NT>
__global__ __launch_bounds__(256) void k_step(JobDev j, const int64_t *d_t, int k, int tiles_x, int tiles_y,
                                              int64_t ntiles) {
    const int64_t t = *d_t + k;
    const int64_t G = gridDim.x;
    const int64_t per_sample = (int64_t)tiles_x * tiles_y;
    for (int64_t tile = xcd_logical(blockIdx.x, G); tile < ntiles; tile += G) {
        const int64_t smp = tile / per_sample;
        const int64_t rem = tile - smp * per_sample;
        const int ty = (int)(rem / tiles_x), tx = (int)(rem - (int64_t)ty * tiles_x);
        tile_update<P, CHANNEL, PARITY, CPT, LAYOUT, NT>(j, t, smp, tx, ty);
    }
}

// Boundary nodes of jobs with interpolated boundaries (AB layout), stepped
// apart from k_step so that the bulk kernel keeps its registers and
// occupancy. Both kernels below read only the source slab and write only
// their own nodes of the destination slab, so they and k_step of the same
// step are independent.
//
// Nodes with interpolated cylinder links (listed in j.special), one thread
// per (node, sample): gather with the interpolation, collide, store.
template <int P, int PARITY>
__global__ __launch_bounds__(64) void k_qlinks(JobDev j, const int64_t *d_t, int k) {
    using PR = Prec<P>;
    using C = typename PR::C;
    using T = typename PR::T;
    const int64_t t = *d_t + k;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= j.n_special) return;
    const int64_t node = j.special[e];
    const int y = (int)(node / j.pitch), x = (int)(node - (int64_t)y * j.pitch);
    const uint32_t m = j.mask[node];
    const T *src_all = (const T *)(PARITY ? j.f2 : j.f);
    T *dst_all = (T *)(PARITY ? j.f : j.f2);
    const Site st = site(j, x, y);
    for (int64_t smp = blockIdx.y; smp < j.S; smp += gridDim.y) {
        const SampleDev &sd = j.smp[smp];
        C f[9], drho, ux, uy;
        gather<P, true, AB_PULL, false, true>(j, src_all + smp * 9 * j.plane, st, m, t, sd.u_peak, sd.omega, f);
        bgk(f, (C)sd.omega, drho, ux, uy);
        scatter<P, true, AB_PULL, false>(j, dst_all + smp * 9 * j.plane, st, m, f);
    }
}

// The two open columns of a finite-difference inlet/outlet. One workgroup
// per (column, chunk of FD_ROWS rows, sample); its threads gather, one node
// each, the column node and the two nodes next to it into the fluid, for the
// chunk's rows plus two halo rows on each side, and share the velocities
// through LDS; the column threads then rebuild, collide and store.
constexpr int FD_RB = 85, FD_HALO = 2, FD_ROWS = FD_RB - 2 * FD_HALO, FD_BLOCK = 256;

template <int P, int PARITY>
__global__ __launch_bounds__(FD_BLOCK) void k_fd_columns(JobDev j, const int64_t *d_t, int k) {
    using PR = Prec<P>;
    using C = typename PR::C;
    using T = typename PR::T;
    __shared__ double ub[FD_RB], u1x[FD_RB], u1y[FD_RB], u2x[FD_RB], u2y[FD_RB];
    const int64_t t = *d_t + k;
    const int chunks = (j.ny + FD_ROWS - 1) / FD_ROWS;
    const bool inlet = (int)blockIdx.x < chunks;
    const int chunk = inlet ? (int)blockIdx.x : (int)blockIdx.x - chunks;
    const int tid = threadIdx.x;
    const int c = tid / FD_RB, r = tid - c * FD_RB;  // c: 0 the column, 1 and 2 into the fluid
    const int x = inlet ? c : j.nx - 1 - c;
    const int y = chunk * FD_ROWS - FD_HALO + r;
    const bool valid = c < 3 && y >= 0 && y < j.ny;
    const bool own = valid && c == 0 && r >= FD_HALO && r < FD_RB - FD_HALO;
    const uint32_t m = valid ? j.mask[(int64_t)y * j.pitch + x] : 0u;
    const T *src_all = (const T *)(PARITY ? j.f2 : j.f);
    T *dst_all = (T *)(PARITY ? j.f : j.f2);
    for (int64_t smp = blockIdx.y; smp < j.S; smp += gridDim.y) {
        const SampleDev &sd = j.smp[smp];
        const T *src = src_all + smp * 9 * j.plane;
        C f[9];
        double rho = 1.0, ux = 0.0;
        if (valid) {
            const Site st = site(j, x, y);
            if (c == 0) {
                gather<P, true, AB_PULL, false, false>(j, src, st, m, t, sd.u_peak, sd.omega, f);
                fd_state(j, f, inlet, y, t, sd.u_peak, rho, ux);
                ub[r] = ux;
            } else {
                C drho, gx, gy;
                gather<P, true, AB_PULL, false, true>(j, src, st, m, t, sd.u_peak, sd.omega, f);
                moments(f, drho, gx, gy);
                if (c == 1) {
                    u1x[r] = (double)gx;
                    u1y[r] = (double)gy;
                } else {
                    u2x[r] = (double)gx;
                    u2y[r] = (double)gy;
                }
            }
        }
        __syncthreads();
        if (own) {
            if (t > 0) {  // the state at t = 0 is the rest state as gathered
                const double sdx = inlet ? 1.0 : -1.0;
                const double dyux = fd_dy(y, j.ny, ub[r - 2], ub[r - 1], ux, ub[r + 1], ub[r + 2]);
                const double dxux = sdx * (-3.0 * ux + 4.0 * u1x[r] - u2x[r]) * 0.5;
                const double dxuy = sdx * (-3.0 * 0.0 + 4.0 * u1y[r] - u2y[r]) * 0.5;
                fd_rebuild(f, rho, ux, dxux, dxuy, dyux, sd.omega);
            }
            C drho, gx, gy;
            bgk(f, (C)sd.omega, drho, gx, gy);
            scatter<P, true, AB_PULL, false>(j, dst_all + smp * 9 * j.plane, site(j, x, y), m, f);
        }
        __syncthreads();  // the LDS rows are reused by the next sample
    }
}

// ------------------------------------------------------------------ fused steps
// Periodic lattices (no boundary rules), AB layout: N = 2..4 steps per launch
// (temporal blocking). A workgroup takes a tile of 64 x TY output nodes of
// one sample and keeps a ring of N - 1 nodes around it in LDS. Phase 1 pulls
// the state at t for tile and ring from the source slab and collides it
// (step t); each later phase pulls from LDS, collides the next step on a
// region one node narrower (held in registers across a barrier, then written
// back to LDS); the last phase covers the tile itself and stores f*(t+N-1)
// to the other slab. Each population crosses HBM once per N steps (the
// ring's re-reads are served by L2: neighbouring tiles run together). Same
// per-node arithmetic as k_step, including the storage rounding of every
// intermediate state.
constexpr int FUSE_TX = 64;

// Buffer loads for the fused kernel: base address and size in a (uniform)
// resource descriptor, a 32-bit byte offset per lane and a uniform offset per
// population plane; no 64-bit address arithmetic per load. 0x00020000 is the
// descriptor's fourth word for raw 32-bit data on this GPU family.
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void *p, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, 0x00020000);
}
template <int P>
struct BufLd;
// raw(): the stored value as loaded; cvt(): its compute value (kept apart so
// that a load's register is not consumed before it is needed)
template <>
struct BufLd<UQ_FP64> {
    using R = double;
    __device__ static inline R raw(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    }
    __device__ static inline double cvt(R v, float) { return v; }
    __device__ static inline double ld(__amdgpu_buffer_rsrc_t r, int voff, int soff, float inv) {
        return cvt(raw(r, voff, soff), inv);
    }
};
template <>
struct BufLd<UQ_FP32> {
    using R = float;
    __device__ static inline R raw(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    }
    __device__ static inline float cvt(R v, float) { return v; }
    __device__ static inline float ld(__amdgpu_buffer_rsrc_t r, int voff, int soff, float inv) {
        return cvt(raw(r, voff, soff), inv);
    }
};
template <>
struct BufLd<UQ_FP16S> {
    using R = unsigned short;
    __device__ static inline R raw(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
        return __builtin_bit_cast(unsigned short, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
    }
    __device__ static inline float cvt(R v, float inv) { return Prec<UQ_FP16S>::up(__builtin_bit_cast(_Float16, v), inv); }
    __device__ static inline float ld(__amdgpu_buffer_rsrc_t r, int voff, int soff, float inv) {
        return cvt(raw(r, voff, soff), inv);
    }
};
template <>
struct BufLd<UQ_BF16S> {
    using R = unsigned short;
    __device__ static inline R raw(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
        return __builtin_bit_cast(unsigned short, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
    }
    __device__ static inline float cvt(R v, float) { return __uint_as_float((uint32_t)v << 16); }
    __device__ static inline float ld(__amdgpu_buffer_rsrc_t r, int voff, int soff, float inv) {
        return cvt(raw(r, voff, soff), inv);
    }
};

// buffer stores: per-lane byte offset + wave-uniform byte offset (cached)
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
template <int P>
struct BufSt;
template <>
struct BufSt<UQ_FP64> {
    __device__ static inline void st(__amdgpu_buffer_rsrc_t r, double v, int voff, int soff, float) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, voff, soff, 0);
    }
};
template <>
struct BufSt<UQ_FP32> {
    __device__ static inline void st(__amdgpu_buffer_rsrc_t r, float v, int voff, int soff, float) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
    }
};
template <>
struct BufSt<UQ_FP16S> {
    __device__ static inline void st(__amdgpu_buffer_rsrc_t r, float v, int voff, int soff, float sc) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, (_Float16)(v * sc)), r, voff, soff, 0);
    }
};
template <>
struct BufSt<UQ_BF16S> {
    __device__ static inline void st(__amdgpu_buffer_rsrc_t r, float v, int voff, int soff, float) {
        __builtin_amdgcn_raw_buffer_store_b16(Prec<UQ_BF16S>::rne(v), r, voff, soff, 0);
    }
};

// wrap a coordinate into [0, n) (it is at most a ring away from it, but the
// ring may exceed a tiny lattice)
__device__ inline int wrap_coord(int v, int n) {
    while (v < 0) v += n;
    while (v >= n) v -= n;
    return v;
}

template <int P, int TY, int N>
__global__ __launch_bounds__(256) void k_stepN(JobDev j, bool src2, int tiles_x, int tiles_y, int64_t ntiles) {
    using PR = Prec<P>;
    using C = typename PR::C;
    using T = typename PR::T;
    constexpr int RG = N - 1;                 // ring width
    constexpr int LW = FUSE_TX + 2 * RG;      // LDS row length
    constexpr int LH = TY + 2 * RG;           // LDS rows
    constexpr int PER = (LW * LH + 255) / 256; // region nodes per thread (bound)
    __shared__ C lds[9][LH][LW];
    const T *src_all = (const T *)(src2 ? j.f2 : j.f);
    T *dst_all = (T *)(src2 ? j.f : j.f2);
    const int nx = j.nx, ny = j.ny;
    // offsets inside one sample fit in 32 bits (9 planes < 2^31 elements)
    const int pitch = (int)j.pitch, plane = (int)j.plane;
    const float inv = j.inv_scale, sc = j.scale;
    const int tid = threadIdx.x;
    const int64_t G = gridDim.x;
    const int64_t per_sample = (int64_t)tiles_x * tiles_y;
    for (int64_t tile = xcd_logical(blockIdx.x, G); tile < ntiles; tile += G) {
        const int64_t smp = tile / per_sample;
        const int64_t rem = tile - smp * per_sample;
        const int ty = (int)(rem / tiles_x), tx = (int)(rem - (int64_t)ty * tiles_x);
        const int x0 = tx * FUSE_TX, y0 = ty * TY;
        const int w = min(FUSE_TX, nx - x0), h = min(TY, ny - y0);
        const T *src = src_all + smp * 9 * (int64_t)plane;
        T *dst = dst_all + smp * 9 * (int64_t)plane;
        const C omega = (C)j.smp[smp].omega;
        const int plane_b = plane * (int)sizeof(T);
        const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(src, 9 * plane_b);
        // phase 1: step t on tile and ring, from the source slab. A thread's
        // elements e = tid + 256 k (their (r, c) advance by (256 / RW,
        // 256 % RW) per k) issue all their loads before any is used.
        {
            const int RW = w + 2 * RG, RH = h + 2 * RG, n_el = RW * RH;
            const int dq = 256 / RW, dr = 256 - dq * RW;
            int rr[PER], cc[PER];
            {
                int r = tid / RW, c = tid - r * RW;
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    rr[k] = r;
                    cc[k] = c;
                    r += dq;
                    c += dr;
                    if (c >= RW) {
                        c -= RW;
                        ++r;
                    }
                }
            }
            // B elements at a time issue their loads together: all of them in
            // FP64 (long load latency per byte, registers to spare), one at a
            // time in the 4- and 2-byte formats (more waves in flight instead)
            constexpr int B = P == UQ_FP64 ? PER : 1;
#pragma unroll
            for (int kb = 0; kb < PER; kb += B) {
                C f[B][9];
#pragma unroll
                for (int q2 = 0; q2 < B; ++q2) {
                    const int k = kb + q2;
                    if (k < PER && tid + 256 * k < n_el) {
                        int gx = x0 - RG + cc[k], gy = y0 - RG + rr[k];
                        if (gx < 0 || gx >= nx) gx = wrap_coord(gx, nx);
                        if (gy < 0 || gy >= ny) gy = wrap_coord(gy, ny);
                        // the pull sources: columns x-1, x, x+1 and rows y-1,
                        // y, y+1 (wrapped), one byte offset per direction
                        const int xm = gx == 0 ? nx - 1 : gx - 1, xp = gx == nx - 1 ? 0 : gx + 1;
                        const int ym = gy == 0 ? ny - 1 : gy - 1, yp = gy == ny - 1 ? 0 : gy + 1;
                        const int r0 = gy * pitch, rm = ym * pitch, rp = yp * pitch;
#pragma unroll
                        for (int i = 0; i < 9; ++i) {
                            const int col = CXd[i] > 0 ? xm : (CXd[i] < 0 ? xp : gx);
                            const int row = CYd[i] > 0 ? rm : (CYd[i] < 0 ? rp : r0);
                            f[q2][i] = BufLd<P>::ld(rsrc, (row + col) * (int)sizeof(T), i * plane_b, inv);
                        }
                    }
                }
#pragma unroll
                for (int q2 = 0; q2 < B; ++q2) {
                    const int k = kb + q2;
                    if (k < PER && tid + 256 * k < n_el) {
                        C drho, ux, uy;
                        bgk(f[q2], omega, drho, ux, uy);
#pragma unroll
                        for (int i = 0; i < 9; ++i) lds[i][rr[k]][cc[k]] = PR::rt(f[q2][i], sc, inv);
                    }
                }
            }
        }
        __syncthreads();
        // middle phases: steps t+1 .. t+N-2 on shrinking regions, in LDS;
        // each thread keeps its new values in registers across the barrier
        auto middle = [&](auto ph_c) {
            constexpr int PH = decltype(ph_c)::value;
            constexpr int PERM = ((LW - 2 * PH) * (LH - 2 * PH) + 255) / 256;
            const int RW = w + 2 * (RG - PH), RH = h + 2 * (RG - PH), n_el = RW * RH;
            const int dq = 256 / RW, dr = 256 - dq * RW;
            C g[PERM][9];
            int rr[PERM], cc[PERM];
            {
                int r = tid / RW, c = tid - r * RW;
#pragma unroll
                for (int k = 0; k < PERM; ++k) {
                    rr[k] = r + PH;
                    cc[k] = c + PH;
                    r += dq;
                    c += dr;
                    if (c >= RW) {
                        c -= RW;
                        ++r;
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < PERM; ++k) {
                if (tid + 256 * k < n_el) {
#pragma unroll
                    for (int i = 0; i < 9; ++i) g[k][i] = lds[i][rr[k] - CYd[i]][cc[k] - CXd[i]];
                    C drho, ux, uy;
                    bgk(g[k], omega, drho, ux, uy);
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < PERM; ++k) {
                if (tid + 256 * k < n_el) {
#pragma unroll
                    for (int i = 0; i < 9; ++i) lds[i][rr[k]][cc[k]] = PR::rt(g[k][i], sc, inv);
                }
            }
            __syncthreads();
        };
        if constexpr (N >= 3) middle(std::integral_constant<int, 1>());
        if constexpr (N >= 4) middle(std::integral_constant<int, 2>());
        // last phase: step t+N-1 on the tile, to the destination slab
        const int cx = tid & 63;
        for (int r = tid >> 6; r < h; r += 4) {
            if (cx < w) {
                C f[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) f[i] = lds[i][r + RG - CYd[i]][cx + RG - CXd[i]];
                C drho, ux, uy;
                bgk(f, omega, drho, ux, uy);
                const int own = (y0 + r) * pitch + x0 + cx;
#pragma unroll
                for (int i = 0; i < 9; ++i) PR::st_nt(dst + (i * plane + own), f[i], sc);
            }
        }
        __syncthreads();  // LDS is reused by the next tile
    }
}

// ------------------------------------------------------------------ fused steps, sliding window
// The same N-step fusion organised as a pipeline down a strip of W columns
// of one sample (W <= 64 - 2(N-1)): each wave of the workgroup computes one
// time level, one lattice row per iteration, two rows behind the level it
// reads. Level 1 pulls from the source slab (D rows ahead, in registers);
// levels 2..N pull from LDS rows of the level below; level N stores to the
// other slab. Only the strip's x-ring (N-1 columns per side) and a chunk's
// y-halo are computed twice (11 % at N = 4 with 52-column strips and 64-row
// chunks, against 45 % for the 8-row tiles above), and every address that
// depends on the row is wave-uniform (scalar registers): a lane keeps one
// column for the whole strip.
// Between two levels each direction is read once, by the row that pulls it:
// c_y = -1 directions one iteration after they are written (rows kept: 2),
// c_y = 0 two iterations after (3), c_y = +1 three after (4). Rows are
// offset by 12 (a multiple of 2, 3 and 4) to keep slots positive.
template <int P, int N>
struct WindowRings {
    static constexpr int NR = N > 1 ? N - 1 : 1;
    using C = typename Prec<P>::C;
    C ra[NR][2][3][64], rb[NR][3][3][64], rc[NR][4][3][64];
};

// One work item of the strip window: strip `strip` (columns [strip W,
// strip W + W)) of rows [chunk H, chunk H + H) of sample smp, N steps, from
// the slab src2 names to the other one; the wave's level is lvl. Ends with
// a barrier, so the rings may be reused by the next item at once.
template <int P, int N, int D>
__device__ __forceinline__ void stepW_item(const JobDev &j, bool src2, int W, int H, int64_t smp, int chunk,
                                           int strip, bool nt, int lvl, WindowRings<P, N> &rings) {
    using PR = Prec<P>;
    using C = typename PR::C;
    using T = typename PR::T;
    constexpr int RG = N - 1;
    auto &ra = rings.ra;
    auto &rb = rings.rb;
    auto &rc = rings.rc;
    const T *src_all = (const T *)(src2 ? j.f2 : j.f);
    T *dst_all = (T *)(src2 ? j.f : j.f2);
    const int nx = j.nx, ny = j.ny;
    const int pitch = (int)j.pitch, plane = (int)j.plane;
    const int plane_b = plane * (int)sizeof(T), pitch_b = pitch * (int)sizeof(T);
    const float inv = j.inv_scale, sc = j.scale;
    const int lane = threadIdx.x & 63;
    {
        const int x0 = strip * W, w = min(W, nx - x0);
        const int yb = chunk * H, ye = min(ny, yb + H);
        const T *src = src_all + smp * 9 * (int64_t)plane;
        T *dst = dst_all + smp * 9 * (int64_t)plane;
        const C omega = (C)j.smp[smp].omega;
        const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(src, 9 * plane_b), wrsrc = make_rsrc(dst, 9 * plane_b);
        const int wvo = (x0 + lane) * (int)sizeof(T);  // level N's store column
        // this lane's column at this level, and its LDS column (0 = x0 - RG)
        const int span = RG - (lvl - 1);  // columns beyond the strip on each side
        const bool lane_on = lane < w + 2 * span;
        const int lc = lane + (lvl - 1);
        int gc = x0 - span + lane;
        while (gc < 0) gc += nx;
        while (gc >= nx) gc -= nx;
        const int vo0 = gc * (int)sizeof(T), vom = (gc == 0 ? nx - 1 : gc - 1) * (int)sizeof(T),
                  vop = (gc == nx - 1 ? 0 : gc + 1) * (int)sizeof(T);
        // level 1 pulls row y + D while it collides row y: D rows of loads in
        // flight per strip. D + 1 register buffers in rotation: each step
        // collides one in place and refills the one the step before used, so
        // a load never targets a live register (that would leave a copy that
        // waits for the load).
        constexpr int B = D + 1;
        using R = typename BufLd<P>::R;
        R buf[B][9];
        auto pull = [&](R *f, int y) {
            int gy = y;
            while (gy < 0) gy += ny;
            while (gy >= ny) gy -= ny;
            const int r0 = gy * pitch_b, rm = (gy == 0 ? ny - 1 : gy - 1) * pitch_b,
                      rp = (gy == ny - 1 ? 0 : gy + 1) * pitch_b;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int vo = CXd[i] > 0 ? vom : (CXd[i] < 0 ? vop : vo0);
                const int ro = CYd[i] > 0 ? rm : (CYd[i] < 0 ? rp : r0);
                f[i] = BufLd<P>::raw(rsrc, vo, i * plane_b + ro);
            }
        };
        const int y1_end = ye + RG;  // level 1 rows: [yb - RG, ye + RG)
        // collide a pulled row and hand it to the next level (or store it)
        auto finish = [&](C *f, int y) {
            C drho, ux, uy;
            bgk(f, omega, drho, ux, uy);
            if (lvl < N) {
                const int sa = (y + 12) & 1, sb = (y + 12) % 3, sc3 = (y + 12) & 3, L = lvl - 1;
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const C v = PR::rt(f[i], sc, inv);
                    const int g = GJd[i];
                    if (CYd[i] < 0) ra[L][sa][g][lc] = v;
                    else if (CYd[i] == 0) rb[L][sb][g][lc] = v;
                    else rc[L][sc3][g][lc] = v;
                }
            } else if (nt) {
                const int own = y * pitch + x0 + lane;
#pragma unroll
                for (int i = 0; i < 9; ++i) PR::st_nt(dst + (i * plane + own), f[i], sc);
            } else {
#pragma unroll
                for (int i = 0; i < 9; ++i) BufSt<P>::st(wrsrc, f[i], wvo, i * plane_b + y * pitch_b, sc);
            }
        };
        // Level 1's loads are issued by every lane of the wave and for every
        // row (rows past the chunk's end reload its last row), so that no
        // register holds a mix of new and old values.
        if (lvl == 1) {
#pragma unroll
            for (int k = 0; k < D; ++k) pull(buf[k], min(yb - RG + k, y1_end - 1));
        }
        const int n_it = (ye - yb) + 3 * RG;
        for (int it0 = 0; it0 < n_it; it0 += B) {
#pragma unroll
            for (int k = 0; k < B; ++k) {
                const int it = it0 + k;
                if (it >= n_it) break;
                const int y = yb - RG + it - 2 * (lvl - 1);  // this level's row (wave-uniform)
                const bool row_on = y >= yb - span && y < ye + span;
                if (lvl == 1) {
                    if (row_on) {
                        pull(buf[(k + D) % B], min(y + D, y1_end - 1));
                        if (lane_on) {
                            C f[9];  // (buffers are written only by loads)
#pragma unroll
                            for (int i = 0; i < 9; ++i) f[i] = BufLd<P>::cvt(buf[k][i], inv);
                            finish(f, y);
                        }
                    }
                } else if (row_on && lane_on) {
                    C f[9];
                    const int L = lvl - 2;
                    const int sa = (y + 13) & 1, sb = (y + 12) % 3, sc3 = (y + 11) & 3;
#pragma unroll
                    for (int i = 0; i < 9; ++i) {
                        const int g = GJd[i], c = lc - CXd[i];
                        f[i] = CYd[i] < 0 ? ra[L][sa][g][c] : (CYd[i] == 0 ? rb[L][sb][g][c] : rc[L][sc3][g][c]);
                    }
                    finish(f, y);
                }
                __syncthreads();
            }
        }
    }
}

// level of a wave of the strip window, rotated with the workgroup index so
// that the levels' different instruction mixes spread evenly over a CU's
// SIMDs
template <int N>
__device__ inline int window_level() {
    return __builtin_amdgcn_readfirstlane((int)((threadIdx.x >> 6) + blockIdx.x) % N) + 1;  // 1..N
}

template <int P, int N, int D>
__global__ __launch_bounds__(64 * N) void k_stepW(JobDev j, bool src2, int W, int strips, int H, int chunks,
                                                  int64_t nwork, bool nt) {
    __shared__ WindowRings<P, N> rings;
    const int lvl = window_level<N>();
    const int64_t G = gridDim.x;
    for (int64_t wk = xcd_logical(blockIdx.x, G); wk < nwork; wk += G) {
        const int64_t smp = wk / ((int64_t)chunks * strips);
        const int rem = (int)(wk - smp * chunks * strips);
        const int chunk = rem / strips;
        stepW_item<P, N, D>(j, src2, W, H, smp, chunk, rem - chunk * strips, nt, lvl, rings);
    }
}

// ------------------------------------------------------------------ fused steps, full rows
// The sliding window over whole rows: K waves per time level, M columns per
// lane, cover the nx <= 64 K M columns of a row, so on a periodic lattice no
// column is computed twice (only a chunk's row halo is). Each LDS row holds
// one direction of the nx columns at 0..nx-1, already shifted by the
// direction's c_x (periodic wrap included), so that every pull from the row
// below reads the lane's own column. N K waves in one workgroup, one barrier
// per row.
// LDS rings of the level below, by the row a direction group pulls from:
// c_y = -1 (row y + 1, slots 0-1) and c_y = 0 (row y, slots 2-3): 2 rows;
// c_y = +1 (row y - 1, slots 4-6): 3 rows. A row sits in slot s mod 2 or
// s mod 3 of its group, s the row step it is written in. A row holds 64 K M
// values (no padding:
// the shifted writes wrap inside the row), so the three rows of a slot, and
// the same slot of the first two groups, lie a multiple of 64 words apart:
// the compiler pairs those accesses into ds_read2st64 / ds_write2st64.
template <int P, int N, int K, int M>
struct RowsRing {
    static constexpr int NR = N > 1 ? N - 1 : 1;
    static constexpr int CW = 64 * K * M;
    using Array = typename Prec<P>::C[NR][7][3][CW];
};

// One work item of the full-row pipeline: rows [chunk H, chunk H + H) of
// sample smp (with the halo rows the levels need), N steps, from the slab
// src2 names to the other one. Every wave of the workgroup passes the same
// number of barriers, the last one after the item's final row step, so the
// rings may be reused by the next item at once.
template <int P, int N, int K, int M, int D>
__device__ __forceinline__ void stepR_item(const JobDev &j, bool src2, int H, int64_t smp, int chunk, bool nt,
                                           typename RowsRing<P, N, K, M>::Array &rg) {
    using PR = Prec<P>;
    using C = typename PR::C;
    using T = typename PR::T;
    constexpr int RG = N - 1;
    const T *src_all = (const T *)(src2 ? j.f2 : j.f);
    T *dst_all = (T *)(src2 ? j.f : j.f2);
    const int nx = j.nx, ny = j.ny;
    const int plane = (int)j.plane;
    const int plane_b = plane * (int)sizeof(T), pitch_b = (int)j.pitch * (int)sizeof(T);
    const float inv = j.inv_scale, sc = j.scale;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lvl = wave / K + 1;  // 1..N
    // Lanes past the lattice take the last column: they read what its own
    // lane reads, compute the same values and write them to the same places
    // (the same bits), so no lane needs a guard and the compiler keeps the
    // collisions and the LDS reads that feed them unconditional.
    int c[M], vo0[M], vom[M], vop[M], wp[M], wm[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        c[m] = min(((wave - (lvl - 1) * K) * M + m) * 64 + lane, nx - 1);
        vo0[m] = c[m] * (int)sizeof(T);
        vom[m] = (c[m] == 0 ? nx - 1 : c[m] - 1) * (int)sizeof(T);
        vop[m] = (c[m] == nx - 1 ? 0 : c[m] + 1) * (int)sizeof(T);
        wp[m] = c[m] == nx - 1 ? 0 : c[m] + 1;  // LDS columns of the c_x = +1 and -1 pushes
        wm[m] = c[m] == 0 ? nx - 1 : c[m] - 1;
    }
    // LDS byte offsets of the lane's columns: x, wm, wp in the ring this
    // level writes (ring lvl - 1), x in the ring it reads (ring lvl - 2).
    // Every ring access is one of these plus a constant (slot and
    // direction-row), which the DS instructions take as their immediate
    // offset; the offsets pass through an empty asm once per turn of the row
    // loops so that the compiler keeps them as the bases instead of hoisting
    // one address register per access out of the loop.
    constexpr int GB = RowsRing<P, N, K, M>::CW * (int)sizeof(C), SB = 3 * GB, RB = 7 * SB;
    char *const ring = reinterpret_cast<char *>(&rg);
    int ox[M], om[M], op[M], orx[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        ox[m] = (lvl - 1) * RB + c[m] * (int)sizeof(C);
        om[m] = (lvl - 1) * RB + wm[m] * (int)sizeof(C);
        op[m] = (lvl - 1) * RB + wp[m] * (int)sizeof(C);
        orx[m] = (lvl - 2) * RB + c[m] * (int)sizeof(C);
    }
    auto at = [&](int base, int slot, int g) -> C & { return *reinterpret_cast<C *>(ring + base + slot * SB + g * GB); };
    auto fresh = [&]() {
#pragma unroll
        for (int m = 0; m < M; ++m) asm("" : "+v"(ox[m]), "+v"(om[m]), "+v"(op[m]), "+v"(orx[m]));
    };
    const int span = RG - (lvl - 1);  // rows beyond the chunk on each side
    constexpr int B = D + 1;
    using R = typename BufLd<P>::R;
    R buf[B][M][9];
    {
        const int yb = chunk * H, ye = min(ny, yb + H);
        const T *src = src_all + smp * 9 * (int64_t)plane;
        T *dst = dst_all + smp * 9 * (int64_t)plane;
        const C omega = (C)j.smp[smp].omega;
        const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(src, 9 * plane_b), wrsrc = make_rsrc(dst, 9 * plane_b);
        auto pull = [&](R (*f)[9], int y) {
            int gy = y;
            while (gy < 0) gy += ny;
            while (gy >= ny) gy -= ny;
            const int r0 = gy * pitch_b, rm = (gy == 0 ? ny - 1 : gy - 1) * pitch_b,
                      rp = (gy == ny - 1 ? 0 : gy + 1) * pitch_b;
#pragma unroll
            for (int m = 0; m < M; ++m)
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const int vo = CXd[i] > 0 ? vom[m] : (CXd[i] < 0 ? vop[m] : vo0[m]);
                    const int ro = CYd[i] > 0 ? rm : (CYd[i] < 0 ? rp : r0);
                    f[m][i] = BufLd<P>::raw(rsrc, vo, i * plane_b + ro);
                }
        };
        // a level hands direction i of its column c on to LDS column
        // (c + c_ix) mod nx, where the level above pulls it: every pull
        // then reads the puller's own column, and the periodic wrap costs no
        // extra copies
        // (the c_y = -1 and c_y = 0 groups use slots of the same index, two
        // apart: their writes of equal c_x go in pairs, ds_write2st64).
        // Slots are named by the row step a row is written in, the same
        // count for every level: a row written in step it goes to slot
        // it mod 2 of the first two groups and it mod 3 of the c_y = +1
        // group, and is read in step it + 1 (c_y <= 0 groups) or it + 2
        // (c_y = +1). The row loops advance six steps at a time, so for
        // the unrolled step u (it = 6 n + u) every slot is a constant and
        // each LDS address is the lane's column base plus an immediate.
        auto put = [&](int u, int m, const C *v) {
            const int sa = u & 1, sc3 = u % 3;
            at(ox[m], sa, 0) = v[4];
            at(ox[m], 2 + sa, 0) = v[0];
            at(om[m], sa, 1) = v[7];
            at(om[m], 2 + sa, 2) = v[3];
            at(op[m], sa, 2) = v[8];
            at(op[m], 2 + sa, 1) = v[1];
            at(ox[m], 4 + sc3, 0) = v[2];
            at(op[m], 4 + sc3, 1) = v[5];
            at(om[m], 4 + sc3, 2) = v[6];
        };
        // collide the lane's M nodes of row y and hand each on to the next
        // level
        auto finish = [&](C (*f)[9], int y, int u) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                C drho, ux, uy;
                bgk(f[m], omega, drho, ux, uy);
            }
            // one uniform branch for all the lane's columns, so that both
            // collisions stay in one block
            if (lvl < N) {
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    C v[9];
#pragma unroll
                    for (int i = 0; i < 9; ++i) v[i] = PR::rt(f[m][i], sc, inv);
                    put(u, m, v);
                }
            } else if (nt) {
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const int own = y * (int)j.pitch + c[m];
#pragma unroll
                    for (int i = 0; i < 9; ++i) PR::st_nt(dst + (i * plane + own), f[m][i], sc);
                }
            } else {
#pragma unroll
                for (int m = 0; m < M; ++m)
#pragma unroll
                    for (int i = 0; i < 9; ++i)
                        BufSt<P>::st(wrsrc, f[m][i], vo0[m], i * plane_b + y * pitch_b, sc);
            }
        };
        const int y1_end = ye + RG;  // level 1 rows: [yb - RG, ye + RG)
        const int n_it = (ye - yb) + 3 * RG;
        // Both loops below pass n_it barriers, one per row step, six steps
        // per turn (the slot period; also a multiple of the B load buffers).
        static_assert(6 % B == 0, "the row loops turn over six steps");
        if (lvl == 1) {
#pragma unroll
            for (int k = 0; k < D; ++k) pull(buf[k], min(yb - RG + k, y1_end - 1));
            for (int it0 = 0; it0 < n_it; it0 += 6) {
#pragma unroll
                for (int u = 0; u < 6; ++u) {
                    const int it = it0 + u;
                    if (it >= n_it) break;
                    const int y = yb - RG + it;
                    if (u == 0) fresh();
                    if (y < ye + span) {
                        pull(buf[(u + D) % B], min(y + D, y1_end - 1));
                        C f[M][9];
#pragma unroll
                        for (int m = 0; m < M; ++m)
#pragma unroll
                            for (int i = 0; i < 9; ++i) f[m][i] = BufLd<P>::cvt(buf[u % B][m][i], inv);
                        finish(f, y, u);
                    }
                    __syncthreads();
                }
            }
        } else {
            // Levels above the first read the level below from the LDS rows.
            // The c_y = 0 and c_y = +1 pulls of the next row (rows y + 1 and
            // y of the level below) are complete before this row step begins
            // and their slots are not rewritten in it, so they are read one
            // step ahead into registers (two sets, alternating; for the first
            // row in the step before it), and only the c_y = -1 pulls (row
            // y + 1, written in the previous step) wait at the start of the
            // step. What is read ahead never sits in LDS for more than one
            // step, hence the short rings.
            C pre[2][M][6];
            // step u reads the rows the level below wrote in steps u - 1
            // (slot (u + 1) mod 2) and u - 2 (slot (u + 1) mod 3)
            auto ahead = [&](C (*q)[6], int u) {  // c_y >= 0 pulls of the next row
                const int sb = (u + 1) & 1, sc3 = (u + 1) % 3;
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    int n = 0;
#pragma unroll
                    for (int i = 0; i < 9; ++i) {
                        if (CYd[i] < 0) continue;
                        q[m][n++] = at(orx[m], CYd[i] == 0 ? 2 + sb : 4 + sc3, GJd[i]);
                    }
                }
            };
            const int y_lo = yb - span, y_hi = ye + span;  // this level's rows
            for (int it0 = 0; it0 < n_it; it0 += 6) {
#pragma unroll
                for (int u = 0; u < 6; ++u) {
                    const int it = it0 + u, k = u & 1;
                    if (it >= n_it) break;
                    const int y = yb - RG + it - 2 * (lvl - 1);  // this level's row (wave-uniform)
                    if (u == 0) fresh();
                    if (y == y_lo - 1) {
                        ahead(pre[k ^ 1], u);  // the first row's
                    } else if (y >= y_lo && y < y_hi) {
                        // row y + 1 of the level below: this row's c_y = -1
                        // pulls and the next row's c_y = 0 pulls (slots of the
                        // same index, two apart); row y: the next row's c_y = +1
                        // pulls. All at the lane's own column, 64-word multiples
                        // apart (ds_read2st64 pairs). Past the last row the
                        // values read ahead are not used.
                        const int sa = (u + 1) & 1, sc3 = (u + 1) % 3;
                        C f[M][9];
                        C (*q)[6] = pre[k ^ 1];
#pragma unroll
                        for (int m = 0; m < M; ++m) {
                            // at the lane's own LDS column
                            f[m][4] = at(orx[m], sa, 0);       // (0, -1)
                            f[m][7] = at(orx[m], sa, 1);       // (-1, -1)
                            f[m][8] = at(orx[m], sa, 2);       // (1, -1)
                            q[m][0] = at(orx[m], 2 + sa, 0);   // (0, 0)
                            q[m][1] = at(orx[m], 2 + sa, 1);   // (1, 0)
                            q[m][3] = at(orx[m], 2 + sa, 2);   // (-1, 0)
                            q[m][2] = at(orx[m], 4 + sc3, 0);  // (0, 1)
                            q[m][4] = at(orx[m], 4 + sc3, 1);  // (1, 1)
                            q[m][5] = at(orx[m], 4 + sc3, 2);  // (-1, 1)
                            // this row's c_y >= 0 pulls, read a step ago
                            f[m][0] = pre[k][m][0];
                            f[m][1] = pre[k][m][1];
                            f[m][2] = pre[k][m][2];
                            f[m][3] = pre[k][m][3];
                            f[m][5] = pre[k][m][4];
                            f[m][6] = pre[k][m][5];
                        }
                        // every LDS read of the step (both columns, and the
                        // next row's read-ahead) is issued before the first
                        // collision, which then waits only for its own three
                        __builtin_amdgcn_sched_barrier(0);
                        finish(f, y, u);
                    }
                    __syncthreads();
                }
            }
        }
    }
}

template <int P, int N, int K, int M, int D>
__global__ __launch_bounds__(64 * N * K) void k_stepR(JobDev j, bool src2, int H, int chunks, int64_t nwork,
                                                      bool nt) {
    __shared__ typename RowsRing<P, N, K, M>::Array rg;
    const int64_t G = gridDim.x;
    for (int64_t wk = xcd_logical(blockIdx.x, G); wk < nwork; wk += G) {
        const int64_t smp = wk / chunks;
        stepR_item<P, N, K, M, D>(j, src2, H, smp, (int)(wk - smp * chunks), nt, rg);
    }
}

// Job of work item wk in a batched table (work0 ascending, job 0 at 0).
__device__ inline int fused_job_of(const FusedJob *jobs, int njobs, int64_t wk) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].work0 <= wk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The table entry of a work item, in scalar registers. Every lane of the
// workgroup reads the same entry, but the compiler cannot tell, and a job's
// pointers built from vector registers would put every buffer access of the
// pipeline in a loop over the distinct descriptors (v_readfirstlane per
// access); each dword goes through readfirstlane once per item instead.
__device__ inline FusedJob fused_entry(const FusedJob *jobs, int njobs, int64_t wk) {
    static_assert(sizeof(FusedJob) % 4 == 0, "FusedJob is a whole number of dwords");
    constexpr int NW = (int)(sizeof(FusedJob) / 4);
    uint32_t w[NW];
    __builtin_memcpy(w, &jobs[fused_job_of(jobs, njobs, wk)], sizeof(FusedJob));
#pragma unroll
    for (int i = 0; i < NW; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    FusedJob q;
    __builtin_memcpy(&q, w, sizeof(FusedJob));
    return q;
}

// Batched form: every chunk of every sample of every job in the table, N
// steps per launch; launch number `launch` of a tick reads the slab of
// parity par ^ (launch & 1) of its job (the state of step t + launch N;
// even N go in pairs, as in the single-job schedule).
template <int P, int N, int K, int M, int D>
__global__ __launch_bounds__(64 * N * K) void k_stepR_multi(const FusedJob *jobs, int njobs, int64_t nwork,
                                                            int launch, bool nt) {
    __shared__ typename RowsRing<P, N, K, M>::Array rg;
    const int64_t G = gridDim.x;
    for (int64_t wk = xcd_logical(blockIdx.x, G); wk < nwork; wk += G) {
        const FusedJob q = fused_entry(jobs, njobs, wk);
        const JobDev j = q.j;
        const int64_t local = wk - q.work0;
        const int64_t smp = local / q.chunks;
        stepR_item<P, N, K, M, D>(j, ((q.par ^ launch) & 1) != 0, q.H, smp, (int)(local - smp * q.chunks), nt, rg);
    }
}

// Batched strip window (see k_stepR_multi): every strip of every row chunk
// of every sample of every job in the table, N steps per launch.
template <int P, int N, int D>
__global__ __launch_bounds__(64 * N) void k_stepW_multi(const FusedJob *jobs, int njobs, int64_t nwork, int launch) {
    __shared__ WindowRings<P, N> rings;
    const int lvl = window_level<N>();
    const int64_t G = gridDim.x;
    for (int64_t wk = xcd_logical(blockIdx.x, G); wk < nwork; wk += G) {
        const FusedJob q = fused_entry(jobs, njobs, wk);
        const JobDev j = q.j;
        const int64_t local = wk - q.work0;
        const int64_t smp = local / ((int64_t)q.chunks * q.strips);
        const int rem = (int)(local - smp * q.chunks * q.strips);
        const int chunk = rem / q.strips;
        stepW_item<P, N, D>(j, ((q.par ^ launch) & 1) != 0, q.W, q.H, smp, chunk, rem - chunk * q.strips, false, lvl,
                            rings);
    }
}

// ------------------------------------------------------------------ fused channel steps, full rows
// The full-row pipeline on the channel with half-way bounce-back walls and
// cylinder and Zou-He inlet / outlet (no interpolated rules): the same wall
// and open-column rules as the single-step gather, applied at every level.
// A bounce-back pull takes the node's own opposite population of the level
// below, so the LDS also keeps the row being computed: 3 rows of the
// c_y = -1 directions (their opposites), 3 of c_y = 0, 4 of c_y = +1. Rows
// outside the channel are not computed (their pulls are bounce-backs);
// along x the end columns are open, walls or periodic, as the node masks
// say. Solid nodes are skipped.
// Level L of a launch computes step t0 + L - 1 (the inflow ramp).
// one LDS array for the three rings (c_y = -1: slots 0-2, c_y = 0: 3-5,
// c_y = +1: 6-9), rows padded to a multiple of 64 values: the rows of a
// slot, and the slots of equal index of the first two groups, lie 64-word
// multiples apart, and the compiler pairs those accesses (ds_read2st64 /
// ds_write2st64)
template <int P, int N, int K, int M>
struct RowsRingCh {
    static constexpr int NR = N > 1 ? N - 1 : 1;
    static constexpr int CW = 64 * K * M + 64;
    using Array = typename Prec<P>::C[NR][10][3][CW];
};

// One work item of the channel pipeline: rows [chunk H, chunk H + H) of
// sample smp, steps t0 .. t0 + N - 1 (t0 = *d_t + k0), from the slab src2
// names to the other one; ends with a barrier, like stepR_item.
template <int P, int N, int K, int M, int D>
__device__ __forceinline__ void stepRC_item(const JobDev &j, const int64_t *d_t, int k0, bool src2, int H,
                                            int64_t smp, int chunk, typename RowsRingCh<P, N, K, M>::Array &rq) {
    using PR = Prec<P>;
    using C = typename PR::C;
    using T = typename PR::T;
    constexpr int RG = N - 1;
    constexpr uint32_t BB_BITS = 0x1FFu << M_BB, OPEN_BITS = 0x1FFu << M_OPEN;
    const int64_t t0 = *d_t + k0;
    const T *src_all = (const T *)(src2 ? j.f2 : j.f);
    T *dst_all = (T *)(src2 ? j.f : j.f2);
    const int nx = j.nx, ny = j.ny;
    const int plane = (int)j.plane;
    const int plane_b = plane * (int)sizeof(T), pitch_b = (int)j.pitch * (int)sizeof(T);
    const float inv = j.inv_scale, sc = j.scale;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lvl = wave / K + 1;  // 1..N
    const int64_t t_lvl = t0 + (lvl - 1);
    // the level's K column blocks rotate with the level, so that the blocks
    // with the open end columns (and the cylinder) fall on different SIMDs
    // at different levels (wave w runs on SIMD w mod 4)
    const int kb = (wave - (lvl - 1) * K + (lvl - 1)) % K;
    int c[M], vo0[M], vom[M], vop[M], mvo[M];
    bool on[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        c[m] = (kb * M + m) * 64 + lane;
        on[m] = c[m] < nx;
        const int cc = on[m] ? c[m] : nx - 1;
        mvo[m] = cc * 4;
        vo0[m] = cc * (int)sizeof(T);
        vom[m] = (cc == 0 ? nx - 1 : cc - 1) * (int)sizeof(T);
        vop[m] = (cc == nx - 1 ? 0 : cc + 1) * (int)sizeof(T);
    }
    const __amdgpu_buffer_rsrc_t mrsrc = make_rsrc(j.mask, ny * (int)j.pitch * 4);
    const int span = RG - (lvl - 1);
    constexpr int B = D + 1;
    using R = typename BufLd<P>::R;
    R buf[B][M][9];
    uint32_t mb[B][M];
    {
        const int yb = chunk * H, ye = min(ny, yb + H);
        const int lo = max(0, yb - span), hi = min(ny, ye + span);  // this level's rows
        const T *src = src_all + smp * 9 * (int64_t)plane;
        T *dst = dst_all + smp * 9 * (int64_t)plane;
        const C omega = (C)j.smp[smp].omega;
        // s(t) 4 u_peak of this level's step (uniform)
        const double a_in = ramp_factor(t_lvl, j.ramp) * 4.0 * j.smp[smp].u_peak;
        const __amdgpu_buffer_rsrc_t rsrc = make_rsrc(src, 9 * plane_b), wrsrc = make_rsrc(dst, 9 * plane_b);
        auto clampy = [&](int y) { return y < 0 ? 0 : (y >= ny ? ny - 1 : y); };
        auto pull = [&](R (*f)[9], int y) {
            const int gy = clampy(y);
            const int r0 = gy * pitch_b, rm = (gy == 0 ? ny - 1 : gy - 1) * pitch_b,
                      rp = (gy == ny - 1 ? 0 : gy + 1) * pitch_b;
#pragma unroll
            for (int m = 0; m < M; ++m)
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const int vo = CXd[i] > 0 ? vom[m] : (CXd[i] < 0 ? vop[m] : vo0[m]);
                    const int ro = CYd[i] > 0 ? rm : (CYd[i] < 0 ? rp : r0);
                    f[m][i] = BufLd<P>::raw(rsrc, vo, i * plane_b + ro);
                }
        };
        auto pullm = [&](uint32_t *mm, int y) {
            const int mo = clampy(y) * (int)j.pitch * 4;
#pragma unroll
            for (int m = 0; m < M; ++m) mm[m] = __builtin_amdgcn_raw_buffer_load_b32(mrsrc, mvo[m], mo, 0);
        };
        auto put = [&](int L, int y, int col, const C *v) {  // by direction-row, c_y = -1 and 0 in pairs
            const int s3 = (y + 12) % 3, s4 = (y + 12) & 3;
            rq[L][s3][0][col] = v[4];
            rq[L][3 + s3][0][col] = v[0];
            rq[L][s3][1][col] = v[7];
            rq[L][3 + s3][1][col] = v[1];
            rq[L][s3][2][col] = v[8];
            rq[L][3 + s3][2][col] = v[3];
            rq[L][6 + s4][0][col] = v[2];
            rq[L][6 + s4][1][col] = v[5];
            rq[L][6 + s4][2][col] = v[6];
        };
        // the open-column rule, then collide, then hand on or store
        auto finish = [&](C (*f)[9], const uint32_t *mm, int y) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                if (mm[m] & OPEN_BITS) {
                    // Zou-He overwrites every pull from beyond the column
                    // (inlet 1, 5, 8; outlet 3, 6, 7) without reading it, so
                    // where it runs (t > 0) and the inlet is not also the
                    // outlet (nx > 1) those pulls need not be zeroed first:
                    // the same values as the single-step gather, which
                    // zeroes them at every step (both conditions uniform)
                    if (t_lvl == 0 || nx == 1) {
#pragma unroll
                        for (int i = 0; i < 9; ++i) f[m][i] = ((mm[m] >> (M_OPEN + i)) & 1u) ? C(0) : f[m][i];
                    }
                    if (t_lvl > 0)
                        zou_he_u(f[m], c[m] == 0, c[m] == 0 ? (C)inflow_u_a(a_in, ny, y) : C(0));
                }
            }
#pragma unroll
            for (int m = 0; m < M; ++m) {
                C drho, ux, uy;
                bgk(f[m], omega, drho, ux, uy);
            }
            // one uniform branch for all the lane's columns (see stepR_item)
            if (lvl < N) {
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    if (!on[m] || (mm[m] & M_SOLID)) continue;
                    C v[9];
#pragma unroll
                    for (int i = 0; i < 9; ++i) v[i] = PR::rt(f[m][i], sc, inv);
                    put(lvl - 1, y, c[m] + 1, v);
                    // end-column copies (read only when x is periodic)
                    if (c[m] == nx - 1) put(lvl - 1, y, 0, v);
                    if (c[m] == 0) put(lvl - 1, y, nx + 1, v);
                }
            } else {
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    if (!on[m] || (mm[m] & M_SOLID)) continue;
#pragma unroll
                    for (int i = 0; i < 9; ++i)
                        BufSt<P>::st(wrsrc, f[m][i], vo0[m], i * plane_b + y * pitch_b, sc);
                }
            }
        };
        const int y_first = yb - RG - 2 * (lvl - 1);  // this level's row at iteration 0
        if (lvl == 1) {
#pragma unroll
            for (int k = 0; k < D; ++k) pull(buf[k], yb - RG + k);
        }
#pragma unroll
        for (int k = 0; k < D; ++k) pullm(mb[k], y_first + k);
        const int n_it = (ye - yb) + 3 * RG;
        for (int it0 = 0; it0 < n_it; it0 += B) {
#pragma unroll
            for (int k = 0; k < B; ++k) {
                const int it = it0 + k;
                if (it >= n_it) break;
                const int y = y_first + it;  // this level's row (wave-uniform)
                const bool row_on = y >= lo && y < hi;
                pullm(mb[(k + D) % B], y + D);
                if (lvl == 1) {
                    pull(buf[(k + D) % B], y + D);
                    if (row_on) {
                        C f[M][9];
#pragma unroll
                        for (int m = 0; m < M; ++m) {
#pragma unroll
                            for (int i = 0; i < 9; ++i) f[m][i] = BufLd<P>::cvt(buf[k][m][i], inv);
                            if (mb[k][m] & BB_BITS) {
                                // bounce-back: the node's own opposite population
#pragma unroll
                                for (int i = 0; i < 9; ++i) {
                                    const C o = BufLd<P>::ld(rsrc, vo0[m], OPPd[i] * plane_b + y * pitch_b, inv);
                                    f[m][i] = ((mb[k][m] >> (M_BB + i)) & 1u) ? o : f[m][i];
                                }
                            }
                        }
                        finish(f, mb[k], y);
                    }
                } else if (row_on) {
                    const int L = lvl - 2;
                    const int pa = (y + 13) % 3, pb = (y + 12) % 3, pc = (y + 11) & 3;  // pull rows
                    const int oa = (y + 12) % 3, oc = (y + 12) & 3;                     // own row
                    C f[M][9];
#pragma unroll
                    for (int m = 0; m < M; ++m) {
                        const int lc = c[m] + 1;
#pragma unroll
                        for (int i = 0; i < 9; ++i) {
                            const int g = GJd[i], cl = lc - CXd[i];
                            f[m][i] = CYd[i] < 0 ? rq[L][pa][g][cl]
                                                 : (CYd[i] == 0 ? rq[L][3 + pb][g][cl] : rq[L][6 + pc][g][cl]);
                        }
                        if (mb[k][m] & BB_BITS) {
                            // this node's populations of the level below, by direction
                            C own[9];
                            own[0] = rq[L][3 + pb][0][lc];
                            own[1] = rq[L][3 + pb][1][lc];
                            own[3] = rq[L][3 + pb][2][lc];
                            own[2] = rq[L][6 + oc][0][lc];
                            own[5] = rq[L][6 + oc][1][lc];
                            own[6] = rq[L][6 + oc][2][lc];
                            own[4] = rq[L][oa][0][lc];
                            own[7] = rq[L][oa][1][lc];
                            own[8] = rq[L][oa][2][lc];
#pragma unroll
                            for (int i = 0; i < 9; ++i)
                                f[m][i] = ((mb[k][m] >> (M_BB + i)) & 1u) ? own[OPPd[i]] : f[m][i];
                        }
                    }
                    finish(f, mb[k], y);
                }
                __syncthreads();
            }
        }
    }
}

template <int P, int N, int K, int M, int D>
__global__ __launch_bounds__(64 * N * K) void k_stepRC(JobDev j, const int64_t *d_t, int k0, bool src2, int H,
                                                       int chunks, int64_t nwork) {
    __shared__ typename RowsRingCh<P, N, K, M>::Array rq;
    const int64_t G = gridDim.x;
    for (int64_t wk = xcd_logical(blockIdx.x, G); wk < nwork; wk += G) {
        const int64_t smp = wk / chunks;
        stepRC_item<P, N, K, M, D>(j, d_t, k0, src2, H, smp, (int)(wk - smp * chunks), rq);
    }
}

// Batched form (see k_stepR_multi); launch number `launch` of a tick runs
// steps t + launch N .. of each job, t its step count at the tick's start.
template <int P, int N, int K, int M, int D>
__global__ __launch_bounds__(64 * N * K) void k_stepRC_multi(const FusedJob *jobs, int njobs, int64_t nwork,
                                                             int launch) {
    __shared__ typename RowsRingCh<P, N, K, M>::Array rq;
    const int64_t G = gridDim.x;
    for (int64_t wk = xcd_logical(blockIdx.x, G); wk < nwork; wk += G) {
        const FusedJob q = fused_entry(jobs, njobs, wk);
        const JobDev j = q.j;
        const int64_t local = wk - q.work0;
        const int64_t smp = local / q.chunks;
        stepRC_item<P, N, K, M, D>(j, q.d_t, launch * N, ((q.par ^ launch) & 1) != 0, q.H, smp,
                                   (int)(local - smp * q.chunks), rq);
    }
}

// The same address as a pointer into global memory. A pointer loaded from a
// table in device memory is generic to the compiler, and the accesses through
// it compile to flat instructions (64-bit addresses in vector registers, and
// waits on the LDS counter as well); rebuilt from its integer value in the
// global address space, they compile to global loads and stores, as those of
// a kernel argument do.
template <typename T>
__device__ inline T *global_ptr(T *p) {
    return (T *)(__attribute__((address_space(1))) T *)(uintptr_t)p;
}

// One step for every live node of every sample of every job in a table
// (continuous batching). Jobs may differ in geometry, lattice, sample count
// and step parity; all use the AA layout, one row per thread. Tiles of job q
// are the global tiles [tile0_q, tile0_{q+1}); a job whose step count has
// reached its target is skipped, so the same launch (or captured graph) stays
// valid while jobs finish.
template <int P>
__global__ __launch_bounds__(256) void k_step_multi(const MultiJob *jobs, int njobs, int64_t ntiles, int k) {
    const int64_t G = gridDim.x;
    for (int64_t tile = xcd_logical(blockIdx.x, G); tile < ntiles; tile += G) {
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].tile0 <= tile) lo = mid;
            else hi = mid - 1;
        }
        const MultiJob &q = jobs[lo];
        const int64_t t = q.t + k;
        if (t >= q.n_steps || k >= q.adv) continue;
        JobDev jd = q.j;
        jd.f = global_ptr(jd.f);
        jd.smp = global_ptr(jd.smp);
        jd.mask = global_ptr(jd.mask);
        const int64_t per_sample = (int64_t)q.tiles_x * q.tiles_y;
        const int64_t local = tile - q.tile0;
        const int64_t smp = local / per_sample;
        const int64_t rem = local - smp * per_sample;
        const int ty = (int)(rem / q.tiles_x), tx = (int)(rem - (int64_t)ty * q.tiles_x);
        if (jd.geom == 1) {
            if (t & 1) tile_update<P, true, 1, 1, UQ_LAYOUT_AA, false>(jd, t, smp, tx, ty);
            else tile_update<P, true, 0, 1, UQ_LAYOUT_AA, false>(jd, t, smp, tx, ty);
        } else {
            if (t & 1) tile_update<P, false, 1, 1, UQ_LAYOUT_AA, false>(jd, t, smp, tx, ty);
            else tile_update<P, false, 0, 1, UQ_LAYOUT_AA, false>(jd, t, smp, tx, ty);
        }
    }
}

__global__ void k_advance_multi(MultiJob *jobs, int njobs) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < njobs) jobs[q].t += jobs[q].adv;
}

// ------------------------------------------------------------------ init
// Equilibrium start. AA stores f~_eq(x) in slot i of node x. AB stores
// g_i(x - c_i) = f~_eq,i(x) (the value the first pull of node x reads), so
// every node computes its own equilibrium once and writes it to the nine
// nodes x - c_i (periodic wrap; the channel starts at rest, f~ = 0).
template <int P, int LAYOUT>
__global__ __launch_bounds__(256) void k_init(JobDev j) {
    using PR = Prec<P>;
    using T = typename PR::T;
    const int64_t cells = (int64_t)j.ny * j.pitch;
    for (int64_t smp = blockIdx.y; smp < j.S; smp += gridDim.y) {
        T *base = (T *)j.f + smp * 9 * j.plane;
        const SampleDev sd = j.smp[smp];
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells;
             c += (int64_t)gridDim.x * blockDim.x) {
            const int y = (int)(c / j.pitch), x = (int)(c - (int64_t)y * j.pitch);
            double f[9];
            for (int i = 0; i < 9; ++i) f[i] = 0.0;
            if (x < j.nx && j.geom == 0) {
                double ux, uy, p;
                if (j.init == UQ_INIT_TGV_HARMONIC) {
                    // perturbed vortex (Eq. taylorGreen), two periods per side,
                    // amplitude u0 (1 + eps) with first-order harmonics of 2 kappa
                    const double kx = 4.0 * M_PI / j.nx, ky = 4.0 * M_PI / j.ny;
                    const double ax = kx * x, ay = ky * y;
                    const double sx = sin(2.0 * ax), cx = cos(2.0 * ax), sy = sin(2.0 * ay), cy = cos(2.0 * ay);
                    const double eps = 0.25 * (sd.zeta[0] * sx * sy + sd.zeta[1] * sx * cy + sd.zeta[2] * cx * sy +
                                               sd.zeta[3] * cx * cy);
                    const double uR = sd.u0 * (1.0 + eps);
                    ux = -uR * cos(ax) * sin(ay);
                    uy = uR * sin(ax) * cos(ay);
                    p = -0.25 * uR * uR * (cos(2.0 * ax) + cos(2.0 * ay));
                } else {
                    // Taylor-Green vortex (Eqs. TGV_vel, TGV_press at t = 0)
                    const double kx = 2.0 * M_PI / j.nx, ky = 2.0 * M_PI / j.ny;
                    const double ax = kx * x + sd.phase_x, ay = ky * y + sd.phase_y;
                    ux = -sd.u0 * cos(ax) * sin(ay);
                    uy = sd.u0 * sin(ax) * cos(ay);
                    p = -0.25 * sd.u0 * sd.u0 * (cos(2.0 * ax) + (kx / ky) * (kx / ky) * cos(2.0 * ay));
                }
                const double drho = 3.0 * p, rho = 1.0 + drho;  // rho = 1 + p/cs2
                const double uu = 1.5 * (ux * ux + uy * uy);
                for (int i = 0; i < 9; ++i) {
                    const double cu = CXd[i] * ux + CYd[i] * uy;
                    f[i] = wgt<double>(i) * (drho + rho * (3.0 * cu + 4.5 * cu * cu - uu));
                }
            }
            if (LAYOUT == UQ_LAYOUT_AB && x < j.nx) {
                const Site s = site(j, x, y);
                for (int i = 0; i < 9; ++i) {
                    const int xd = sx_of(s, -CXd[i]), yd = sy_of(s, -CYd[i]);
                    PR::st(base + i * j.plane + (int64_t)yd * j.pitch + xd, (typename PR::C)f[i], j.scale);
                }
            } else if (LAYOUT != UQ_LAYOUT_AB) {
                for (int i = 0; i < 9; ++i) PR::st(base + i * j.plane + c, (typename PR::C)f[i], j.scale);
            }
        }
    }
}

// ------------------------------------------------------------------ QoIs
// Neumaier's compensated sum
struct NSum {
    double s = 0.0, c = 0.0;
    __device__ inline void add(double x) {
        const double t = s + x;
        c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
        s = t;
    }
    __device__ inline double val() const { return s + c; }
};

// One workgroup per sample: KE, momentum-exchange force, non-finite count.
template <int P, bool CHANNEL, int MODE>
__global__ __launch_bounds__(256) void k_qoi(JobDev j, int64_t t, double *out) {
    using PR = Prec<P>;
    using C = typename PR::C;
    using T = typename PR::T;
    const int64_t smp = blockIdx.x;
    const T *base = (const T *)(MODE == AB_PULL && (t & 1) ? j.f2 : j.f) + smp * 9 * j.plane;
    const SampleDev sd = j.smp[smp];
    NSum ke, fx, fy;
    double bad = 0.0;
    const int64_t cells = (int64_t)j.nx * j.ny;
    for (int64_t c = threadIdx.x; c < cells; c += blockDim.x) {
        const int y = (int)(c / j.nx), x = (int)(c - (int64_t)y * j.nx);
        uint32_t m = 0;
        if (CHANNEL) {
            m = j.mask[(int64_t)y * j.pitch + x];
            if (m & M_SOLID) continue;
        }
        const Site s = site(j, x, y);
        C f[9], drho, ux, uy;
        gather<P, CHANNEL, MODE>(j, base, s, m, t, sd.u_peak, sd.omega, f);
        if (CHANNEL && (m & (0x1FFu << M_CYL))) {
            bgk(f, (C)sd.omega, drho, ux, uy);
            for (int k = 1; k < 9; ++k)
                if (m & (1u << (M_CYL + k))) {
                    // exchange on link k: c_k (f*_k(x) + what the wall returns
                    // at t+1), both unshifted; half-way: 2 c_k f*_k(x)
                    const double fk = (double)f[k] + wgt<double>(k);
                    double back = fk;
                    if (MODE == AB_PULL && (m & M_QLINK)) {
                        const int i = OPPd[k];
                        const double q = j.q[(int64_t)i * j.ny * j.pitch + (int64_t)y * j.pitch + x];
                        if (q >= 0.5) {
                            const double a = 1.0 / (2.0 * q);
                            back = a * fk + (1.0 - a) * ((double)f[i] + wgt<double>(i));
                        } else if (q > 0.0) {
                            // f*_k of the node behind, x - c_k = x + c_i
                            const int xb = sx_of(s, CXd[i]), yb = sy_of(s, CYd[i]);
                            C g[9], gr, gx, gy;
                            gather<P, CHANNEL, MODE>(j, base, site(j, xb, yb), j.mask[(int64_t)yb * j.pitch + xb], t,
                                                     sd.u_peak, sd.omega, g);
                            bgk(g, (C)sd.omega, gr, gx, gy);
                            back = 2.0 * q * fk + (1.0 - 2.0 * q) * ((double)g[k] + wgt<double>(k));
                        }
                    }
                    fx.add(CXd[k] * (fk + back));
                    fy.add(CYd[k] * (fk + back));
                }
        } else {
            moments(f, drho, ux, uy);
        }
        const double dux = (double)ux, duy = (double)uy;
        if (!isfinite(dux) || !isfinite(duy) || !isfinite((double)drho)) bad += 1.0;
        ke.add(dux * dux + duy * duy);
    }
    // fixed-order block reduction (deterministic)
    __shared__ double red[4][256];
    red[0][threadIdx.x] = ke.val();
    red[1][threadIdx.x] = fx.val();
    red[2][threadIdx.x] = fy.val();
    red[3][threadIdx.x] = bad;
    __syncthreads();
    if (threadIdx.x < 4) {
        NSum acc;
        for (int k = 0; k < (int)blockDim.x; ++k) acc.add(red[threadIdx.x][k]);
        double v = acc.val();
        if (threadIdx.x == 0) v *= j.ke_norm;
        out[smp * 4 + threadIdx.x] = v;
    }
}

// Per-sample fields: out[s][4][ny][nx] = ux, uy, rho, |u| (0 at solid nodes).
template <int P, bool CHANNEL, int MODE>
__global__ __launch_bounds__(256) void k_fields(JobDev j, int64_t t, double *out) {
    using PR = Prec<P>;
    using C = typename PR::C;
    using T = typename PR::T;
    const int64_t cells = (int64_t)j.nx * j.ny;
    for (int64_t smp = blockIdx.y; smp < j.S; smp += gridDim.y) {
    const T *base = (const T *)(MODE == AB_PULL && (t & 1) ? j.f2 : j.f) + smp * 9 * j.plane;
    const double u_peak = j.smp[smp].u_peak, omega = j.smp[smp].omega;
    double *o = out + smp * 4 * cells;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(c / j.nx), x = (int)(c - (int64_t)y * j.nx);
        uint32_t m = 0;
        if (CHANNEL) {
            m = j.mask[(int64_t)y * j.pitch + x];
            if (m & M_SOLID) {
                o[c] = 0.0;
                o[cells + c] = 0.0;
                o[2 * cells + c] = 0.0;
                o[3 * cells + c] = 0.0;
                continue;
            }
        }
        const Site s = site(j, x, y);
        C f[9], drho, ux, uy;
        gather<P, CHANNEL, MODE>(j, base, s, m, t, u_peak, omega, f);
        moments(f, drho, ux, uy);
        o[c] = (double)ux;
        o[cells + c] = (double)uy;
        o[2 * cells + c] = 1.0 + (double)drho;
        o[3 * cells + c] = sqrt((double)ux * (double)ux + (double)uy * (double)uy);
    }
    }
}

// One sample's unshifted populations, natural order [9][ny][nx] in double.
template <int P, bool CHANNEL, int MODE>
__global__ __launch_bounds__(256) void k_export(JobDev j, int64_t t, int64_t smp, double *out) {
    using PR = Prec<P>;
    using C = typename PR::C;
    using T = typename PR::T;
    const int64_t cells = (int64_t)j.nx * j.ny;
    const T *base = (const T *)(MODE == AB_PULL && (t & 1) ? j.f2 : j.f) + smp * 9 * j.plane;
    const double u_peak = j.smp[smp].u_peak, omega = j.smp[smp].omega;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(c / j.nx), x = (int)(c - (int64_t)y * j.nx);
        uint32_t m = 0;
        if (CHANNEL) {
            m = j.mask[(int64_t)y * j.pitch + x];
            if (m & M_SOLID) {
                for (int i = 0; i < 9; ++i) out[i * cells + c] = 0.0;
                continue;
            }
        }
        const Site s = site(j, x, y);
        C f[9];
        gather<P, CHANNEL, MODE>(j, base, s, m, t, u_peak, omega, f);
        for (int i = 0; i < 9; ++i) out[i * cells + c] = (double)f[i] + wgt<double>(i);
    }
}

// ------------------------------------------------------------------ field statistics from the slab
// Statistics of a field QoI read straight from the populations, without a
// per-sample field buffer: the value of a (sample, node) is formed from its
// pulled populations exactly as k_fields forms it (velocity u_x, u_y; density
// 1 + drho; speed |u|; 0 at solid nodes), and every sum over the samples runs
// in ascending sample order with Neumaier compensation (FP64), output by
// output, so the result does not depend on the launch shape.
// Field QoIs: which = 0 velocity (two components), 1 density, 2 speed.
constexpr int FP_JB = 16;  // samples per LDS block of values
constexpr int FP_KA = 12;  // (component, coefficient) pairs per thread

template <int P, bool CHANNEL, int MODE>
__device__ inline void field_value(const JobDev &j, const typename Prec<P>::T *base, int64_t t, int64_t smp,
                                   int64_t c, int which, double &v0, double &v1) {
    using C = typename Prec<P>::C;
    const int y = (int)(c / j.nx), x = (int)(c - (int64_t)y * j.nx);
    uint32_t m = 0;
    v0 = v1 = 0.0;
    if (CHANNEL) {
        m = j.mask[(int64_t)y * j.pitch + x];
        if (m & M_SOLID) return;
    }
    C f[9], drho, ux, uy;
    gather<P, CHANNEL, MODE>(j, base, site(j, x, y), m, t, j.smp[smp].u_peak, j.smp[smp].omega, f);
    moments(f, drho, ux, uy);
    if (which == 0) {
        v0 = (double)ux;
        v1 = (double)uy;
    } else if (which == 1) {
        v0 = 1.0 + (double)drho;
    } else {
        v0 = sqrt((double)ux * (double)ux + (double)uy * (double)uy);
    }
}

// SC-gPC coefficients c_k(o) = sum_j a_j Phi_k(xi_j) M_j(o) (Eq.
// coef_discrete) of a field: a workgroup takes 64 nodes (one per lane) and
// 4 FP_KA (component, k) pairs (FP_KA per wave); per block of FP_JB samples
// the four waves form the values of the 64 nodes into LDS, then every
// thread adds its pairs' terms. coeffs[k][n_out], o = component * cells + node.
template <int P, bool CHANNEL, int MODE>
__global__ __launch_bounds__(256) void k_field_coeffs(JobDev j, int64_t t, int which,
                                                      const double *__restrict__ wphi, int K, double *coeffs) {
    using T = typename Prec<P>::T;
    __shared__ double val[FP_JB][2][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t cells = (int64_t)j.nx * j.ny;
    const int comps = which == 0 ? 2 : 1;
    const int64_t c = (int64_t)blockIdx.x * 64 + lane;
    const bool on = c < cells;
    const int npair = comps * K;
    const int p0 = (int)blockIdx.y * 4 * FP_KA + w * FP_KA;
    int kq[FP_KA], cq[FP_KA];
#pragma unroll
    for (int q = 0; q < FP_KA; ++q) {
        const int p = min(p0 + q, npair - 1);
        cq[q] = p / K;
        kq[q] = p - cq[q] * K;
    }
    const T *slab = (const T *)(MODE == AB_PULL && (t & 1) ? j.f2 : j.f);
    NSum acc[FP_KA];
    for (int64_t j0 = 0; j0 < j.S; j0 += FP_JB) {
        const int nj = (int)min((int64_t)FP_JB, j.S - j0);
#pragma unroll
        for (int i = 0; i < FP_JB / 4; ++i) {
            const int jj = w + 4 * i;
            double v0 = 0.0, v1 = 0.0;
            if (jj < nj && on)
                field_value<P, CHANNEL, MODE>(j, slab + (j0 + jj) * 9 * j.plane, t, j0 + jj, c, which, v0, v1);
            val[jj][0][lane] = v0;
            val[jj][1][lane] = v1;
        }
        __syncthreads();
        for (int jj = 0; jj < nj; ++jj) {
            const double *wr = wphi + (j0 + jj) * K;
#pragma unroll
            for (int q = 0; q < FP_KA; ++q) acc[q].add(wr[kq[q]] * val[jj][cq[q]][lane]);
        }
        __syncthreads();
    }
    if (on) {
#pragma unroll
        for (int q = 0; q < FP_KA; ++q)
            if (p0 + q < npair) coeffs[(int64_t)kq[q] * comps * cells + cq[q] * cells + c] = acc[q].val();
    }
}

// The rest of a field's statistics, one thread per node (both velocity
// components): SC (wphi != null): mean = c_0, var = sum_{k>=1} c_k^2 (Eq.
// gpc_std) and the quadrature variance sum_j a_j (M_j - mean)^2; MC: mean
// (Eq. meanMCS), var with 1/(N-1) (Eq. varMCS) and 1/N, two passes.
template <int P, bool CHANNEL, int MODE>
__global__ __launch_bounds__(256) void k_field_finish(JobDev j, int64_t t, int which, const double *__restrict__ a,
                                                      int K, const double *coeffs, double *mean, double *var,
                                                      double *var_alt) {
    using T = typename Prec<P>::T;
    const int64_t cells = (int64_t)j.nx * j.ny;
    const int comps = which == 0 ? 2 : 1;
    const int64_t n_out = comps * cells;
    const T *slab = (const T *)(MODE == AB_PULL && (t & 1) ? j.f2 : j.f);
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (int64_t)gridDim.x * blockDim.x) {
        double mu[2] = {0.0, 0.0};
        if (K > 0) {
            for (int q = 0; q < comps; ++q) {
                const int64_t o = q * cells + c;
                mu[q] = coeffs[o];
                NSum v;
                for (int k = 1; k < K; ++k) {
                    const double ck = coeffs[(int64_t)k * n_out + o];
                    v.add(ck * ck);
                }
                mean[o] = mu[q];
                var[o] = v.val();
            }
        } else {
            NSum s0, s1;
            for (int64_t smp = 0; smp < j.S; ++smp) {
                double v0, v1;
                field_value<P, CHANNEL, MODE>(j, slab + smp * 9 * j.plane, t, smp, c, which, v0, v1);
                s0.add(v0);
                s1.add(v1);
            }
            mu[0] = s0.val() / (double)j.S;
            mu[1] = s1.val() / (double)j.S;
        }
        NSum q0, q1;
        for (int64_t smp = 0; smp < j.S; ++smp) {
            double v0, v1;
            field_value<P, CHANNEL, MODE>(j, slab + smp * 9 * j.plane, t, smp, c, which, v0, v1);
            const double e0 = v0 - mu[0], e1 = v1 - mu[1];
            if (K > 0) {
                q0.add(a[smp] * e0 * e0);
                q1.add(a[smp] * e1 * e1);
            } else {
                q0.add(e0 * e0);
                q1.add(e1 * e1);
            }
        }
        const double qs[2] = {q0.val(), q1.val()};
        for (int q = 0; q < comps; ++q) {
            const int64_t o = q * cells + c;
            if (K > 0) {
                var_alt[o] = qs[q];
            } else {
                mean[o] = mu[q];
                var[o] = j.S > 1 ? qs[q] / (double)(j.S - 1) : 0.0;
                var_alt[o] = qs[q] / (double)j.S;
            }
        }
    }
}

// ------------------------------------------------------------------ scalar statistics
// A scalar QoI (one value per sample): every sum over the samples is split
// across a workgroup's 256 threads (thread r takes samples r, r + 256, ...
// in order, a compensated partial each) and the partials are combined in
// thread order by a compensated sum, so the result does not depend on
// timing. SC: workgroup k forms c_k (Eq. coef_discrete); then one workgroup
// forms mean = c_0, var = sum_{k>=1} c_k^2 and the quadrature variance. MC:
// one workgroup forms mean, var (1/(N-1)) and var_alt (1/N).
__device__ inline double block_nsum(double part, double *red) {
    red[threadIdx.x] = part;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        NSum acc;
        for (int i = 0; i < (int)blockDim.x; ++i) acc.add(red[i]);
        red[0] = acc.val();
    }
    __syncthreads();
    r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_scalar_coeffs(const double *M, int64_t S, const double *wphi, int K,
                                                       double *coeffs) {
    __shared__ double red[256];
    const int k = blockIdx.x;
    NSum acc;
    for (int64_t jx = threadIdx.x; jx < S; jx += blockDim.x) acc.add(wphi[jx * K + k] * M[jx]);
    const double v = block_nsum(acc.val(), red);
    if (threadIdx.x == 0) coeffs[k] = v;
}

__global__ __launch_bounds__(256) void k_scalar_finish(const double *M, int64_t S, const double *a, int K,
                                                       const double *coeffs, double *mean, double *var,
                                                       double *var_alt) {
    __shared__ double red[256];
    double mu;
    if (K > 0) {
        mu = coeffs[0];
    } else {
        NSum s;
        for (int64_t jx = threadIdx.x; jx < S; jx += blockDim.x) s.add(M[jx]);
        mu = block_nsum(s.val(), red) / (double)S;
    }
    NSum q;
    for (int64_t jx = threadIdx.x; jx < S; jx += blockDim.x) {
        const double e = M[jx] - mu;
        q.add(K > 0 ? a[jx] * e * e : e * e);
    }
    const double qs = block_nsum(q.val(), red);
    if (threadIdx.x == 0) {
        mean[0] = mu;
        if (K > 0) {
            NSum v;
            for (int k = 1; k < K; ++k) v.add(coeffs[k] * coeffs[k]);
            var[0] = v.val();
            var_alt[0] = qs;
        } else {
            var[0] = S > 1 ? qs / (double)(S - 1) : 0.0;
            var_alt[0] = qs / (double)S;
        }
    }
}

// ------------------------------------------------------------------ small kernels
__global__ void k_advance(int64_t *d_t, int64_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *d_t += n;
}

// out[0] = smallest s < S with qoi[4s + 3] != 0 (non-finite values in sample
// s), else S. One workgroup of 256: strided scan, then an LDS min-reduction.
__global__ __launch_bounds__(256) void k_first_bad(const double *qoi, int64_t S, int64_t *out) {
    __shared__ int64_t red[256];
    int64_t first = S;
    for (int64_t s = threadIdx.x; s < S; s += blockDim.x)
        if (qoi[4 * s + 3] != 0.0) {
            first = s;
            break;
        }
    red[threadIdx.x] = first;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = min(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// which: UQ_QOI_KE -> KE; UQ_QOI_CD / UQ_QOI_CL -> 2 F/(u_peak^2 D) with the
// sample's peak inflow velocity and rho0 = 1
__global__ void k_select(const double *qoi, const SampleDev *smp, int64_t S, int which, double dia, double u_fac,
                         double *M) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    if (which == UQ_QOI_KE) {
        M[s] = qoi[4 * s];
    } else {
        const double u = u_fac * smp[s].u_peak;
        const double F = which == UQ_QOI_CD ? qoi[4 * s + 1] : qoi[4 * s + 2];
        M[s] = 2.0 * F / (u * u * dia);
    }
}

// ------------------------------------------------------------------ launchers
// Launch a read-only state kernel (QoIs, fields, export) in the access mode
// of the job's layout and the parity of t.
#define UQ_DISPATCH_P(KERNEL, PP, MODE_, CH_, GRID, BLOCK, STREAM, ...)                               \
    do {                                                                                           \
        if (CH_) {                                                                                 \
            if (MODE_ == AA_EVEN) KERNEL<PP, true, AA_EVEN><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);  \
            else if (MODE_ == AA_ODD) KERNEL<PP, true, AA_ODD><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__); \
            else KERNEL<PP, true, AB_PULL><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);               \
        } else {                                                                                   \
            if (MODE_ == AA_EVEN) KERNEL<PP, false, AA_EVEN><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__); \
            else if (MODE_ == AA_ODD) KERNEL<PP, false, AA_ODD><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__); \
            else KERNEL<PP, false, AB_PULL><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);              \
        }                                                                                          \
    } while (0)

#define UQ_DISPATCH(KERNEL, PARITY, GRID, BLOCK, STREAM, ...)                                      \
    do {                                                                                           \
        const int md_ = j.layout == UQ_LAYOUT_AB ? AB_PULL : ((PARITY) ? AA_ODD : AA_EVEN);        \
        const bool ch_ = j.geom == 1;                                                              \
        switch (j.prec) {                                                                          \
            case UQ_FP64: UQ_DISPATCH_P(KERNEL, UQ_FP64, md_, ch_, GRID, BLOCK, STREAM, __VA_ARGS__); break;   \
            case UQ_FP32: UQ_DISPATCH_P(KERNEL, UQ_FP32, md_, ch_, GRID, BLOCK, STREAM, __VA_ARGS__); break;   \
            case UQ_FP16S: UQ_DISPATCH_P(KERNEL, UQ_FP16S, md_, ch_, GRID, BLOCK, STREAM, __VA_ARGS__); break; \
            default: UQ_DISPATCH_P(KERNEL, UQ_BF16S, md_, ch_, GRID, BLOCK, STREAM, __VA_ARGS__); break;       \
        }                                                                                          \
    } while (0)

hipError_t launch_init(const JobDev &j, hipStream_t s) {
    const int64_t cells = (int64_t)j.ny * j.pitch;
    dim3 grid((unsigned)std::min<int64_t>((cells + 255) / 256, 1024), (unsigned)std::min<int64_t>(j.S, 65535));
    const bool ab = j.layout == UQ_LAYOUT_AB;
    switch (j.prec) {
        case UQ_FP64:
            if (ab) k_init<UQ_FP64, UQ_LAYOUT_AB><<<grid, 256, 0, s>>>(j);
            else k_init<UQ_FP64, UQ_LAYOUT_AA><<<grid, 256, 0, s>>>(j);
            break;
        case UQ_FP32:
            if (ab) k_init<UQ_FP32, UQ_LAYOUT_AB><<<grid, 256, 0, s>>>(j);
            else k_init<UQ_FP32, UQ_LAYOUT_AA><<<grid, 256, 0, s>>>(j);
            break;
        case UQ_FP16S:
            if (ab) k_init<UQ_FP16S, UQ_LAYOUT_AB><<<grid, 256, 0, s>>>(j);
            else k_init<UQ_FP16S, UQ_LAYOUT_AA><<<grid, 256, 0, s>>>(j);
            break;
        default:
            if (ab) k_init<UQ_BF16S, UQ_LAYOUT_AB><<<grid, 256, 0, s>>>(j);
            else k_init<UQ_BF16S, UQ_LAYOUT_AA><<<grid, 256, 0, s>>>(j);
            break;
    }
    return hipGetLastError();
}

template <int P, bool CH, int CPT>
static void step_p(const JobDev &j, const int64_t *d_t, int k, int parity, bool nt, dim3 grid, dim3 block,
                   hipStream_t s, int tiles_x, int tiles_y, int64_t ntiles) {
#define UQ_STEP(PAR, LAY, NT_) k_step<P, CH, PAR, CPT, LAY, NT_><<<grid, block, 0, s>>>(j, d_t, k, tiles_x, tiles_y, ntiles)
    if (j.layout == UQ_LAYOUT_AB) {
        if (nt) { if (parity) UQ_STEP(1, UQ_LAYOUT_AB, true); else UQ_STEP(0, UQ_LAYOUT_AB, true); }
        else { if (parity) UQ_STEP(1, UQ_LAYOUT_AB, false); else UQ_STEP(0, UQ_LAYOUT_AB, false); }
    } else {
        if (parity) UQ_STEP(1, UQ_LAYOUT_AA, false); else UQ_STEP(0, UQ_LAYOUT_AA, false);
    }
#undef UQ_STEP
}

template <int CPT>
static void step_cpt(const JobDev &j, const int64_t *d_t, int k, int parity, bool nt, dim3 grid, dim3 block,
                     hipStream_t s, int tiles_x, int tiles_y, int64_t ntiles) {
    const bool ch = j.geom == 1;
    switch (j.prec) {
        case UQ_FP64:
            if (ch) step_p<UQ_FP64, true, CPT>(j, d_t, k, parity, nt, grid, block, s, tiles_x, tiles_y, ntiles);
            else step_p<UQ_FP64, false, CPT>(j, d_t, k, parity, nt, grid, block, s, tiles_x, tiles_y, ntiles);
            break;
        case UQ_FP32:
            if (ch) step_p<UQ_FP32, true, CPT>(j, d_t, k, parity, nt, grid, block, s, tiles_x, tiles_y, ntiles);
            else step_p<UQ_FP32, false, CPT>(j, d_t, k, parity, nt, grid, block, s, tiles_x, tiles_y, ntiles);
            break;
        case UQ_FP16S:
            if (ch) step_p<UQ_FP16S, true, CPT>(j, d_t, k, parity, nt, grid, block, s, tiles_x, tiles_y, ntiles);
            else step_p<UQ_FP16S, false, CPT>(j, d_t, k, parity, nt, grid, block, s, tiles_x, tiles_y, ntiles);
            break;
        default:
            if (ch) step_p<UQ_BF16S, true, CPT>(j, d_t, k, parity, nt, grid, block, s, tiles_x, tiles_y, ntiles);
            else step_p<UQ_BF16S, false, CPT>(j, d_t, k, parity, nt, grid, block, s, tiles_x, tiles_y, ntiles);
            break;
    }
}

hipError_t launch_step(const JobDev &j, const int64_t *d_t, int k, int parity, const StepShape &shape,
                       hipStream_t s_main, const SideStream *side) {
    const int cpt = shape.cpt <= 1 ? 1 : 2;
    const int bx = shape.bx == 128 || shape.bx == 256 ? shape.bx : BX;
    const int by = 256 / bx;
    const int tiles_x = (j.nx + bx - 1) / bx;
    const int tiles_y = (j.ny + by * cpt - 1) / (by * cpt);
    const int64_t ntiles = (int64_t)j.S * tiles_x * tiles_y;
    int64_t G = ntiles;
    if (shape.persistent > 0) G = std::min<int64_t>(ntiles, (int64_t)256 * shape.persistent);
    if (G > 0x7fffffff) G = 0x7fffffff;
    dim3 block(bx, by);
    dim3 grid((unsigned)G);
    const bool nt = shape.nt != 0;
    const bool odd = parity & 1;
    const unsigned gs = (unsigned)std::min<int64_t>(j.S, 65535);
    const bool fd_cols = j.geom == 1 && j.xbc == UQ_XBC_INTERP && j.layout == UQ_LAYOUT_AB;
    // boundary-node kernels: on the side stream when there is one
    hipStream_t s = s_main;
    if ((j.n_special > 0 || fd_cols) && side && side->stream) {
        hipError_t e = hipEventRecord(side->fork, s_main);
        if (e == hipSuccess) e = hipStreamWaitEvent(side->stream, side->fork, 0);
        if (e != hipSuccess) return e;
        s = side->stream;
    }
    if (j.n_special > 0) {
        dim3 og((unsigned)((j.n_special + 63) / 64), gs);
#define UQ_QL(PP)                                                        \
    do {                                                                 \
        if (odd) k_qlinks<PP, 1><<<og, 64, 0, s>>>(j, d_t, k);           \
        else k_qlinks<PP, 0><<<og, 64, 0, s>>>(j, d_t, k);               \
    } while (0)
        switch (j.prec) {
            case UQ_FP64: UQ_QL(UQ_FP64); break;
            case UQ_FP32: UQ_QL(UQ_FP32); break;
            case UQ_FP16S: UQ_QL(UQ_FP16S); break;
            default: UQ_QL(UQ_BF16S); break;
        }
#undef UQ_QL
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (fd_cols) {
        dim3 fg((unsigned)(2 * ((j.ny + FD_ROWS - 1) / FD_ROWS)), gs);
#define UQ_FDC(PP)                                                                  \
    do {                                                                            \
        if (odd) k_fd_columns<PP, 1><<<fg, FD_BLOCK, 0, s>>>(j, d_t, k);             \
        else k_fd_columns<PP, 0><<<fg, FD_BLOCK, 0, s>>>(j, d_t, k);                 \
    } while (0)
        switch (j.prec) {
            case UQ_FP64: UQ_FDC(UQ_FP64); break;
            case UQ_FP32: UQ_FDC(UQ_FP32); break;
            case UQ_FP16S: UQ_FDC(UQ_FP16S); break;
            default: UQ_FDC(UQ_BF16S); break;
        }
#undef UQ_FDC
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (cpt == 1) step_cpt<1>(j, d_t, k, parity & 1, nt, grid, block, s_main, tiles_x, tiles_y, ntiles);
    else step_cpt<2>(j, d_t, k, parity & 1, nt, grid, block, s_main, tiles_x, tiles_y, ntiles);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && s != s_main) {
        e = hipEventRecord(side->join, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(s_main, side->join, 0);
    }
    return e;
}

hipError_t launch_step_multi(const MultiJob *jobs, int njobs, int64_t ntiles, int k, int prec, hipStream_t s) {
    if (ntiles <= 0 || njobs <= 0) return hipSuccess;
    const int64_t G = std::min<int64_t>(ntiles, 0x7fffffff);
    dim3 block(BX, BY);
    switch (prec) {
        case UQ_FP64: k_step_multi<UQ_FP64><<<(unsigned)G, block, 0, s>>>(jobs, njobs, ntiles, k); break;
        case UQ_FP32: k_step_multi<UQ_FP32><<<(unsigned)G, block, 0, s>>>(jobs, njobs, ntiles, k); break;
        case UQ_FP16S: k_step_multi<UQ_FP16S><<<(unsigned)G, block, 0, s>>>(jobs, njobs, ntiles, k); break;
        default: k_step_multi<UQ_BF16S><<<(unsigned)G, block, 0, s>>>(jobs, njobs, ntiles, k); break;
    }
    return hipGetLastError();
}

hipError_t launch_advance_multi(MultiJob *jobs, int njobs, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    k_advance_multi<<<(unsigned)((njobs + 63) / 64), 64, 0, s>>>(jobs, njobs);
    return hipGetLastError();
}

bool fused_supported(const JobDev &j) {
    // periodic AB jobs whose per-sample slab fits one buffer descriptor's range
    const int64_t b = j.prec == UQ_FP64 ? 8 : (j.prec == UQ_FP32 ? 4 : 2);
    return j.geom == 0 && j.layout == UQ_LAYOUT_AB && 9 * j.plane * b < ((int64_t)1 << 31);
}

template <int P, int N>
static void stepN_p(const JobDev &j, bool src2, int fty, hipStream_t s) {
    const int tiles_x = (j.nx + FUSE_TX - 1) / FUSE_TX;
    auto go = [&](auto ty_c) {
        constexpr int TY = decltype(ty_c)::value;
        const int tiles_y = (j.ny + TY - 1) / TY;
        const int64_t ntiles = (int64_t)j.S * tiles_x * tiles_y;
        const int64_t G = std::min<int64_t>(ntiles, 0x7fffffff);
        k_stepN<P, TY, N><<<(unsigned)G, 256, 0, s>>>(j, src2, tiles_x, tiles_y, ntiles);
    };
    // FP64 tiles are half as tall (the LDS tile holds doubles)
    if constexpr (P == UQ_FP64) {
        if (fty <= 4) go(std::integral_constant<int, 4>());
        else go(std::integral_constant<int, 8>());
    } else {
        if (fty <= 8) go(std::integral_constant<int, 8>());
        else go(std::integral_constant<int, 16>());
    }
}

// strips of at most 64 - 2(N - 1) columns (a wave's 64 lanes less the ring
// of N - 1 columns per side), balanced
void window_strips(int nx, int n, int *W, int *strips) {
    const int wmax = 64 - 2 * (n - 1);
    *strips = (nx + wmax - 1) / wmax;
    *W = (nx + *strips - 1) / *strips;
}

template <int P, int N>
static void stepW_p(const JobDev &j, bool src2, int rows, bool nt, hipStream_t s) {
    int W, strips;
    window_strips(j.nx, N, &W, &strips);
    const int H = std::max(8, std::min(rows, j.ny));
    const int chunks = (j.ny + H - 1) / H;
    const int64_t nwork = (int64_t)j.S * strips * chunks;
    const int64_t G = std::min<int64_t>(nwork, 0x7fffffff);
    // rows of loads in flight: 3 (2 at FP64, whose registers are scarcer)
    constexpr int D = P == UQ_FP64 ? 2 : 3;
    k_stepW<P, N, D><<<(unsigned)G, 64 * N, 0, s>>>(j, src2, W, strips, H, chunks, nwork, nt);
}

// full-row kernel: K waves per level of M columns per lane cover nx, with
// N K <= 16 waves and (N - 1) 27 LDS rows of 64 K M + 2 values within 160 KB
template <int P, int N, int K, int M>
static void stepR_k(const JobDev &j, bool src2, int rows, bool nt, hipStream_t s) {
    const int H = std::max(8, std::min(rows, j.ny));
    const int chunks = (j.ny + H - 1) / H;
    const int64_t nwork = (int64_t)j.S * chunks;
    const int64_t G = std::min<int64_t>(nwork, 0x7fffffff);
    k_stepR<P, N, K, M, 2><<<(unsigned)G, 64 * N * K, 0, s>>>(j, src2, H, chunks, nwork, nt);
}

// Shapes of the full-row kernels: K waves per level of M columns per lane
// (K <= 4 with one column, <= 6 with two: rows up to 768 columns), N K <= 16
// waves, and (N - 1) LDS rings of ROWS direction-rows (21 on the periodic
// lattice, 30 on the channel) of about 64 K M compute values within 160 KB.
// The shape used for a lattice nx wide: the fewest columns per lane (M = 1,
// else 2) whose K = ceil(nx / 64 M) fits; 0 if none.
static constexpr int RING_ROWS_TGV = 21, RING_ROWS_CH = 30;

// Registers: in single precision a lane of the periodic kernel colliding two
// columns fits 128 VGPRs (4 waves per SIMD: up to 16 waves), the channel
// kernel's about 165 (12 waves, 3 per SIMD); in double precision two columns
// keep to 8 waves (256 VGPRs) and one column to 12 (168). One column per
// lane fits 128 in single precision. (__launch_bounds__ holds the compiler to
// the budget of the workgroup size, so these limits only keep out shapes
// that would spill.)
static constexpr bool rows_regs_fit(int prec, int waves, int M, bool channel) {
    return prec == UQ_FP64 ? waves <= (M == 2 ? 8 : 12) : (M == 2 && channel ? waves <= 12 : true);
}

// values per LDS row: the periodic kernel's rows hold its 64 K M columns
// (shifted writes wrap inside the row); the channel's also two end columns,
// padded to a multiple of 64
static constexpr int ring_cols(int rows, int K, int M) { return 64 * K * M + (rows == RING_ROWS_CH ? 64 : 0); }

static constexpr bool rows_fit(int prec, int n, int rows, int K, int M) {
    return n * K <= 16 && K <= (M == 2 ? 6 : 4) && rows_regs_fit(prec, n * K, M, rows == RING_ROWS_CH) &&
           (int64_t)(n - 1) * rows * ring_cols(rows, K, M) * (prec == UQ_FP64 ? 8 : 4) <= 160 * 1024;
}

static int rows_shape(int prec, int n, int rows, int nx, int *K, int *M) {
    for (int m = 1; m <= 2; ++m) {
        const int k = std::max(2, (nx + 64 * m - 1) / (64 * m));
        if (rows_fit(prec, n, rows, k, m)) {
            *K = k;
            *M = m;
            return 1;
        }
    }
    return 0;
}

static int rows_max_nx(int prec, int n, int rows) {
    int best = 0;
    for (int nx = 64; nx <= 768; nx += 64) {
        int K, M;
        if (rows_shape(prec, n, rows, nx, &K, &M)) best = nx;
    }
    return best;
}

int full_rows_max_nx(int prec, int n) { return rows_max_nx(prec, n, RING_ROWS_TGV); }
int channel_rows_max_nx(int prec, int n) { return rows_max_nx(prec, n, RING_ROWS_CH); }

// the instances (K, M) a launcher may take
#define UQ_ROWS_CASES(CASE) \
    CASE(2, 1) CASE(3, 1) CASE(4, 1) CASE(2, 2) CASE(3, 2) CASE(4, 2) CASE(5, 2) CASE(6, 2)

template <int P, int N>
static void stepR_p(const JobDev &j, bool src2, int rows, bool nt, hipStream_t s) {
    int K = 0, M = 0;
    if (!rows_shape(P, N, RING_ROWS_TGV, j.nx, &K, &M)) return;
#define UQ_ROWS_CASE(kk, mm)                                                      \
    if constexpr (rows_fit(P, N, RING_ROWS_TGV, kk, mm)) {                        \
        if (K == kk && M == mm) return stepR_k<P, N, kk, mm>(j, src2, rows, nt, s); \
    }
    UQ_ROWS_CASES(UQ_ROWS_CASE)
#undef UQ_ROWS_CASE
}

bool channel_fusable(const JobDev &j) {
    const int64_t b = j.prec == UQ_FP64 ? 8 : (j.prec == UQ_FP32 ? 4 : 2);
    return j.geom == 1 && j.layout == UQ_LAYOUT_AB && j.n_special == 0 && j.q == nullptr &&
           j.xbc != UQ_XBC_INTERP && 9 * j.plane * b < ((int64_t)1 << 31) && j.plane * 4 < ((int64_t)1 << 31);
}

template <int P, int N, int K, int M>
static void stepRC_k(const JobDev &j, const int64_t *d_t, int k, bool src2, int rows, hipStream_t s) {
    const int H = std::max(8, std::min(rows, j.ny));
    const int chunks = (j.ny + H - 1) / H;
    const int64_t nwork = (int64_t)j.S * chunks;
    const int64_t G = std::min<int64_t>(nwork, 0x7fffffff);
    k_stepRC<P, N, K, M, 2><<<(unsigned)G, 64 * N * K, 0, s>>>(j, d_t, k, src2, H, chunks, nwork);
}

template <int P, int N>
static void stepRC_p(const JobDev &j, const int64_t *d_t, int k, bool src2, int rows, hipStream_t s) {
    int K = 0, M = 0;
    if (!rows_shape(P, N, RING_ROWS_CH, j.nx, &K, &M)) return;
#define UQ_ROWS_CASE(kk, mm)                                                              \
    if constexpr (rows_fit(P, N, RING_ROWS_CH, kk, mm)) {                                 \
        if (K == kk && M == mm) return stepRC_k<P, N, kk, mm>(j, d_t, k, src2, rows, s);  \
    }
    UQ_ROWS_CASES(UQ_ROWS_CASE)
#undef UQ_ROWS_CASE
}

// ------------------------------------------------------------------ batched fused launches
// One launch of a batched fused instance (kind 0: periodic rows,
// k_stepR_multi; kind 1: channel rows, k_stepRC_multi; kind 2: periodic
// strips, k_stepW_multi): every work item of the table's jobs. The server
// keeps to N in {4, 6, 8} (periodic rows), {2, 3, 4} (channel) and 4 (strips)
// and to single precision storage (FP32, FP16S, BF16S), so that a tick of 48
// steps holds a whole number of launch pairs of every instance.
int rows_instance(int kind, int prec, int n, int nx, int *K, int *M) {
    if (kind == 2) {  // strips: any width
        *K = *M = 0;
        return 1;
    }
    return rows_shape(prec, n, kind == 0 ? RING_ROWS_TGV : RING_ROWS_CH, nx, K, M);
}

template <int P, int N, int K, int M>
static void multi_k(int kind, const FusedJob *jobs, int njobs, int64_t nwork, int launch, hipStream_t s) {
    const int64_t G = std::min<int64_t>(nwork, 0x7fffffff);
    if (kind == 0) {
        if constexpr (rows_fit(P, N, RING_ROWS_TGV, K, M))
            k_stepR_multi<P, N, K, M, 2><<<(unsigned)G, 64 * N * K, 0, s>>>(jobs, njobs, nwork, launch, false);
    } else {
        if constexpr (N <= 4 && rows_fit(P, N, RING_ROWS_CH, K, M))
            k_stepRC_multi<P, N, K, M, 2><<<(unsigned)G, 64 * N * K, 0, s>>>(jobs, njobs, nwork, launch);
    }
}

template <int P, int N>
static bool multi_n(int kind, int K, int M, const FusedJob *jobs, int njobs, int64_t nwork, int launch,
                    hipStream_t s) {
#define UQ_MULTI_CASE(kk, mm)                                         \
    if (K == kk && M == mm) {                                         \
        multi_k<P, N, kk, mm>(kind, jobs, njobs, nwork, launch, s);   \
        return true;                                                  \
    }
    UQ_ROWS_CASES(UQ_MULTI_CASE)
#undef UQ_MULTI_CASE
    return false;
}

template <int P>
static bool multi_p(int kind, int n, int K, int M, const FusedJob *jobs, int njobs, int64_t nwork, int launch,
                    hipStream_t s) {
    if (kind == 2) {
        if (n != 4) return false;
        const int64_t G = std::min<int64_t>(nwork, 0x7fffffff);
        k_stepW_multi<P, 4, 3><<<(unsigned)G, 256, 0, s>>>(jobs, njobs, nwork, launch);
        return true;
    }
    if (kind == 0) {
        if (n == 4) return multi_n<P, 4>(0, K, M, jobs, njobs, nwork, launch, s);
        if (n == 6) return multi_n<P, 6>(0, K, M, jobs, njobs, nwork, launch, s);
        if (n == 8) return multi_n<P, 8>(0, K, M, jobs, njobs, nwork, launch, s);
        return false;
    }
    if (n == 2) return multi_n<P, 2>(1, K, M, jobs, njobs, nwork, launch, s);
    if (n == 3) return multi_n<P, 3>(1, K, M, jobs, njobs, nwork, launch, s);
    if (n == 4) return multi_n<P, 4>(1, K, M, jobs, njobs, nwork, launch, s);
    return false;
}

bool fused_multi_supported(int kind, int prec, int n, int K, int M) {
    if (prec == UQ_FP64) return false;
    if (kind == 2) return n == 4;
    if (kind == 0 ? (n != 4 && n != 6 && n != 8) : (n < 2 || n > 4)) return false;
    return rows_fit(prec, n, kind == 0 ? RING_ROWS_TGV : RING_ROWS_CH, K, M);
}

hipError_t launch_fused_multi(int kind, int prec, int n, int K, int M, const FusedJob *jobs, int njobs,
                              int64_t nwork, int launch, hipStream_t s) {
    if (njobs <= 0 || nwork <= 0) return hipSuccess;
    if (!fused_multi_supported(kind, prec, n, K, M)) return hipErrorInvalidValue;
    bool ok = false;
    switch (prec) {
        case UQ_FP32: ok = multi_p<UQ_FP32>(kind, n, K, M, jobs, njobs, nwork, launch, s); break;
        case UQ_FP16S: ok = multi_p<UQ_FP16S>(kind, n, K, M, jobs, njobs, nwork, launch, s); break;
        default: ok = multi_p<UQ_BF16S>(kind, n, K, M, jobs, njobs, nwork, launch, s); break;
    }
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

// *d_t[q] += n for every job of a table (one thread per job)
__global__ void k_advance_ptrs(int64_t *const *d_t, int njobs, int64_t n) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < njobs) *d_t[q] += n;
}

hipError_t launch_advance_ptrs(int64_t *const *d_t, int njobs, int64_t n, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    k_advance_ptrs<<<(unsigned)((njobs + 63) / 64), 64, 0, s>>>(d_t, njobs, n);
    return hipGetLastError();
}

#undef UQ_ROWS_CASES

template <int P>
static void fused_ch_p(const JobDev &j, int n, const int64_t *d_t, int k, bool src2, int fty, hipStream_t s) {
    if (n == 2) stepRC_p<P, 2>(j, d_t, k, src2, fty, s);
    else if (n == 3) stepRC_p<P, 3>(j, d_t, k, src2, fty, s);
    else stepRC_p<P, 4>(j, d_t, k, src2, fty, s);
}

template <int P>
static void fused_p(const JobDev &j, int n, bool src2, int fty, int window, bool nt, hipStream_t s) {
    if (window == 2) {
        if (n == 2) stepR_p<P, 2>(j, src2, fty, nt, s);
        else if (n == 3) stepR_p<P, 3>(j, src2, fty, nt, s);
        else if (n == 4) stepR_p<P, 4>(j, src2, fty, nt, s);
        else if (n == 5) stepR_p<P, 5>(j, src2, fty, nt, s);
        else if (n == 6) stepR_p<P, 6>(j, src2, fty, nt, s);
        else if (n == 7) stepR_p<P, 7>(j, src2, fty, nt, s);
        else stepR_p<P, 8>(j, src2, fty, nt, s);
    } else if (window) {
        if (n == 2) stepW_p<P, 2>(j, src2, fty, nt, s);
        else if (n == 3) stepW_p<P, 3>(j, src2, fty, nt, s);
        else stepW_p<P, 4>(j, src2, fty, nt, s);
    } else {
        if (n == 2) stepN_p<P, 2>(j, src2, fty, s);
        else if (n == 3) stepN_p<P, 3>(j, src2, fty, s);
        else stepN_p<P, 4>(j, src2, fty, s);
    }
}

hipError_t launch_fused(const JobDev &j, int n, bool src2, int fty, int window, bool nt, const int64_t *d_t, int k,
                        hipStream_t s) {
    if (j.geom == 1) {
        if (!channel_fusable(j) || window != 2 || n < 2 || n > 4 || j.nx > channel_rows_max_nx(j.prec, n))
            return hipErrorInvalidValue;
        switch (j.prec) {
            case UQ_FP64: fused_ch_p<UQ_FP64>(j, n, d_t, k, src2, fty, s); break;
            case UQ_FP32: fused_ch_p<UQ_FP32>(j, n, d_t, k, src2, fty, s); break;
            case UQ_FP16S: fused_ch_p<UQ_FP16S>(j, n, d_t, k, src2, fty, s); break;
            default: fused_ch_p<UQ_BF16S>(j, n, d_t, k, src2, fty, s); break;
        }
        return hipGetLastError();
    }
    if (!fused_supported(j) || n < 2 || n > (window == 2 ? 8 : 4)) return hipErrorInvalidValue;
    if (window == 2 && j.nx > full_rows_max_nx(j.prec, n)) return hipErrorInvalidValue;
    switch (j.prec) {
        case UQ_FP64: fused_p<UQ_FP64>(j, n, src2, fty, window, nt, s); break;
        case UQ_FP32: fused_p<UQ_FP32>(j, n, src2, fty, window, nt, s); break;
        case UQ_FP16S: fused_p<UQ_FP16S>(j, n, src2, fty, window, nt, s); break;
        default: fused_p<UQ_BF16S>(j, n, src2, fty, window, nt, s); break;
    }
    return hipGetLastError();
}

void tile_counts(const JobDev &j, int cpt, int *tiles_x, int *tiles_y) {
    *tiles_x = (j.nx + BX - 1) / BX;
    *tiles_y = (j.ny + BY * cpt - 1) / (BY * cpt);
}

hipError_t launch_advance(int64_t *d_t, int64_t n, hipStream_t s) {
    k_advance<<<1, 64, 0, s>>>(d_t, n);
    return hipGetLastError();
}

hipError_t launch_select_scalar(const JobDev &j, const double *qoi, int which, double *M, hipStream_t s) {
    k_select<<<(unsigned)((j.S + 255) / 256), 256, 0, s>>>(qoi, j.smp, j.S, which, j.dia, j.u_fac, M);
    return hipGetLastError();
}

hipError_t launch_first_bad(const double *qoi, int64_t S, int64_t *out, hipStream_t s) {
    k_first_bad<<<1, 256, 0, s>>>(qoi, S, out);
    return hipGetLastError();
}

hipError_t launch_qoi_scalars(const JobDev &j, int64_t t, double *out, hipStream_t s) {
    dim3 grid((unsigned)j.S);
    UQ_DISPATCH(k_qoi, t & 1, grid, 256, s, j, t, out);
    return hipGetLastError();
}

hipError_t launch_fields(const JobDev &j, int64_t t, double *out, hipStream_t s) {
    const int64_t cells = (int64_t)j.nx * j.ny;
    dim3 grid((unsigned)std::min<int64_t>((cells + 255) / 256, 4096), (unsigned)std::min<int64_t>(j.S, 65535));
    UQ_DISPATCH(k_fields, t & 1, grid, 256, s, j, t, out);
    return hipGetLastError();
}

hipError_t launch_field_moments(const JobDev &j, int64_t t, int qoi, const double *wphi, const double *a, int K,
                                double *coeffs, double *mean, double *var, double *var_alt, hipStream_t s) {
    const int which = qoi == UQ_QOI_VEL ? 0 : (qoi == UQ_QOI_RHO ? 1 : 2);
    const int64_t cells = (int64_t)j.nx * j.ny;
    if (K > 0) {
        const int npair = (which == 0 ? 2 : 1) * K;
        dim3 grid((unsigned)((cells + 63) / 64), (unsigned)((npair + 4 * FP_KA - 1) / (4 * FP_KA)));
        UQ_DISPATCH(k_field_coeffs, t & 1, grid, 256, s, j, t, which, wphi, K, coeffs);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    dim3 grid2((unsigned)std::min<int64_t>((cells + 255) / 256, 65535));
    UQ_DISPATCH(k_field_finish, t & 1, grid2, 256, s, j, t, which, a, K, coeffs, mean, var, var_alt);
    return hipGetLastError();
}

hipError_t launch_scalar_moments(const double *M, int64_t S, const double *wphi, const double *a, int K,
                                 double *coeffs, double *mean, double *var, double *var_alt, hipStream_t s) {
    if (K > 0) {
        k_scalar_coeffs<<<(unsigned)K, 256, 0, s>>>(M, S, wphi, K, coeffs);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    k_scalar_finish<<<1, 256, 0, s>>>(M, S, a, K, coeffs, mean, var, var_alt);
    return hipGetLastError();
}

hipError_t launch_export(const JobDev &j, int64_t t, int64_t sample, double *out, hipStream_t s) {
    const int64_t cells = (int64_t)j.nx * j.ny;
    dim3 grid((unsigned)std::min<int64_t>((cells + 255) / 256, 4096));
    UQ_DISPATCH(k_export, t & 1, grid, 256, s, j, t, sample, out);
    return hipGetLastError();
}

}  // namespace uqi
