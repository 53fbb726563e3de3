// Host side of the UQ layer: validation, collocation / Monte Carlo sample
// sets, the orthonormal Legendre basis and the mapping of reference
// variables to solver inputs (Sec. "Uncertainty quantification methods" and
// "Core class design" of OpenLB-UQ, arXiv 2508.13867).
#include <cmath>
#include <cstring>
#include <string>

#include "uq_internal.h"

namespace uqi {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }
uq_status fail(uq_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

}  // namespace uqi

extern "C" const char *uq_last_error(void) { return uqi::g_err.c_str(); }

namespace uqi {

// ------------------------------------------------------------------ validation
uq_status validate_problem(const uq_problem &p) {
    if (p.geometry != UQ_GEOM_TGV && p.geometry != UQ_GEOM_CHANNEL) return fail(UQ_EINVAL, "unknown geometry");
    if (p.precision < UQ_FP64 || p.precision > UQ_BF16S) return fail(UQ_EINVAL, "unknown precision");
    if (p.nx < 2 || p.ny < 2) return fail(UQ_EINVAL, "nx and ny must be >= 2");
    if (p.geometry == UQ_GEOM_CHANNEL && p.ny < 3) return fail(UQ_EINVAL, "channel needs ny >= 3");
    if ((int64_t)p.nx * p.ny > (int64_t)1 << 30) return fail(UQ_EINVAL, "lattice too large");
    if (p.n_dists < 0 || p.n_dists > UQ_MAX_DIMS) return fail(UQ_EINVAL, "n_dists out of range");
    if (p.geometry == UQ_GEOM_CHANNEL) {
        if (p.xbc < UQ_XBC_ZOUHE || p.xbc > UQ_XBC_PERIODIC) return fail(UQ_EINVAL, "unknown xbc");
        if (p.D < 0) return fail(UQ_EINVAL, "D must be >= 0");
        if (p.ramp < 0) return fail(UQ_EINVAL, "ramp must be >= 0");
    }
    for (int k = 0; k < p.n_dists; ++k) {
        const uq_dist &q = p.dists[k];
        if (q.target < UQ_T_NU || q.target > UQ_T_U_PEAK) return fail(UQ_EINVAL, "unknown target");
        if (!(q.hi >= q.lo) || !std::isfinite(q.lo) || !std::isfinite(q.hi))
            return fail(UQ_EINVAL, "distribution needs finite lo <= hi");
        bool tgv_only = q.target == UQ_T_U0 || q.target == UQ_T_PHASE_X || q.target == UQ_T_PHASE_Y;
        bool ch_only = q.target == UQ_T_RE || q.target == UQ_T_U_PEAK;
        if (tgv_only && p.geometry != UQ_GEOM_TGV) return fail(UQ_EINVAL, "target applies to the TGV only");
        if (ch_only && p.geometry != UQ_GEOM_CHANNEL) return fail(UQ_EINVAL, "target applies to the channel only");
        if (q.target == UQ_T_RE && !(q.lo > 0)) return fail(UQ_EINVAL, "Re must be positive");
        for (int m = 0; m < k; ++m)
            if (p.dists[m].target == q.target) return fail(UQ_EINVAL, "each target may be driven once");
    }
    if (p.rule == UQ_RULE_GL_TENSOR) {
        if (p.n_dists < 1) return fail(UQ_EINVAL, "collocation needs at least one uncertain input");
        if (p.n_per_dim < 1 || p.n_per_dim > 64) return fail(UQ_EINVAL, "n_per_dim must be in [1, 64]");
        if (p.order < 0 || p.order > 32) return fail(UQ_EINVAL, "order must be in [0, 32]");
        double S = std::pow((double)p.n_per_dim, p.n_dists);
        if (S > 1e7) return fail(UQ_EINVAL, "tensor rule too large");
    } else if (p.rule == UQ_RULE_MC) {
        if (p.n_dists < 1) return fail(UQ_EINVAL, "Monte Carlo needs at least one uncertain input");
        if (p.mc_n < 2 || p.mc_n > 10000000) return fail(UQ_EINVAL, "mc_n must be in [2, 1e7]");
    } else {
        return fail(UQ_EINVAL, "unknown rule");
    }
    return UQ_OK;
}

// ------------------------------------------------------------------ Gauss-Legendre
// Nodes: eigenvalues of the symmetric tridiagonal Jacobi matrix of the
// Legendre weight (zero diagonal, off-diagonal b_k = k / sqrt(4k^2 - 1)),
// found by Sturm-sequence bisection (Golub & Welsch 1969 set the problem up
// this way). Weights of the probability measure dx/2: Christoffel numbers
// lambda = 1 / sum_{m<n} p_m(x)^2 with p_m orthonormal under dx/2.
static double jacobi_b(int k) { return k / std::sqrt(4.0 * k * k - 1.0); }

// number of eigenvalues of the n x n Jacobi matrix that are < x
static int sturm_count(int n, double x) {
    int c = 0;
    double q = -x;  // d_1 = a_1 - x, a = 0
    if (q < 0) ++c;
    for (int k = 1; k < n; ++k) {
        double b = jacobi_b(k);
        if (q == 0.0) q = 1e-300;
        q = -x - b * b / q;
        if (q < 0) ++c;
    }
    return c;
}

// orthonormal Legendre polynomials under dx/2 by the Jacobi recurrence
// b_{m+1} p_{m+1} = x p_m - b_m p_{m-1}, p_0 = 1
static void ortho_legendre_all(int nmax, double x, double *p) {
    p[0] = 1.0;
    if (nmax >= 1) p[1] = x / jacobi_b(1);
    for (int m = 1; m < nmax; ++m) p[m + 1] = (x * p[m] - jacobi_b(m) * p[m - 1]) / jacobi_b(m + 1);
}

static void gauss_legendre_prob(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    std::vector<double> p(n + 1);
    for (int k = 0; k < n; ++k) {
        // k-th smallest eigenvalue: smallest x with sturm_count(x) > k
        double lo = -1.0, hi = 1.0;
        for (int it = 0; it < 200; ++it) {
            double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            if (sturm_count(n, mid) > k)
                hi = mid;
            else
                lo = mid;
        }
        x[k] = 0.5 * (lo + hi);
        ortho_legendre_all(n - 1, x[k], p.data());
        double s = 0.0;
        for (int m = 0; m < n; ++m) s += p[m] * p[m];
        w[k] = 1.0 / s;
    }
    // symmetric rule: enforce exact antisymmetry of the nodes
    for (int k = 0; k < n / 2; ++k) {
        double v = 0.5 * (x[n - 1 - k] - x[k]);
        double ww = 0.5 * (w[k] + w[n - 1 - k]);
        x[k] = -v;
        x[n - 1 - k] = v;
        w[k] = w[n - 1 - k] = ww;
    }
    if (n % 2) x[n / 2] = 0.0;
}

// ------------------------------------------------------------------ multi-indices
// total degree <= P, graded: degree ascending; within one degree the
// multi-indices in descending lexicographic order (alpha_0 most significant)
static void compositions(int d, int left, int pos, std::vector<int32_t> &cur, std::vector<int32_t> &out) {
    if (pos == d - 1) {
        cur[pos] = left;
        out.insert(out.end(), cur.begin(), cur.end());
        return;
    }
    for (int v = left; v >= 0; --v) {
        cur[pos] = v;
        compositions(d, left - v, pos + 1, cur, out);
    }
}

static void multi_indices(int d, int P, std::vector<int32_t> &out) {
    out.clear();
    std::vector<int32_t> cur(d, 0);
    for (int g = 0; g <= P; ++g) compositions(d, g, 0, cur, out);
}

// ------------------------------------------------------------------ Monte Carlo
// SplitMix64 (Steele, Lea & Flood 2014) in counter form: output number c of
// the generator seeded with `seed` is the finaliser applied to seed + c*gamma.
static inline uint64_t splitmix_at(uint64_t seed, uint64_t c) {
    uint64_t z = seed + c * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// ------------------------------------------------------------------ rule
uq_status build_rule(const uq_problem &p, Rule &r) {
    uq_status st = validate_problem(p);
    if (st != UQ_OK) return st;
    r = Rule();
    r.d = p.n_dists;
    const int d = r.d;
    if (p.rule == UQ_RULE_GL_TENSOR) {
        const int n = p.n_per_dim;
        std::vector<double> x1, w1;
        gauss_legendre_prob(n, x1, w1);
        int64_t S = 1;
        for (int k = 0; k < d; ++k) S *= n;
        r.S = S;
        r.xi.resize(S * d);
        r.a.resize(S);
        for (int64_t j = 0; j < S; ++j) {
            int64_t stride = S;
            double wj = 1.0;
            for (int k = 0; k < d; ++k) {
                stride /= n;
                int m = (int)((j / stride) % n);
                r.xi[j * d + k] = x1[m];
                wj *= w1[m];
            }
            r.a[j] = wj;
        }
        multi_indices(d, p.order, r.alpha);
        r.K = (int)(r.alpha.size() / d);
        r.phi.resize(S * r.K);
        std::vector<double> pv((size_t)d * (p.order + 1));
        for (int64_t j = 0; j < S; ++j) {
            for (int k = 0; k < d; ++k) ortho_legendre_all(p.order, r.xi[j * d + k], &pv[(size_t)k * (p.order + 1)]);
            for (int t = 0; t < r.K; ++t) {
                double v = 1.0;
                for (int k = 0; k < d; ++k) v *= pv[(size_t)k * (p.order + 1) + r.alpha[(size_t)t * d + k]];
                r.phi[j * r.K + t] = v;
            }
        }
    } else {
        const int64_t N = p.mc_n;
        r.S = N;
        r.K = 0;
        r.xi.resize(N * d);
        r.a.assign(N, 1.0 / (double)N);
        for (int64_t j = 0; j < N; ++j)
            for (int k = 0; k < d; ++k) {
                uint64_t bits = splitmix_at(p.seed, (uint64_t)(j * d + k + 1));
                double u = (double)(bits >> 11) * 0x1.0p-53;
                r.xi[j * d + k] = 2.0 * u - 1.0;
            }
    }
    return UQ_OK;
}

void map_inputs(const uq_problem &p, const double *xi, SampleInputs &o) {
    o.nu = p.nu;
    o.u0 = p.u0;
    o.phase_x = p.phase_x;
    o.phase_y = p.phase_y;
    o.u_peak = p.u_peak;
    bool has_re = false;
    double re = 0.0;
    for (int k = 0; k < p.n_dists; ++k) {
        const uq_dist &q = p.dists[k];
        double v = q.lo + (q.hi - q.lo) * 0.5 * (xi[k] + 1.0);
        switch (q.target) {
            case UQ_T_NU: o.nu = v; break;
            case UQ_T_U0: o.u0 = v; break;
            case UQ_T_PHASE_X: o.phase_x = v; break;
            case UQ_T_PHASE_Y: o.phase_y = v; break;
            case UQ_T_RE: has_re = true; re = v; break;
            case UQ_T_U_PEAK: o.u_peak = v; break;
        }
    }
    // Re from the peak inflow velocity and the diameter (cylinder section)
    if (has_re) o.nu = p.u_peak * (double)p.D / re;
}

}  // namespace uqi

extern "C" uq_status uq_rule_size(const uq_problem *p, int64_t *S, int32_t *K) {
    if (!p) return uqi::fail(UQ_EINVAL, "null problem");
    uqi::Rule r;
    uq_status st = uqi::build_rule(*p, r);
    if (st != UQ_OK) return st;
    if (S) *S = r.S;
    if (K) *K = r.K;
    return UQ_OK;
}

extern "C" uq_status uq_rule_points(const uq_problem *p, double *xi, double *a, int32_t *alpha, double *phi) {
    if (!p) return uqi::fail(UQ_EINVAL, "null problem");
    uqi::Rule r;
    uq_status st = uqi::build_rule(*p, r);
    if (st != UQ_OK) return st;
    if (xi) std::memcpy(xi, r.xi.data(), sizeof(double) * r.xi.size());
    if (a) std::memcpy(a, r.a.data(), sizeof(double) * r.a.size());
    if (alpha) std::memcpy(alpha, r.alpha.data(), sizeof(int32_t) * r.alpha.size());
    if (phi) std::memcpy(phi, r.phi.data(), sizeof(double) * r.phi.size());
    return UQ_OK;
}
