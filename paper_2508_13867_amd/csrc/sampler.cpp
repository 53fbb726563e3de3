// Host side of the UQ layer: validation, collocation / Monte Carlo sample
// sets, the orthonormal Legendre basis and the mapping of reference
// variables to solver inputs (Sec. "Uncertainty quantification methods" and
// "Core class design" of OpenLB-UQ, arXiv 2508.13867).
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

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
    if (p.init != UQ_INIT_TGV && p.init != UQ_INIT_TGV_HARMONIC) return fail(UQ_EINVAL, "unknown init");
    if (p.init == UQ_INIT_TGV_HARMONIC && p.geometry != UQ_GEOM_TGV)
        return fail(UQ_EINVAL, "the harmonic initial field is a vortex option");
    if (p.geometry == UQ_GEOM_CHANNEL) {
        if (p.xbc < UQ_XBC_ZOUHE || p.xbc > UQ_XBC_INTERP) return fail(UQ_EINVAL, "unknown xbc");
        if (p.D < 0) return fail(UQ_EINVAL, "D must be >= 0");
        if (p.ramp < 0) return fail(UQ_EINVAL, "ramp must be >= 0");
        if (p.cyl_bc != UQ_CYL_HALFWAY && p.cyl_bc != UQ_CYL_BOUZIDI) return fail(UQ_EINVAL, "unknown cyl_bc");
        if (p.force_ref != UQ_FORCE_REF_PEAK && p.force_ref != UQ_FORCE_REF_MEAN)
            return fail(UQ_EINVAL, "unknown force_ref");
        const bool interp = p.xbc == UQ_XBC_INTERP || p.cyl_bc == UQ_CYL_BOUZIDI;
        if (interp && p.layout == UQ_LAYOUT_AA)
            return fail(UQ_EINVAL, "interpolated boundaries read neighbours' previous state: they need the AB layout");
        if (p.xbc == UQ_XBC_INTERP && p.nx < 4) return fail(UQ_EINVAL, "the interpolated inlet/outlet needs nx >= 4");
        // extent of the cylinder's solid nodes
        double x0 = 0, x1 = -1, y0 = 0, y1 = -1;
        if (p.cyl_bc == UQ_CYL_BOUZIDI) {
            if (!(p.cyl_d > 0) || !std::isfinite(p.cyl_x) || !std::isfinite(p.cyl_y))
                return fail(UQ_EINVAL, "the interpolated cylinder needs a finite centre and cyl_d > 0");
            const double r = 0.5 * p.cyl_d;
            x0 = p.cyl_x - r, x1 = p.cyl_x + r, y0 = p.cyl_y - r, y1 = p.cyl_y + r;
            if (y0 < 2.0 || y1 > p.ny - 3.0 || x0 < 3.0 || x1 > p.nx - 4.0)
                return fail(UQ_EINVAL, "the interpolated cylinder must stay 2 nodes inside the walls and 3 nodes "
                                       "from the x ends");
        } else if (p.D > 0) {
            const double r = 0.5 * p.D;
            x0 = p.cx - r, x1 = p.cx + r, y0 = p.cy - r, y1 = p.cy + r;
        }
        if (p.xbc == UQ_XBC_INTERP && x1 >= x0 && (x0 < 3.0 || x1 > p.nx - 4.0))
            return fail(UQ_EINVAL, "the interpolated inlet/outlet needs the cylinder 3 nodes away from both columns");
    }
    for (int k = 0; k < p.n_dists; ++k) {
        const uq_dist &q = p.dists[k];
        if (q.target < UQ_T_NU || q.target > UQ_T_ZETA11) return fail(UQ_EINVAL, "unknown target");
        if (q.target >= UQ_T_ZETA00 && !(p.geometry == UQ_GEOM_TGV && p.init == UQ_INIT_TGV_HARMONIC))
            return fail(UQ_EINVAL, "perturbation amplitudes apply to the harmonic vortex only");
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
    } else if (p.rule == UQ_RULE_MC || p.rule == UQ_RULE_HALTON || p.rule == UQ_RULE_LHS) {
        if (p.n_dists < 1) return fail(UQ_EINVAL, "sampling needs at least one uncertain input");
        if (p.mc_n < 2 || p.mc_n > 10000000) return fail(UQ_EINVAL, "mc_n must be in [2, 1e7]");
    } else if (p.rule == UQ_RULE_SMOLYAK_CC) {
        if (p.n_dists < 1) return fail(UQ_EINVAL, "collocation needs at least one uncertain input");
        if (p.level < 0 || p.level > 8) return fail(UQ_EINVAL, "level must be in [0, 8]");
        if (p.order < 0 || p.order > 32) return fail(UQ_EINVAL, "order must be in [0, 32]");
        if (p.n_dists * (p.level + 1) > 64) return fail(UQ_EINVAL, "sparse grid too large");
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

// ------------------------------------------------------------------ Clenshaw-Curtis / Smolyak
// 1-D nested Clenshaw-Curtis rule of level i >= 1: m(1) = 1 (the midpoint),
// m(i) = 2^(i-1) + 1 nodes x_j = -cos(pi j/(m-1)); weights of the probability
// measure dx/2 from the closed form (Clenshaw & Curtis 1960)
//   w_j = c_j/n (1 - sum_{k=1}^{n/2} b_k cos(2 k j pi/n)/(4k^2 - 1)),
// n = m - 1, c_0 = c_n = 1/2 (else 1), b_{n/2} = 1 (else 2); summing to one.
static int cc_points(int i) { return i <= 1 ? 1 : (1 << (i - 1)) + 1; }

static void cc_weights(int i, std::vector<double> &w) {
    const int m = cc_points(i);
    w.assign(m, 0.0);
    if (m == 1) {
        w[0] = 1.0;
        return;
    }
    const int n = m - 1;
    for (int j = 0; j <= n; ++j) {
        double s = 0.0;
        for (int k = 1; k <= n / 2; ++k) {
            const double b = (2 * k == n) ? 1.0 : 2.0;
            s += b * std::cos(2.0 * k * j * M_PI / n) / (4.0 * k * k - 1.0);
        }
        const double c = (j == 0 || j == n) ? 0.5 : 1.0;
        w[j] = c / n * (1.0 - s);
    }
}

// Smolyak sparse grid by the combination technique:
//   A(l, d) = sum over levels i (i_k >= 1) with l + 1 <= |i| <= l + d of
//             (-1)^(l + d - |i|) C(d - 1, l + d - |i|) (U^{i_1} x ... x U^{i_d}).
// Nodes are identified by their index on the finest 1-D grid (level l + 1),
// so coinciding nodes of different tensor grids merge exactly.
static void smolyak(int d, int l, std::vector<double> &xi, std::vector<double> &a, int64_t &S) {
    const int imax = l + 1;
    const int mf = cc_points(imax);  // finest 1-D grid
    std::map<std::vector<int>, double> acc;
    std::vector<int> lev(d, 1);
    std::vector<std::vector<double>> W(imax + 1);
    for (int i = 1; i <= imax; ++i) cc_weights(i, W[i]);
    auto binom = [](int n, int k) {
        double r = 1.0;
        for (int t = 1; t <= k; ++t) r = r * (n - k + t) / t;
        return r;
    };
    for (;;) {
        int sum = 0;
        for (int k = 0; k < d; ++k) sum += lev[k];
        if (sum >= l + 1 && sum <= l + d) {
            const int e = l + d - sum;
            const double coef = ((e & 1) ? -1.0 : 1.0) * binom(d - 1, e);
            // tensor grid of this level multi-index
            std::vector<int> j(d, 0), key(d);
            for (;;) {
                double wt = coef;
                for (int k = 0; k < d; ++k) {
                    const int m = cc_points(lev[k]);
                    key[k] = m == 1 ? (mf - 1) / 2 : j[k] * ((mf - 1) / (m - 1));
                    wt *= W[lev[k]][j[k]];
                }
                acc[key] += wt;
                int k = d - 1;
                while (k >= 0 && ++j[k] == cc_points(lev[k])) j[k--] = 0;
                if (k < 0) break;
            }
        }
        int k = d - 1;
        while (k >= 0 && ++lev[k] > imax) lev[k--] = 1;
        if (k < 0) break;
    }
    S = (int64_t)acc.size();
    xi.assign((size_t)S * d, 0.0);
    a.assign((size_t)S, 0.0);
    int64_t s = 0;
    for (auto &kv : acc) {  // std::map order: lexicographic, input 0 first
        for (int k = 0; k < d; ++k)
            xi[(size_t)s * d + k] = mf == 1 ? 0.0 : -std::cos(M_PI * kv.first[k] / (mf - 1));
        a[(size_t)s] = kv.second;
        ++s;
    }
    // the middle node is exactly zero
    for (auto &v : xi)
        if (std::fabs(v) < 1e-15) v = 0.0;
}

// ------------------------------------------------------------------ Halton / LHS
static double radical_inverse(uint64_t n, uint64_t base) {
    double inv = 1.0 / (double)base, f = inv, r = 0.0;
    while (n > 0) {
        r += f * (double)(n % base);
        n /= base;
        f *= inv;
    }
    return r;
}

static const int kPrimes[UQ_MAX_DIMS] = {2, 3, 5, 7, 11, 13, 17, 19};

// uniform integer in [0, n) from one generator output (Lemire's multiply-shift)
static inline uint64_t bounded(uint64_t r, uint64_t n) { return (uint64_t)(((unsigned __int128)r * n) >> 64); }

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
    } else if (p.rule == UQ_RULE_SMOLYAK_CC) {
        smolyak(d, p.level, r.xi, r.a, r.S);
        multi_indices(d, p.order, r.alpha);
        r.K = (int)(r.alpha.size() / d);
        r.phi.resize(r.S * r.K);
        std::vector<double> pv((size_t)d * (p.order + 1));
        for (int64_t j = 0; j < r.S; ++j) {
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
        if (p.rule == UQ_RULE_HALTON) {
            for (int64_t j = 0; j < N; ++j)
                for (int k = 0; k < d; ++k) r.xi[j * d + k] = 2.0 * radical_inverse((uint64_t)j + 1, kPrimes[k]) - 1.0;
        } else if (p.rule == UQ_RULE_LHS) {
            // input k: Fisher-Yates shuffle of the strata 0..N-1 driven by draws
            // c = k*2N + i + 1 (i = N-1 .. 1), then the position inside stratum
            // s of sample j from draw c = k*2N + N + j + 1
            std::vector<int64_t> perm((size_t)N);
            for (int k = 0; k < d; ++k) {
                for (int64_t i = 0; i < N; ++i) perm[(size_t)i] = i;
                const uint64_t base = (uint64_t)k * 2 * (uint64_t)N;
                for (int64_t i = N - 1; i >= 1; --i) {
                    const uint64_t t = bounded(splitmix_at(p.seed, base + (uint64_t)i + 1), (uint64_t)i + 1);
                    std::swap(perm[(size_t)i], perm[(size_t)t]);
                }
                for (int64_t j = 0; j < N; ++j) {
                    const double u = (double)(splitmix_at(p.seed, base + (uint64_t)N + (uint64_t)j + 1) >> 11) * 0x1.0p-53;
                    r.xi[j * d + k] = 2.0 * (((double)perm[(size_t)j] + u) / (double)N) - 1.0;
                }
            }
        } else {
            for (int64_t j = 0; j < N; ++j)
                for (int k = 0; k < d; ++k) {
                    uint64_t bits = splitmix_at(p.seed, (uint64_t)(j * d + k + 1));
                    double u = (double)(bits >> 11) * 0x1.0p-53;
                    r.xi[j * d + k] = 2.0 * u - 1.0;
                }
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
    for (int k = 0; k < 4; ++k) o.zeta[k] = 0.0;
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
            case UQ_T_ZETA00: o.zeta[0] = v; break;
            case UQ_T_ZETA01: o.zeta[1] = v; break;
            case UQ_T_ZETA10: o.zeta[2] = v; break;
            case UQ_T_ZETA11: o.zeta[3] = v; break;
        }
    }
    // Re from the nominal inflow velocity (peak, or the mean 2/3 of it) and
    // the diameter (cylinder section)
    if (has_re) {
        const double U = p.force_ref == UQ_FORCE_REF_MEAN ? p.u_peak * (2.0 / 3.0) : p.u_peak;
        const double dia = p.cyl_bc == UQ_CYL_BOUZIDI ? p.cyl_d : (double)p.D;
        o.nu = U * dia / re;
    }
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

extern "C" uq_status uq_tgv_units(int32_t n, double Ma, double Re, double *nu_lat, double *u_lat, double *dx,
                                  double *dt, double *tau) {
    if (n < 2 || !(Ma > 0) || !(Re > 0)) return uqi::fail(UQ_EINVAL, "need n >= 2, Ma > 0, Re > 0");
    // physical box of side 2 pi resolved by n nodes (Table tab:simulation_parameters)
    const double h = 2.0 * M_PI / (double)(n - 1);
    const double ul = Ma / std::sqrt(3.0);
    const double k = h * ul;                 // time step: dx times the lattice velocity
    const double nl = (1.0 / Re) * k / (h * h);
    if (nu_lat) *nu_lat = nl;
    if (u_lat) *u_lat = ul;
    if (dx) *dx = h;
    if (dt) *dt = k;
    if (tau) *tau = 3.0 * nl + 0.5;
    return UQ_OK;
}
