/*
 * FP64 reference implementation of the non-intrusive LBM-UQ method
 * (OpenLB-UQ, arXiv 2508.13867). TEST INFRASTRUCTURE ONLY: it is called by
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark,
 * never by the product path. It shares no code, header or table with the GPU
 * library; every constant below is derived here from the paper's definitions.
 *
 * Plain, slow, single-threaded double precision. Per sample it runs a
 * two-array D2Q9 BGK scheme in the paper's order: collide (Sec. "Lattice
 * Boltzmann methods", collision/streaming split), then stream, then complete
 * the populations that streaming leaves undefined (boundaries).
 *
 * Readings of passages where the paper is silent or garbled are listed at the
 * top of each function; all of them are collected in the design notes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* D2Q9 velocity set and weights (Sec. "Lattice Boltzmann methods", velocity
 * set and Eq. weightsDdQ9). Reading: the scalar prefactor "w" in the weight
 * equation is 1 (the weights must sum to one). Ordering within the groups is
 * not fixed by the paper; we use rest, the four axis directions
 * counter-clockwise from +x, then the four diagonals counter-clockwise from
 * (+1,+1).                                                                   */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

static double W(int i) {
    if (i == 0) return 4.0 / 9.0;
    if (i <= 4) return 1.0 / 9.0;
    return 1.0 / 36.0;
}

/* opposite direction: the j with c_j = -c_i, found by search (no table). */
static int OPP(int i) {
    for (int j = 0; j < 9; ++j)
        if (CX[j] == -CX[i] && CY[j] == -CY[i]) return j;
    return -1;
}

/* c_s^2 = 1/3 in lattice units. Pinned by reproducing the paper's Table
 * tab:simulation_parameters with tau = nu/c_s^2 + 1/2.                      */
static const double CS2 = 1.0 / 3.0;

void oracle_d2q9(int *cx, int *cy, double *w, int *opp) {
    for (int i = 0; i < 9; ++i) {
        cx[i] = CX[i];
        cy[i] = CY[i];
        w[i] = W(i);
        opp[i] = OPP(i);
    }
}

/* Second-order equilibrium, Eq. "equilibrium":
 * f_i^eq = w_i rho (1 + u.c_i/cs2 + (u.c_i)^2/(2 cs2^2) - u.u/(2 cs2)).     */
static double feq(int i, double rho, double ux, double uy) {
    double cu = ux * CX[i] + uy * CY[i];
    double uu = ux * ux + uy * uy;
    return W(i) * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
}

void oracle_feq(double rho, double ux, double uy, double *out) {
    for (int i = 0; i < 9; ++i) out[i] = feq(i, rho, ux, uy);
}

/* Moments rho = sum f_i, rho u = sum c_i f_i (Sec. "Lattice Boltzmann
 * methods", moment equations).                                              */
static void moments(const double *f, double *rho, double *ux, double *uy) {
    double r = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < 9; ++i) {
        r += f[i];
        jx += CX[i] * f[i];
        jy += CY[i] * f[i];
    }
    *rho = r;
    *ux = jx / r;
    *uy = jy / r;
}

/* BGK collision, Eq. bgkCollision with the collision half of the
 * collide/stream split: f* = f - (f - f^eq)/tau.                            */
static void collide(const double *f, double tau, double *fs) {
    double rho, ux, uy;
    moments(f, &rho, &ux, &uy);
    for (int i = 0; i < 9; ++i) fs[i] = f[i] - (f[i] - feq(i, rho, ux, uy)) / tau;
}

void oracle_collide(const double *f, double tau, double *out) { collide(f, tau, out); }

/* Unit conversion of the paper's four-dimensional TGV case (Table
 * tab:simulation_parameters): dx = 2 pi/(n-1), lattice speed Ma/sqrt(3),
 * dt = dx * u_lat, nu_phys = 1/Re, nu_lat = nu_phys dt/dx^2,
 * tau = nu_lat/cs2 + 1/2.                                                   */
void oracle_table1_units(int n, double Ma, double Re, double *tau, double *dx, double *dt) {
    const double pi = acos(-1.0);
    double h = 2.0 * pi / (double)(n - 1);
    double ulat = Ma / sqrt(3.0);
    double k = h * ulat;
    double nu_lat = (1.0 / Re) * k / (h * h);
    *dx = h;
    *dt = k;
    *tau = nu_lat / CS2 + 0.5;
}

/* ------------------------------------------------------------------------ */
/* Quadrature and polynomial basis (Sec. "Generalized polynomial chaos").    */

/* Legendre polynomial P_n(x) by the three-term recurrence
 * (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}; also returns P_n'(x).           */
static double legendre(int n, double x, double *dp) {
    double p0 = 1.0, p1 = x;
    if (n == 0) {
        if (dp) *dp = 0.0;
        return 1.0;
    }
    for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
    }
    if (dp) *dp = n * (x * p1 - p0) / (x * x - 1.0);
    return p1;
}

/* Orthonormal Legendre basis for the uniform density on [-1,1]:
 * E[phi_m phi_n] = delta_mn with phi_n = sqrt(2n+1) P_n (so gamma_k = 1 in
 * Eq. coef_integral).                                                       */
double oracle_legendre_orthonormal(int n, double x) {
    return sqrt(2.0 * n + 1.0) * legendre(n, x, NULL);
}

/* n-point Gauss-Legendre rule on [-1,1] (textbook weights, sum 2): nodes are
 * the roots of P_n found by Newton's method from the Chebyshev-like guess
 * cos(pi (i + 3/4)/(n + 1/2)); weights 2/((1-x^2) P_n'(x)^2). Nodes are
 * returned in increasing order.                                             */
int oracle_gauss_legendre(int n, double *x, double *w) {
    if (n < 1) return -1;
    const double pi = acos(-1.0);
    for (int i = 0; i < n; ++i) {
        double z = cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p = legendre(n, z, &dp);
            double dz = p / dp;
            z -= dz;
            if (fabs(dz) < 1e-17) break;
        }
        legendre(n, z, &dp);
        /* the guess for index i approaches the i-th largest root */
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    if (n % 2 == 1) x[n / 2] = 0.0; /* the middle root is exactly zero */
    return 0;
}

/* Tensor-product collocation rule over d independent uniform inputs
 * (Sec. "Quadrature and collocation", tensor products; step 1 of the SC-gPC
 * procedure). Reading: weights are those of the probability measure h, i.e.
 * each one-dimensional rule is divided by 2 so the weights sum to one and the
 * zeroth coefficient is the mean (Eq. gpc_mean). Samples are enumerated with
 * dimension 0 varying slowest.                                              */
int oracle_gl_tensor(int d, int n, double *xi, double *a) {
    if (d < 1 || n < 1) return -1;
    double *x1 = malloc(sizeof(double) * n), *w1 = malloc(sizeof(double) * n);
    oracle_gauss_legendre(n, x1, w1);
    long S = 1;
    for (int k = 0; k < d; ++k) S *= n;
    for (long j = 0; j < S; ++j) {
        long rem = j;
        double wj = 1.0;
        for (int k = d - 1; k >= 0; --k) {
            int m = (int)(rem % n);
            rem /= n;
            xi[j * d + k] = x1[m];
            wj *= 0.5 * w1[m];
        }
        a[j] = wj;
    }
    free(x1);
    free(w1);
    return 0;
}

/* Total-degree multi-indices |alpha| <= P in d dimensions (reading of the
 * truncated expansion Eq. gPC for d > 1, which the paper leaves open), in
 * graded order: by total degree, and within one degree with alpha_0 largest
 * first, then alpha_1, and so on. Returns K = C(d+P, P); fills alpha[K*d] if
 * not NULL. Enumeration is a plain odometer over [0,P]^d filtered by degree,
 * repeated per degree.                                                      */
int oracle_multi_indices(int d, int P, int *alpha) {
    int K = 0;
    int *cur = calloc((size_t)d, sizeof(int));
    for (int deg = 0; deg <= P; ++deg) {
        /* odometer that counts down from (P,...,P) to (0,...,0) in the
         * lexicographic order with the first coordinate most significant   */
        long total = 1;
        for (int k = 0; k < d; ++k) total *= (P + 1);
        for (long code = total - 1; code >= 0; --code) {
            long rem = code;
            int s = 0;
            for (int k = d - 1; k >= 0; --k) {
                cur[k] = (int)(rem % (P + 1));
                rem /= (P + 1);
                s += cur[k];
            }
            if (s != deg) continue;
            if (alpha)
                for (int k = 0; k < d; ++k) alpha[K * d + k] = cur[k];
            ++K;
        }
    }
    free(cur);
    return K;
}

/* Phi table Phi[j*K + k] = prod_m phi_{alpha_k,m}(xi_{j,m}).                */
void oracle_phi_table(long S, int d, const double *xi, int K, const int *alpha, double *phi) {
    for (long j = 0; j < S; ++j)
        for (int k = 0; k < K; ++k) {
            double v = 1.0;
            for (int m = 0; m < d; ++m) v *= oracle_legendre_orthonormal(alpha[k * d + m], xi[j * d + m]);
            phi[j * K + k] = v;
        }
}

/* Monte Carlo draws (Sec. "Monte Carlo and quasi Monte Carlo sampling";
 * the paper seeds its example with 123456 but names no generator). Reading:
 * SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) run sequentially from `seed`;
 * output number c (c = 1, 2, ...) is used for sample j, dimension k with
 * c = j*d + k + 1. The top 53 bits give u in [0,1), and xi = 2u - 1.
 * This implementation steps the generator state one increment at a time.   */
static uint64_t splitmix_next(uint64_t *state) {
    *state += 0x9E3779B97F4A7C15ULL;
    uint64_t z = *state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

void oracle_splitmix64_stream(uint64_t seed, long n, uint64_t *out) {
    uint64_t s = seed;
    for (long c = 0; c < n; ++c) out[c] = splitmix_next(&s);
}

void oracle_mc_points(uint64_t seed, long N, int d, double *xi, double *a) {
    uint64_t s = seed;
    for (long j = 0; j < N; ++j) {
        for (int k = 0; k < d; ++k) {
            uint64_t r = splitmix_next(&s);
            double u = (double)(r >> 11) * (1.0 / 9007199254740992.0);
            xi[j * d + k] = 2.0 * u - 1.0;
        }
        a[j] = 1.0 / (double)N;
    }
}

/* ------------------------------------------------------------------------ */
/* Compensated summation (Neumaier's improvement of Kahan's algorithm).      */
typedef struct {
    double s, c;
} nsum;

static void nadd(nsum *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}
static double nval(const nsum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------------ */
/* Statistics over samples (Sec. "Monte Carlo and quasi Monte Carlo
 * sampling", Eqs. meanMCS and varMCS; Sec. "Generalized polynomial chaos",
 * Eqs. coef_discrete, gpc_mean, gpc_std). M is [S][n_out] row-major.        */

/* MC: mean (Eq. meanMCS), unbiased variance 1/(N-1) (Eq. varMCS) and the
 * 1/N variant used in the non-intrusive UQ algorithm's Monte Carlo branch.  */
void oracle_mc_stats(long S, long n_out, const double *M, double *mean, double *var, double *var_n) {
    for (long o = 0; o < n_out; ++o) {
        nsum s = {0, 0};
        for (long j = 0; j < S; ++j) nadd(&s, M[j * n_out + o]);
        double m = nval(&s) / (double)S;
        nsum q = {0, 0};
        for (long j = 0; j < S; ++j) {
            double e = M[j * n_out + o] - m;
            nadd(&q, e * e);
        }
        mean[o] = m;
        var[o] = S > 1 ? nval(&q) / (double)(S - 1) : 0.0;
        var_n[o] = nval(&q) / (double)S;
    }
}

/* SC-gPC: coefficients by discrete projection (Eq. coef_discrete, gamma_k=1
 * for the orthonormal basis), mean = coefficient 0 (Eq. gpc_mean), variance
 * = sum of squares of the other retained coefficients (Eq. gpc_std), and the
 * quadrature variance sum_j a_j (M_j - mean)^2 as a diagnostic.
 * coeffs is [K][n_out].                                                      */
void oracle_gpc_stats(long S, long n_out, const double *M, const double *a, int K, const double *phi,
                      double *coeffs, double *mean, double *var, double *var_quad) {
    for (long o = 0; o < n_out; ++o) {
        for (int k = 0; k < K; ++k) {
            nsum s = {0, 0};
            for (long j = 0; j < S; ++j) nadd(&s, a[j] * M[j * n_out + o] * phi[j * K + k]);
            coeffs[(long)k * n_out + o] = nval(&s);
        }
        mean[o] = coeffs[o];
        nsum v = {0, 0};
        for (int k = 1; k < K; ++k) {
            double c = coeffs[(long)k * n_out + o];
            nadd(&v, c * c);
        }
        var[o] = nval(&v);
        nsum q = {0, 0};
        for (long j = 0; j < S; ++j) {
            double e = M[j * n_out + o] - mean[o];
            nadd(&q, a[j] * e * e);
        }
        var_quad[o] = nval(&q);
    }
}

/* ------------------------------------------------------------------------ */
/* Taylor-Green vortex, one deterministic sample (Sec. "Taylor--Green vortex
 * flow with uncertain viscosity", Eqs. TGV_vel, TGV_press, KineticEnergy).
 * Readings: nodes x, y = 0..n-1 and k = 2 pi/n; the initial density is
 * rho = 1 + p/cs2 (the equation of state with the reference pressure P0
 * taken as the one at rho = 1); two optional phase shifts enter as
 * (k x + phi_x), (k y + phi_y), a translate of the same exact solution;
 * tau = nu/cs2 + 1/2 (lattice units, dt = 1).
 *
 * State f(x, t) is the post-streaming, pre-collision population; the QoIs at
 * step n are moments of f(., n). f is stored [9][ny][nx].                  */

static long idx(int i, int y, int x, int nx, int ny) { return ((long)i * ny + y) * nx + x; }

static void tgv_init(int nx, int ny, double u0, double phx, double phy, double *f) {
    const double pi = acos(-1.0);
    double kx = 2.0 * pi / nx, ky = 2.0 * pi / ny;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double ax = kx * x + phx, ay = ky * y + phy;
            double ux = -u0 * cos(ax) * sin(ay);
            double uy = u0 * sin(ax) * cos(ay);
            double p = -0.25 * u0 * u0 * (cos(2.0 * ax) + (kx / ky) * (kx / ky) * cos(2.0 * ay));
            double rho = 1.0 + p / CS2;
            for (int i = 0; i < 9; ++i) f[idx(i, y, x, nx, ny)] = feq(i, rho, ux, uy);
        }
}

/* The four-dimensional perturbed vortex (Sec. "Taylor--Green vortex flow with
 * four-dimensional uncertain initial velocity perturbation", Eq. taylorGreen
 * and the perturbation eps_d): on the physical box [0, 2 pi) resolved by n
 * nodes, u = u0R (-cos 2X sin 2Y, sin 2X cos 2Y), p = -u0R^2/4 (cos 4X +
 * cos 4Y) (the printed (2/2)^2 read as 1), u0R = u0 (1 + eps),
 * eps = 1/4 sum_{i,j} zeta_ij k_i(4X) k_j(4Y), k_0 = sin, k_1 = cos, with
 * X = 2 pi x/n. Reading: the paper's physical amplitude is 1, so its
 * additive perturbation is a relative one for a lattice amplitude u0.        */
static void tgv_harmonic_init(int nx, int ny, double u0, const double *zeta, double *f) {
    const double pi = acos(-1.0);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double X = 2.0 * pi * x / nx, Y = 2.0 * pi * y / ny;
            double kx[2] = {sin(4.0 * X), cos(4.0 * X)}, ky[2] = {sin(4.0 * Y), cos(4.0 * Y)};
            double eps = 0.0;
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) eps += zeta[2 * i + j] * kx[i] * ky[j];
            eps *= 0.25;
            double uR = u0 * (1.0 + eps);
            double ux = -uR * cos(2.0 * X) * sin(2.0 * Y);
            double uy = uR * sin(2.0 * X) * cos(2.0 * Y);
            double p = -0.25 * uR * uR * (cos(4.0 * X) + cos(4.0 * Y));
            double rho = 1.0 + p / CS2;
            for (int i = 0; i < 9; ++i) f[idx(i, y, x, nx, ny)] = feq(i, rho, ux, uy);
        }
}

static void periodic_step(int nx, int ny, double tau, double *f, double *tmp) {
    double fc[9], fs[9];
    /* collision at every node, written to tmp */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            for (int i = 0; i < 9; ++i) fc[i] = f[idx(i, y, x, nx, ny)];
            collide(fc, tau, fs);
            for (int i = 0; i < 9; ++i) tmp[idx(i, y, x, nx, ny)] = fs[i];
        }
    /* streaming f_i(x + c_i, t+1) = f*_i(x, t), periodic in both axes */
    for (int i = 0; i < 9; ++i)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int xd = (x + CX[i] + nx) % nx, yd = (y + CY[i] + ny) % ny;
                f[idx(i, yd, xd, nx, ny)] = tmp[idx(i, y, x, nx, ny)];
            }
}

/* Run one TGV sample for `steps` steps. Outputs (each may be NULL):
 * f_out [9][ny][nx]; rho/ux/uy [ny][nx]; ke (normalised by ke_u0, the
 * nominal amplitude: reading of Eq. KineticEnergy when u0 is uncertain).   */
int oracle_tgv_run(int nx, int ny, double nu, double u0, double phx, double phy, long steps, double ke_u0,
                   double *f_out, double *rho_out, double *ux_out, double *uy_out, double *ke_out) {
    double tau = nu / CS2 + 0.5;
    if (!(tau > 0.5) || nx < 1 || ny < 1) return -1;
    long n = (long)nx * ny;
    double *f = malloc(sizeof(double) * 9 * n), *tmp = malloc(sizeof(double) * 9 * n);
    tgv_init(nx, ny, u0, phx, phy, f);
    for (long t = 0; t < steps; ++t) periodic_step(nx, ny, tau, f, tmp);
    nsum ke = {0, 0};
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double fc[9], rho, ux, uy;
            for (int i = 0; i < 9; ++i) fc[i] = f[idx(i, y, x, nx, ny)];
            moments(fc, &rho, &ux, &uy);
            long c = (long)y * nx + x;
            if (rho_out) rho_out[c] = rho;
            if (ux_out) ux_out[c] = ux;
            if (uy_out) uy_out[c] = uy;
            nadd(&ke, ux * ux + uy * uy);
        }
    if (ke_out) *ke_out = 2.0 / ((double)nx * ny * ke_u0 * ke_u0) * nval(&ke);
    if (f_out) memcpy(f_out, f, sizeof(double) * 9 * n);
    free(f);
    free(tmp);
    return 0;
}

/* Run one sample of the perturbed vortex; outputs as oracle_tgv_run plus the
 * speed field |u| [ny][nx].                                                  */
int oracle_tgv_harmonic_run(int nx, int ny, double nu, double u0, const double *zeta, long steps, double ke_u0,
                            double *f_out, double *rho_out, double *ux_out, double *uy_out, double *speed_out,
                            double *ke_out) {
    double tau = nu / CS2 + 0.5;
    if (!(tau > 0.5) || nx < 1 || ny < 1) return -1;
    long n = (long)nx * ny;
    double *f = malloc(sizeof(double) * 9 * n), *tmp = malloc(sizeof(double) * 9 * n);
    tgv_harmonic_init(nx, ny, u0, zeta, f);
    for (long t = 0; t < steps; ++t) periodic_step(nx, ny, tau, f, tmp);
    nsum ke = {0, 0};
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double fc[9], rho, ux, uy;
            for (int i = 0; i < 9; ++i) fc[i] = f[idx(i, y, x, nx, ny)];
            moments(fc, &rho, &ux, &uy);
            long c = (long)y * nx + x;
            if (rho_out) rho_out[c] = rho;
            if (ux_out) ux_out[c] = ux;
            if (uy_out) uy_out[c] = uy;
            if (speed_out) speed_out[c] = sqrt(ux * ux + uy * uy);
            nadd(&ke, ux * ux + uy * uy);
        }
    if (ke_out) *ke_out = 2.0 / ((double)nx * ny * ke_u0 * ke_u0) * nval(&ke);
    if (f_out) memcpy(f_out, f, sizeof(double) * 9 * n);
    free(f);
    free(tmp);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Channel flow past a cylinder, one deterministic sample (Sec. "Flow past a
 * circular cylinder with uncertain inlet velocity").
 *   - channel of nx x ny nodes; no-slip walls below row 0 and above row
 *     ny-1. By default half-way (walls at y = -1/2 and y = ny - 1/2, so
 *     H = ny) with half-way bounce-back; optionally at y = -q_lo and
 *     y = ny - 1 + q_hi with the interpolated bounce-back below (used by
 *     tests of that scheme on a straight wall);
 *   - cylinder, two variants: (0) solid nodes 4((x-cx)^2 + (y-cy)^2) <= D^2
 *     (integer test) with half-way bounce-back on every link into it; (1)
 *     the exact circle of centre (ccx, ccy) and radius R (solid iff
 *     (x-ccx)^2 + (y-ccy)^2 <= R^2) with the linear interpolated
 *     bounce-back of Bouzidi, Firdaouss and Lallemand (Phys. Fluids 13,
 *     3452, 2001), the second-order curved-wall scheme the paper uses;
 *   - x boundary mode xbc: 0 = velocity inlet at x = 0 and pressure outlet
 *     (rho = 1) at x = nx-1 by Zou & He (Phys. Fluids 9, 1591, 1997) on every
 *     row of the open columns (at the corner nodes the populations arriving
 *     from beyond the wall come from the wall rule first, and Zou-He
 *     completes the rest); 1 = solid walls half-way at x = -1/2 and
 *     x = nx - 1/2; 2 = periodic; 3 = the same inlet and outlet by the
 *     finite-difference velocity-gradient reconstruction of Latt et al.
 *     (Phys. Rev. E 77, 056703, 2008), the paper's interpolated boundaries:
 *     every population of an open-column node is rebuilt as equilibrium plus
 *     the first-order non-equilibrium part -w_i rho tau/cs2 Q_i : grad u,
 *     Q_i = c_i c_i - cs2 I, with grad u from second-order finite
 *     differences (one-sided into the fluid across the column, central along
 *     it, one-sided at its ends); the inlet takes the prescribed velocity
 *     and rho from the known populations, the outlet rho = 1, u_y = 0 and
 *     u_x from the known populations;
 *   - parabolic inlet u_x(y) = s(t) 4 u_peak (y - y_lo)(y_hi - y)/H^2,
 *     u_y = 0, between the wall positions y_lo, y_hi (H = y_hi - y_lo), with
 *     the start-up ramp s(t) = sin^2(pi t/(2 T_r)) for t < T_r, else 1 (the
 *     paper ramps the inflow without giving the form);
 *   - initial state: equilibrium at rho = 1, u = 0 (Sec. cylinder,
 *     equilibrium initialisation; s(0) = 0); tests may start from a uniform
 *     u = (ux_init, 0) instead;
 *   - forces by momentum exchange on the cylinder links (Ladd 1994; for
 *     interpolated links Mei et al., J. Comput. Phys. 175, 2002):
 *     F = sum_{fluid x, k: x + c_k in cylinder} c_k (f*_k(x, t) +
 *     f_opp(k)(x, t+1)), with f* the collision of the final state and
 *     f_opp(k)(x, t+1) what the wall rule returns from it (half-way:
 *     f*_k(x, t), so F = sum 2 c_k f*_k), a lattice evaluation of the surface
 *     integrals Eqs. dragForce/liftForce;
 *   - C_D = 2 F_x/(rho0 U^2 D), C_L = 2 F_y/(rho0 U^2 D), rho0 = 1, U the
 *     sample's peak inlet velocity (force_ref 0) or its mean 2/3 u_peak
 *     (force_ref 1), D the diameter (2R for the circle).                     */

typedef struct {
    int nx, ny, xbc;
    int cyl;            /* 0: integer mask; 1: exact circle, interpolated */
    int D, cx, cy;      /* integer cylinder (D = 0: none)                 */
    double ccx, ccy, R; /* exact circle                                   */
    double q_lo, q_hi;  /* < 0: half-way walls                            */
    double q_fix;       /* >= 0: every link fraction replaced (tests)     */
    double nu, u_peak;
    long ramp, steps;
    double ux_init;
    int force_ref;
} oracle_channel_opts;

typedef struct {
    oracle_channel_opts o;
    int nx, ny;
    double tau, y_lo, y_hi;
    unsigned char *solid; /* [ny][nx] */
    double *q;            /* [9][ny][nx] link fraction of pull direction i, 0 = none */
} channel;

static int in_cylinder(const channel *c, double x, double y) {
    if (c->o.cyl == 1) {
        double dx = x - c->o.ccx, dy = y - c->o.ccy;
        return dx * dx + dy * dy <= c->o.R * c->o.R;
    }
    if (c->o.D <= 0) return 0;
    long dx = (long)x - c->o.cx, dy = (long)y - c->o.cy;
    return 4 * (dx * dx + dy * dy) <= (long)c->o.D * c->o.D;
}

/* point inside the solid of the interpolated geometry (circle or walls)  */
static int in_solid_exact(const channel *c, double x, double y) {
    if (c->o.q_lo >= 0.0 && (y < c->y_lo || y > c->y_hi)) return 1;
    return c->o.cyl == 1 && in_cylinder(c, x, y);
}

/* fraction q in (0, 1] of the link from fluid node (x, y) towards
 * (x - CX[i], y - CY[i]) at which it enters the solid, by bisection on the
 * segment (one crossing: the solid pieces are convex).                      */
static double link_fraction(const channel *c, int x, int y, int i) {
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (in_solid_exact(c, x - mid * CX[i], y - mid * CY[i]))
            hi = mid;
        else
            lo = mid;
    }
    return 0.5 * (lo + hi);
}

static double ramp_factor(long t, long T) {
    if (T <= 0 || t >= T) return 1.0;
    const double pi = acos(-1.0);
    double s = sin(pi * (double)t / (2.0 * (double)T));
    return s * s;
}

static double inlet_ux(const channel *c, int y, long t) {
    double H = c->y_hi - c->y_lo;
    return ramp_factor(t, c->o.ramp) * 4.0 * c->o.u_peak * (y - c->y_lo) * (c->y_hi - y) / (H * H);
}

/* classify the source node x - c_i of a pull for node (x, y):
 * 0 = fluid node inside (coordinates returned), 1 = half-way bounce-back
 * (cylinder or wall), 2 = open boundary, 3 = interpolated wall link.        */
static int ch_source(const channel *c, int x, int y, int i, int *xs, int *ys) {
    int sx = x - CX[i], sy = y - CY[i];
    if (sy < 0 || sy >= c->ny) return c->o.q_lo >= 0.0 ? 3 : 1;
    if (sx < 0 || sx >= c->nx) {
        if (c->o.xbc == 2) {
            sx = (sx + c->nx) % c->nx;
        } else if (c->o.xbc == 1) {
            return 1;
        } else {
            return 2;
        }
    }
    if (c->solid[(long)sy * c->nx + sx]) return c->o.cyl == 1 ? 3 : 1;
    *xs = sx;
    *ys = sy;
    return 0;
}

/* What the wall returns for pull direction i at fluid node (x, y), from the
 * post-collision field fs: half-way bounce-back f*_k(x), k = opp(i), or the
 * linear interpolation of Bouzidi et al. with link fraction q,
 *   q <  1/2: 2q f*_k(x) + (1 - 2q) f*_k(x - c_k)
 *   q >= 1/2: f*_k(x)/(2q) + (1 - 1/(2q)) f*_i(x)
 * (x - c_k = x + c_i; where that node is not fluid the half-way rule is
 * used).                                                                    */
static double wall_return(const channel *c, const double *fs, int x, int y, int i, int kind) {
    int nx = c->nx, ny = c->ny, k = OPP(i);
    double fk = fs[idx(k, y, x, nx, ny)];
    if (kind != 3) return fk;
    double q = c->q[idx(i, y, x, nx, ny)];
    if (q >= 0.5) return fk / (2.0 * q) + (1.0 - 1.0 / (2.0 * q)) * fs[idx(i, y, x, nx, ny)];
    int xb = x + CX[i], yb = y + CY[i];
    if (xb < 0 || xb >= nx || yb < 0 || yb >= ny || c->solid[(long)yb * nx + xb]) return fk;
    return 2.0 * q * fk + (1.0 - 2.0 * q) * fs[idx(k, yb, xb, nx, ny)];
}

/* Zou-He completion of the unknown populations at an open-column node. */
static void zou_he_inlet(double *f, double ux) {
    double rho = (f[0] + f[2] + f[4] + 2.0 * (f[3] + f[6] + f[7])) / (1.0 - ux);
    f[1] = f[3] + (2.0 / 3.0) * rho * ux;
    f[5] = f[7] - 0.5 * (f[2] - f[4]) + (1.0 / 6.0) * rho * ux;
    f[8] = f[6] + 0.5 * (f[2] - f[4]) + (1.0 / 6.0) * rho * ux;
}

static void zou_he_outlet(double *f) {
    double rho = 1.0;
    double ux = -1.0 + (f[0] + f[2] + f[4] + 2.0 * (f[1] + f[5] + f[8])) / rho;
    f[3] = f[1] - (2.0 / 3.0) * rho * ux;
    f[7] = f[5] + 0.5 * (f[2] - f[4]) - (1.0 / 6.0) * rho * ux;
    f[6] = f[8] - 0.5 * (f[2] - f[4]) - (1.0 / 6.0) * rho * ux;
}

/* Velocity and density imposed at open-column node (x, y) of the streamed
 * field f: inlet prescribed u and rho from the known populations, outlet
 * rho = 1, u_y = 0, u_x from the known populations (the Zou-He relations).  */
static void open_state(const channel *c, const double *f, int x, int y, long t, double *rho, double *ux,
                       double *uy) {
    int nx = c->nx, ny = c->ny;
    double g[9];
    for (int i = 0; i < 9; ++i) g[i] = f[idx(i, y, x, nx, ny)];
    if (x == 0) {
        *ux = inlet_ux(c, y, t);
        *uy = 0.0;
        *rho = (g[0] + g[2] + g[4] + 2.0 * (g[3] + g[6] + g[7])) / (1.0 - *ux);
    } else {
        *rho = 1.0;
        *ux = -1.0 + (g[0] + g[2] + g[4] + 2.0 * (g[1] + g[5] + g[8]));
        *uy = 0.0;
    }
}

/* finite-difference reconstruction of both open columns (xbc 3) on the
 * streamed field f, at time t                                               */
static void fd_open_columns(const channel *c, double *f, long t) {
    int nx = c->nx, ny = c->ny;
    double *U = malloc(sizeof(double) * 3 * ny * 2); /* rho, ux, uy per column node */
    for (int side = 0; side < 2; ++side) {
        int x = side == 0 ? 0 : nx - 1;
        for (int y = 0; y < ny; ++y) {
            double *u = U + 3 * (side * ny + y);
            open_state(c, f, x, y, t, &u[0], &u[1], &u[2]);
        }
    }
    for (int side = 0; side < 2; ++side) {
        int x = side == 0 ? 0 : nx - 1, s = side == 0 ? 1 : -1;
        for (int y = 0; y < ny; ++y) {
            const double *u = U + 3 * (side * ny + y);
            /* across the column: u at x, x + s, x + 2s (interior moments) */
            double r1, u1x, u1y, r2, u2x, u2y, g[9];
            for (int i = 0; i < 9; ++i) g[i] = f[idx(i, y, x + s, nx, ny)];
            moments(g, &r1, &u1x, &u1y);
            for (int i = 0; i < 9; ++i) g[i] = f[idx(i, y, x + 2 * s, nx, ny)];
            moments(g, &r2, &u2x, &u2y);
            double dxux = s * (-3.0 * u[1] + 4.0 * u1x - u2x) / 2.0;
            double dxuy = s * (-3.0 * u[2] + 4.0 * u1y - u2y) / 2.0;
            /* along the column: central, one-sided at the ends */
            const double *um, *uc = u, *up;
            double dyux, dyuy;
            if (y == 0) {
                up = U + 3 * (side * ny + 1);
                um = U + 3 * (side * ny + 2);
                dyux = (-3.0 * uc[1] + 4.0 * up[1] - um[1]) / 2.0;
                dyuy = (-3.0 * uc[2] + 4.0 * up[2] - um[2]) / 2.0;
            } else if (y == ny - 1) {
                um = U + 3 * (side * ny + ny - 2);
                up = U + 3 * (side * ny + ny - 3);
                dyux = (3.0 * uc[1] - 4.0 * um[1] + up[1]) / 2.0;
                dyuy = (3.0 * uc[2] - 4.0 * um[2] + up[2]) / 2.0;
            } else {
                um = U + 3 * (side * ny + y - 1);
                up = U + 3 * (side * ny + y + 1);
                dyux = (up[1] - um[1]) / 2.0;
                dyuy = (up[2] - um[2]) / 2.0;
            }
            for (int i = 0; i < 9; ++i) {
                double Qxx = CX[i] * CX[i] - CS2, Qyy = CY[i] * CY[i] - CS2, Qxy = CX[i] * CY[i];
                double QS = Qxx * dxux + Qyy * dyuy + Qxy * (dxuy + dyux);
                f[idx(i, y, x, nx, ny)] = feq(i, u[0], u[1], u[2]) - W(i) * u[0] * c->tau / CS2 * QS;
            }
        }
    }
    free(U);
}

static void channel_step(const channel *c, long t, double *f, double *fs) {
    int nx = c->nx, ny = c->ny;
    /* collision at every fluid node */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (c->solid[(long)y * nx + x]) continue;
            double a[9], b[9];
            for (int i = 0; i < 9; ++i) a[i] = f[idx(i, y, x, nx, ny)];
            collide(a, c->tau, b);
            for (int i = 0; i < 9; ++i) fs[idx(i, y, x, nx, ny)] = b[i];
        }
    /* streaming by pull, the wall rule where the source is not fluid, then
     * the open columns with the inflow of time t+1                         */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (c->solid[(long)y * nx + x]) continue;
            double g[9];
            int open = 0;
            for (int i = 0; i < 9; ++i) {
                int xs = 0, ys = 0;
                int k = ch_source(c, x, y, i, &xs, &ys);
                if (k == 0)
                    g[i] = fs[idx(i, ys, xs, nx, ny)];
                else if (k == 2) {
                    g[i] = 0.0;
                    open = 1;
                } else
                    g[i] = wall_return(c, fs, x, y, i, k);
            }
            if (open && c->o.xbc == 0) {
                if (x == 0)
                    zou_he_inlet(g, inlet_ux(c, y, t + 1));
                else
                    zou_he_outlet(g);
            }
            for (int i = 0; i < 9; ++i) f[idx(i, y, x, nx, ny)] = g[i];
        }
    if (c->o.xbc == 3) fd_open_columns(c, f, t + 1);
}

static int channel_setup(channel *c, const oracle_channel_opts *o) {
    memset(c, 0, sizeof *c);
    c->o = *o;
    c->nx = o->nx;
    c->ny = o->ny;
    c->tau = o->nu / CS2 + 0.5;
    if (!(c->tau > 0.5) || o->nx < 2 || o->ny < 3) return -1;
    if (o->xbc == 3 && (o->nx < 4 || o->ny < 3)) return -1;
    c->y_lo = o->q_lo >= 0.0 ? -o->q_lo : -0.5;
    c->y_hi = o->q_hi >= 0.0 ? (o->ny - 1) + o->q_hi : o->ny - 0.5;
    long n = (long)o->nx * o->ny;
    c->solid = calloc((size_t)n, 1);
    c->q = calloc((size_t)(9 * n), sizeof(double));
    for (int y = 0; y < o->ny; ++y)
        for (int x = 0; x < o->nx; ++x) c->solid[(long)y * o->nx + x] = (unsigned char)in_cylinder(c, x, y);
    for (int y = 0; y < o->ny; ++y)
        for (int x = 0; x < o->nx; ++x) {
            if (c->solid[(long)y * o->nx + x]) continue;
            for (int i = 1; i < 9; ++i) {
                int xs, ys;
                if (ch_source(c, x, y, i, &xs, &ys) != 3) continue;
                c->q[idx(i, y, x, o->nx, o->ny)] = o->q_fix >= 0.0 ? o->q_fix : link_fraction(c, x, y, i);
            }
        }
    return 0;
}

static void channel_free(channel *c) {
    free(c->solid);
    free(c->q);
}

/* Run one channel sample. Outputs (each may be NULL): f_out [9][ny][nx]
 * (solid nodes hold 0), rho/ux/uy [ny][nx] (0 at solid nodes), force[2]
 * = (F_x, F_y) at the final step, cd_cl[2], wall_force[2] (the same
 * momentum-exchange sum over the links into the channel walls: not a
 * quantity of interest, it closes the global momentum balance in tests),
 * q_out [9][ny][nx] (the link fractions).                                    */
int oracle_channel_run_opts(const oracle_channel_opts *o, double *f_out, double *rho_out, double *ux_out,
                            double *uy_out, double *force, double *cd_cl, double *wall_force, double *q_out) {
    channel c;
    if (channel_setup(&c, o) != 0) {
        channel_free(&c);
        return -1;
    }
    int nx = c.nx, ny = c.ny;
    long n = (long)nx * ny;
    double *f = calloc((size_t)(9 * n), sizeof(double)), *fs = calloc((size_t)(9 * n), sizeof(double));
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (c.solid[(long)y * nx + x]) continue;
            for (int i = 0; i < 9; ++i) f[idx(i, y, x, nx, ny)] = feq(i, 1.0, o->ux_init, 0.0);
        }
    for (long t = 0; t < o->steps; ++t) channel_step(&c, t, f, fs);

    /* collide the final state everywhere, then exchange momentum */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long cc = (long)y * nx + x;
            if (c.solid[cc]) {
                for (int i = 0; i < 9; ++i) fs[idx(i, y, x, nx, ny)] = 0.0;
                continue;
            }
            double a[9], b[9];
            for (int i = 0; i < 9; ++i) a[i] = f[idx(i, y, x, nx, ny)];
            collide(a, c.tau, b);
            for (int i = 0; i < 9; ++i) fs[idx(i, y, x, nx, ny)] = b[i];
        }
    nsum Fx = {0, 0}, Fy = {0, 0}, Wx = {0, 0}, Wy = {0, 0};
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long cc = (long)y * nx + x;
            if (c.solid[cc]) {
                if (rho_out) rho_out[cc] = 0.0;
                if (ux_out) ux_out[cc] = 0.0;
                if (uy_out) uy_out[cc] = 0.0;
                continue;
            }
            double a[9], rho, ux, uy;
            for (int i = 0; i < 9; ++i) a[i] = f[idx(i, y, x, nx, ny)];
            moments(a, &rho, &ux, &uy);
            if (rho_out) rho_out[cc] = rho;
            if (ux_out) ux_out[cc] = ux;
            if (uy_out) uy_out[cc] = uy;
            for (int k = 1; k < 9; ++k) {
                /* link x -> x + c_k meets a wall iff the pull of direction
                 * opp(k) at x has its source there                          */
                int xs = 0, ys = 0, i = OPP(k);
                int kind = ch_source(&c, x, y, i, &xs, &ys);
                if (kind != 1 && kind != 3) continue;
                double ex = fs[idx(k, y, x, nx, ny)] + wall_return(&c, fs, x, y, i, kind);
                int xn = x + CX[k], yn = y + CY[k];
                int into_cyl = xn >= 0 && xn < nx && yn >= 0 && yn < ny && c.solid[(long)yn * nx + xn];
                if (into_cyl) {
                    nadd(&Fx, CX[k] * ex);
                    nadd(&Fy, CY[k] * ex);
                } else {
                    nadd(&Wx, CX[k] * ex);
                    nadd(&Wy, CY[k] * ex);
                }
            }
        }
    double fx = nval(&Fx), fy = nval(&Fy);
    if (force) {
        force[0] = fx;
        force[1] = fy;
    }
    if (wall_force) {
        wall_force[0] = nval(&Wx);
        wall_force[1] = nval(&Wy);
    }
    if (cd_cl) {
        double D = o->cyl == 1 ? 2.0 * o->R : (double)o->D;
        double U = o->force_ref == 1 ? (2.0 / 3.0) * o->u_peak : o->u_peak;
        double q = 1.0 * U * U * D;
        cd_cl[0] = D > 0 ? 2.0 * fx / q : 0.0;
        cd_cl[1] = D > 0 ? 2.0 * fy / q : 0.0;
    }
    if (f_out) memcpy(f_out, f, sizeof(double) * 9 * n);
    if (q_out) memcpy(q_out, c.q, sizeof(double) * 9 * n);
    channel_free(&c);
    free(f);
    free(fs);
    return 0;
}

/* The half-way variant with the integer cylinder (the argument list of the
 * first channel interface).                                                 */
int oracle_channel_run(int nx, int ny, int xbc, int D, int cx, int cy, double nu, double u_peak, long ramp,
                       long steps, double ux_init, double *f_out, double *rho_out, double *ux_out, double *uy_out,
                       double *force, double *cd_cl, double *wall_force) {
    oracle_channel_opts o;
    memset(&o, 0, sizeof o);
    o.nx = nx;
    o.ny = ny;
    o.xbc = xbc;
    o.cyl = 0;
    o.D = D;
    o.cx = cx;
    o.cy = cy;
    o.q_lo = o.q_hi = o.q_fix = -1.0;
    o.nu = nu;
    o.u_peak = u_peak;
    o.ramp = ramp;
    o.steps = steps;
    o.ux_init = ux_init;
    return oracle_channel_run_opts(&o, f_out, rho_out, ux_out, uy_out, force, cd_cl, wall_force, NULL);
}

/* Count of solid cylinder nodes, for geometry checks. */
long oracle_cylinder_nodes(int nx, int ny, int D, int cx, int cy) {
    channel c;
    memset(&c, 0, sizeof c);
    c.o.D = D;
    c.o.cx = cx;
    c.o.cy = cy;
    long s = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) s += in_cylinder(&c, x, y);
    return s;
}

/* ------------------------------------------------------------------------ */
/* Sparse-grid collocation (Sec. "Quadrature and collocation": Clenshaw-
 * Curtis rules combined into sparse Smolyak grids).                         */

/* nested 1-D Clenshaw-Curtis rule of level i >= 1: 1 node (x = 0) at level 1,
 * else m = 2^(i-1) + 1 nodes x_j = -cos(pi j/(m-1)).                        */
int oracle_cc_points(int i) { return i <= 1 ? 1 : (1 << (i - 1)) + 1; }

/* Weights for the probability measure dx/2: the unique weights that
 * integrate the Chebyshev polynomials T_0..T_{m-1} exactly, found by solving
 * sum_j w_j T_k(x_j) = int T_k dx/2 (= 1/(1-k^2) for even k, 0 for odd k)
 * with Gaussian elimination and partial pivoting.                           */
int oracle_cc_rule(int i, double *x, double *w) {
    int m = oracle_cc_points(i);
    const double pi = acos(-1.0);
    if (m == 1) {
        x[0] = 0.0;
        w[0] = 1.0;
        return 1;
    }
    for (int j = 0; j < m; ++j) x[j] = -cos(pi * j / (m - 1));
    x[(m - 1) / 2] = 0.0;
    double *A = malloc(sizeof(double) * m * (m + 1));
    for (int k = 0; k < m; ++k) {
        for (int j = 0; j < m; ++j) A[k * (m + 1) + j] = cos(k * acos(x[j])); /* T_k(x_j) */
        A[k * (m + 1) + m] = (k % 2) ? 0.0 : 1.0 / (1.0 - (double)k * k);
    }
    for (int c = 0; c < m; ++c) {
        int piv = c;
        for (int r = c + 1; r < m; ++r)
            if (fabs(A[r * (m + 1) + c]) > fabs(A[piv * (m + 1) + c])) piv = r;
        for (int t = 0; t <= m; ++t) {
            double tmp = A[c * (m + 1) + t];
            A[c * (m + 1) + t] = A[piv * (m + 1) + t];
            A[piv * (m + 1) + t] = tmp;
        }
        for (int r = 0; r < m; ++r) {
            if (r == c) continue;
            double f = A[r * (m + 1) + c] / A[c * (m + 1) + c];
            for (int t = c; t <= m; ++t) A[r * (m + 1) + t] -= f * A[c * (m + 1) + t];
        }
    }
    for (int j = 0; j < m; ++j) w[j] = A[j * (m + 1) + m] / A[j * (m + 1) + j];
    free(A);
    return m;
}

/* Smolyak grid of level l in d dimensions by the difference formula
 *   A(l, d) = sum_{|i| <= l + d} D^{i_1} x ... x D^{i_d},
 *   D^1 = U^1, D^i = U^i - U^{i-1} (a signed rule on the nested nodes).
 * Nodes are keyed by their index on the finest grid (level l+1); the union of
 * all tensor grids is returned in lexicographic key order (input 0 first),
 * with the summed weights. Returns the number of nodes; xi/a may be NULL to
 * query it. Plain arrays: a dense table over the finest tensor grid.        */
long oracle_smolyak(int d, int l, double *xi, double *a) {
    int L = l + 1;
    int mf = oracle_cc_points(L);
    long cells = 1;
    for (int k = 0; k < d; ++k) cells *= mf;
    double *acc = calloc((size_t)cells, sizeof(double));
    unsigned char *used = calloc((size_t)cells, 1);
    /* difference rules on the finest index grid: D[i][idx] */
    double **D = malloc(sizeof(double *) * (L + 1));
    double *xs = malloc(sizeof(double) * mf), *ws = malloc(sizeof(double) * mf);
    for (int i = 1; i <= L; ++i) {
        D[i] = calloc((size_t)mf, sizeof(double));
        int m = oracle_cc_rule(i, xs, ws);
        for (int j = 0; j < m; ++j) {
            int key = m == 1 ? (mf - 1) / 2 : j * ((mf - 1) / (m - 1));
            D[i][key] += ws[j];
        }
        if (i > 1) {
            int mp = oracle_cc_rule(i - 1, xs, ws);
            for (int j = 0; j < mp; ++j) {
                int key = mp == 1 ? (mf - 1) / 2 : j * ((mf - 1) / (mp - 1));
                D[i][key] -= ws[j];
            }
        }
    }
    int *lev = malloc(sizeof(int) * d), *idx = malloc(sizeof(int) * d);
    for (int k = 0; k < d; ++k) lev[k] = 1;
    for (;;) {
        int s = 0;
        for (int k = 0; k < d; ++k) s += lev[k];
        if (s <= l + d) {
            /* every node of the finest grid that belongs to level lev[k] in
             * each input: D^{lev} is supported on the level-lev nodes        */
            for (int k = 0; k < d; ++k) idx[k] = 0;
            for (;;) {
                double w = 1.0;
                int member = 1;
                long flat = 0;
                for (int k = 0; k < d; ++k) {
                    int m = oracle_cc_points(lev[k]);
                    int step = m == 1 ? 0 : (mf - 1) / (m - 1);
                    int on = m == 1 ? (idx[k] == (mf - 1) / 2) : (idx[k] % step == 0);
                    if (!on) member = 0;
                    w *= D[lev[k]][idx[k]];
                    flat = flat * mf + idx[k];
                }
                if (member) {
                    acc[flat] += w;
                    used[flat] = 1;
                }
                int k = d - 1;
                while (k >= 0 && ++idx[k] == mf) idx[k--] = 0;
                if (k < 0) break;
            }
        }
        int k = d - 1;
        while (k >= 0 && ++lev[k] > L) lev[k--] = 1;
        if (k < 0) break;
    }
    const double pi = acos(-1.0);
    long S = 0;
    for (long c = 0; c < cells; ++c) {
        if (!used[c]) continue;
        if (xi) {
            long rem = c;
            for (int k = d - 1; k >= 0; --k) {
                int id = (int)(rem % mf);
                rem /= mf;
                double v = mf == 1 ? 0.0 : -cos(pi * id / (mf - 1));
                if (mf > 1 && 2 * id == mf - 1) v = 0.0;
                xi[S * d + k] = v;
            }
        }
        if (a) a[S] = acc[c];
        ++S;
    }
    for (int i = 1; i <= L; ++i) free(D[i]);
    free(D);
    free(xs);
    free(ws);
    free(lev);
    free(idx);
    free(acc);
    free(used);
    return S;
}

/* Quasi Monte Carlo (Sec. "Monte Carlo and quasi Monte Carlo sampling"):
 * Halton points with indices 1..N, input k in base = k-th prime: the base-p
 * digits of the index mirrored about the radix point, computed as an integer
 * digit reversal divided once by p^ndigits.                                 */
void oracle_halton(long N, int d, double *xi, double *a) {
    static const int primes[8] = {2, 3, 5, 7, 11, 13, 17, 19};
    for (long j = 0; j < N; ++j) {
        for (int k = 0; k < d; ++k) {
            unsigned long long n = (unsigned long long)(j + 1), rev = 0, den = 1, p = (unsigned long long)primes[k];
            while (n > 0) {
                rev = rev * p + n % p;
                den *= p;
                n /= p;
            }
            xi[j * d + k] = 2.0 * ((double)rev / (double)den) - 1.0;
        }
        a[j] = 1.0 / (double)N;
    }
}

/* Latin hypercube sampling (Sec. "Sampling strategies"): for input k the N
 * strata are shuffled by Fisher-Yates, exchanging position i (i = N-1 .. 1)
 * with position floor(r (i+1) / 2^64), r the SplitMix64 output number
 * c = k*2N + i + 1 of the generator seeded with `seed`; sample j then lies in
 * stratum perm[j] at fraction u = (output k*2N + N + j + 1 >> 11) 2^-53.     */
void oracle_lhs(uint64_t seed, long N, int d, double *xi, double *a) {
    long *perm = malloc(sizeof(long) * N);
    for (int k = 0; k < d; ++k) {
        for (long i = 0; i < N; ++i) perm[i] = i;
        uint64_t s = seed;
        /* run the generator to output number k*2N, then draw in order */
        for (long c = 0; c < (long)k * 2 * N; ++c) splitmix_next(&s);
        uint64_t *draws = malloc(sizeof(uint64_t) * 2 * N);
        for (long c = 0; c < 2 * N; ++c) draws[c] = splitmix_next(&s);
        for (long i = N - 1; i >= 1; --i) {
            uint64_t r = draws[i];
            long t = (long)(((unsigned __int128)r * (unsigned __int128)(i + 1)) >> 64);
            long tmp = perm[i];
            perm[i] = perm[t];
            perm[t] = tmp;
        }
        for (long j = 0; j < N; ++j) {
            double u = (double)(draws[N + j] >> 11) * (1.0 / 9007199254740992.0);
            xi[j * d + k] = 2.0 * (((double)perm[j] + u) / (double)N) - 1.0;
        }
        free(draws);
    }
    for (long j = 0; j < N; ++j) a[j] = 1.0 / (double)N;
    free(perm);
}
