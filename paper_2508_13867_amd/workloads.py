"""Problem definitions of the synthetic workloads (plain data, no arithmetic
of the method). Shapes follow the paper's two test cases (Taylor-Green vortex,
Sec. "Taylor--Green vortex flow with uncertain viscosity"; channel flow past a
cylinder, Sec. "Flow past a circular cylinder with uncertain inlet
velocity"); every input is uniform and every sample set is seeded or a
deterministic collocation rule. All values are in lattice units.

Each problem is a dict: geometry, precision, nx, ny, steps, nominal inputs,
dists = [(target, lo, hi)], rule = {kind: gl, n, order} | {kind: mc, N, seed}.
"""
from math import pi

SEED = 123456  # the seed of the paper's Monte Carlo example

# 64^2 FP64 vortex, nu ~ U(0.008, 0.012) at 5 Gauss-Legendre nodes, order 4
TGV_SMALL_FP64 = dict(
    name="tgv64_fp64_gl5", geometry="tgv", precision="fp64", nx=64, ny=64, steps=1000,
    u0=0.01, nu=0.01, dists=[("nu", 0.008, 0.012)], rule=dict(kind="gl", n=5, order=4),
)

FOUR_D_INPUTS = [("nu", 0.004, 0.006), ("u0", 0.018, 0.022), ("phase_x", 0.0, 2 * pi), ("phase_y", 0.0, 2 * pi)]

# 256^2 FP32 vortex, 4-D inputs, 4^4 = 256 collocation samples, order 3
TGV_BATCHED_FP32 = dict(
    name="tgv256_fp32_gl4x4", geometry="tgv", precision="fp32", nx=256, ny=256, steps=5000,
    u0=0.02, nu=0.005, dists=FOUR_D_INPUTS, rule=dict(kind="gl", n=4, order=3),
)

# 128^2 vortex, same inputs, 4096 Monte Carlo samples; precision swept
TGV_MC = dict(
    name="tgv128_mc4096", geometry="tgv", precision="fp32", nx=128, ny=128, steps=2000,
    u0=0.02, nu=0.005, dists=FOUR_D_INPUTS, rule=dict(kind="mc", N=4096, seed=SEED),
)

# 440 x 82 channel, cylinder D = 20 at (40, 41), Re ~ U(16, 24) via nu,
# u_peak ~ 0.05 (1 +- 0.1), 8 x 8 collocation, order 7, 20000 steps
CYLINDER_FP32 = dict(
    name="cyl440x82_fp32_gl8x8", geometry="channel", precision="fp32", nx=440, ny=82, steps=20000,
    u_peak=0.05, nu=0.05, D=20, cx=40, cy=41, ramp=4000, xbc="zouhe",
    dists=[("re", 16.0, 24.0), ("u_peak", 0.045, 0.055)], rule=dict(kind="gl", n=8, order=7),
)

# The paper's own cylinder set-up (Sec. "Flow past a circular cylinder with
# uncertain inlet velocity", Table tab:uq_results at n_x = 20): channel 22D x
# 4D with D = 20 nodes (walls half-way outside rows 0 and 79), the exact
# circle at (2D, (ny-1)/2) with interpolated bounce-back, finite-difference
# inlet/outlet, u_in(xi) = u(1 + 0.2 xi) (0.2 +- 0.04 relative), Re = 20 at
# the nominal inflow with nu fixed, C_D and Re on the mean inflow velocity
# (lattice mean 0.04, peak 0.06), 11-node Gauss-Legendre collocation.
CYLINDER_PAPER_FP32 = dict(
    name="cyl440x80_paper_fp32", geometry="channel", precision="fp32", nx=440, ny=80, steps=40000,
    u_peak=0.06, nu=0.04, cyl_bc="bouzidi", cyl_x=40.0, cyl_y=39.5, cyl_d=20.0, ramp=4000, xbc="interp",
    force_ref="mean", layout="ab", dists=[("u_peak", 0.048, 0.072)], rule=dict(kind="gl", n=11, order=10),
)

# the same with 1000 Monte Carlo samples: the batched form of that study
CYLINDER_PAPER_MC_FP32 = dict(CYLINDER_PAPER_FP32, name="cyl440x80_paper_mc1000_fp32",
                              rule=dict(kind="mc", N=1000, seed=SEED))

WORKLOADS = {w["name"]: w for w in (TGV_SMALL_FP64, TGV_BATCHED_FP32, TGV_MC, CYLINDER_FP32, CYLINDER_PAPER_FP32,
                                    CYLINDER_PAPER_MC_FP32)}


def scaled(spec, **over):
    """Copy of a workload with some entries replaced (smaller test cases)."""
    out = dict(spec)
    out.update(over)
    return out


def serving_trace(n_jobs=16, seed=SEED, load=1.2, rate_nodes_per_s=5.0e10, max_S_steps=7.0e5,
                  steps_range=(400, 3000)):
    """Seeded Poisson-arrival stream of UQ jobs (the serving mix): Taylor-Green
    vortices of 64^2..256^2 or cylinder channels of diameter 10..20 (22D x
    4.1D lattice), 1- to 4-D uniform inputs, tensor Gauss-Legendre rules of
    5..256 nodes or Monte Carlo with 256..1024 samples, FP32, steps
    log-uniform in steps_range with samples x steps capped at max_S_steps.
    Inter-arrival times are exponential with mean (mean job work) /
    (load x rate_nodes_per_s). Returns [(arrival_s, spec), ...]."""
    import numpy as np

    rng = np.random.default_rng(seed)
    jobs = []
    for q in range(n_jobs):
        steps = int(round(np.exp(rng.uniform(np.log(steps_range[0]), np.log(steps_range[1])))))
        if rng.random() < 0.6:
            n = int(rng.choice([64, 96, 128, 192, 256]))
            d = int(rng.integers(1, 5))
            dists = FOUR_D_INPUTS[:d] if d > 1 else [("nu", 0.004, 0.006)]
            if rng.random() < 0.5:
                per = {1: (5, 16), 2: (3, 16), 3: (2, 6), 4: (2, 4)}[d]
                npd = int(rng.integers(per[0], per[1] + 1))
                rule = dict(kind="gl", n=npd, order=min(npd - 1, 3))
                S = npd ** d
            else:
                S = int(rng.choice([256, 512, 1024]))
                rule = dict(kind="mc", N=S, seed=SEED + q)
            spec = dict(name=f"trace{q}_tgv{n}", geometry="tgv", precision="fp32", nx=n, ny=n, u0=0.02,
                        nu=0.005, dists=dists, rule=rule)
        else:
            D = int(rng.choice([10, 14, 20]))
            nx, ny = 22 * D, int(round(4.1 * D))
            d = int(rng.integers(1, 3))
            dists = [("re", 16.0, 24.0), ("u_peak", 0.045, 0.055)][:d]
            if rng.random() < 0.6:
                npd = int(rng.integers(3, 9)) if d == 2 else int(rng.integers(5, 17))
                rule = dict(kind="gl", n=npd, order=min(npd - 1, 5))
                S = npd ** d
            else:
                S = int(rng.choice([256, 512]))
                rule = dict(kind="mc", N=S, seed=SEED + q)
            spec = dict(name=f"trace{q}_cyl{D}", geometry="channel", precision="fp32", nx=nx, ny=ny, u_peak=0.05,
                        nu=0.05 * D / 20.0, D=D, cx=2 * D, cy=ny // 2, xbc="zouhe", dists=dists, rule=rule)
        steps = max(2, min(steps, int(max_S_steps / S)))
        spec["steps"] = steps
        if spec["geometry"] == "channel":
            spec["ramp"] = steps // 5
        spec["work"] = float(S) * spec["nx"] * spec["ny"] * steps
        jobs.append(spec)
    mean_service = sum(j["work"] for j in jobs) / len(jobs) / rate_nodes_per_s
    gaps = rng.exponential(mean_service / load, size=n_jobs)
    t = np.cumsum(gaps) - gaps[0]
    return [(float(a), j) for a, j in zip(t, jobs)]


def serving_mix(n_jobs=200, seed=SEED, max_work=2.0e11, steps_range=(1000, 20000)):
    """The serving mix at full scale: seeded UQ jobs, 60 % Taylor-Green
    vortices on 64^2..1024^2 lattices and 40 % cylinder channels of diameter
    10..40 (22D x 4.1D lattice, Zou-He inlet/outlet, half-way walls and
    cylinder), 1- to 4-D (vortex) or 1- to 2-D (channel) uniform inputs,
    tensor Gauss-Legendre rules of 5..256 nodes or Monte Carlo with
    256..4096 samples, FP32; steps log-uniform in steps_range, cut so that
    no job exceeds max_work node updates. Returns [spec, ...] in arrival
    order; arrival times are drawn by the caller (poisson_arrivals)."""
    import numpy as np

    rng = np.random.default_rng(seed)
    jobs = []
    for q in range(n_jobs):
        steps = int(round(np.exp(rng.uniform(np.log(steps_range[0]), np.log(steps_range[1])))))
        mc = rng.random() < 0.5
        if rng.random() < 0.6:
            n = int(rng.choice([64, 128, 192, 256, 384, 512, 768, 1024]))
            nx = ny = n
            d = int(rng.integers(1, 5))
            dists = FOUR_D_INPUTS[:d] if d > 1 else [("nu", 0.004, 0.006)]
            per = {1: (5, 16), 2: (3, 16), 3: (2, 6), 4: (2, 4)}[d]
            spec = dict(name=f"mix{q}_tgv{n}", geometry="tgv", precision="fp32", nx=nx, ny=ny, u0=0.02,
                        nu=0.005, dists=dists)
        else:
            D = int(rng.choice([10, 14, 20, 28, 40]))
            nx, ny = 22 * D, int(round(4.1 * D))
            d = int(rng.integers(1, 3))
            dists = [("re", 16.0, 24.0), ("u_peak", 0.045, 0.055)][:d]
            per = {1: (5, 16), 2: (3, 16)}[d]
            spec = dict(name=f"mix{q}_cyl{D}", geometry="channel", precision="fp32", nx=nx, ny=ny, u_peak=0.05,
                        nu=0.05 * D / 20.0, D=D, cx=2 * D, cy=ny // 2, xbc="zouhe", dists=dists)
        if mc:
            S = int(rng.choice([256, 512, 1024, 2048, 4096]))
            spec["rule"] = dict(kind="mc", N=S, seed=SEED + q)
        else:
            npd = int(rng.integers(per[0], per[1] + 1))
            spec["rule"] = dict(kind="gl", n=npd, order=min(npd - 1, 3))
            S = npd ** d
        steps = max(2, min(steps, int(max_work / (S * nx * ny))))
        spec["steps"] = steps
        if spec["geometry"] == "channel":
            spec["ramp"] = steps // 5
        spec["work"] = float(S) * nx * ny * steps
        jobs.append(spec)
    return jobs


def poisson_arrivals(jobs, rate_nodes_per_s, load, seed=SEED + 1):
    """Seeded Poisson arrival times for `jobs` at an offered load of `load`
    times a service rate of rate_nodes_per_s node updates per second: the
    mean inter-arrival time is the mean job work / (load * rate)."""
    import numpy as np

    rng = np.random.default_rng(seed)
    mean_service = sum(j["work"] for j in jobs) / len(jobs) / rate_nodes_per_s
    gaps = rng.exponential(mean_service / load, size=len(jobs))
    return [float(t) for t in np.cumsum(gaps) - gaps[0]]


# 128^2 vortex, 4-D inputs, level-3 Smolyak sparse grid of nested
# Clenshaw-Curtis rules (137 points, the paper's sparse-grid size), order 3
TGV_SMOLYAK = dict(
    name="tgv128_smolyak_l3", geometry="tgv", precision="fp32", nx=128, ny=128, steps=2000,
    u0=0.02, nu=0.005, dists=FOUR_D_INPUTS, rule=dict(kind="smolyak", level=3, order=3),
)
WORKLOADS[TGV_SMOLYAK["name"]] = TGV_SMOLYAK


# Four-dimensional perturbed vortex (Sec. "Taylor--Green vortex flow with
# four-dimensional uncertain initial velocity perturbation"): zeta_ij ~
# U(-0.025, 0.025) i.i.d., N = n Monte Carlo samples, Ma = 1.6 / n,
# Re = 40 n, lattice units of Table tab:simulation_parameters, T_max = 100.
ZETA_INPUTS = [("zeta00", -0.025, 0.025), ("zeta01", -0.025, 0.025), ("zeta10", -0.025, 0.025),
               ("zeta11", -0.025, 0.025)]
TGV4D_T_MAX = 100.0


def tgv4d(n, units, precision="fp32", seed=SEED):
    """The perturbed-vortex problem at resolution n; units is the result of
    tgv_units(n, 1.6 / n, 40 n) (lattice viscosity and velocity)."""
    return dict(name=f"tgv4d_{n}", geometry="tgv", init="harmonic", precision=precision, nx=n, ny=n, steps=0,
                u0=units["u_lat"], nu=units["nu"], dists=ZETA_INPUTS, rule=dict(kind="mc", N=n, seed=seed + n))
