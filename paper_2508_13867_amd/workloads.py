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

WORKLOADS = {w["name"]: w for w in (TGV_SMALL_FP64, TGV_BATCHED_FP32, TGV_MC, CYLINDER_FP32)}


def scaled(spec, **over):
    """Copy of a workload with some entries replaced (smaller test cases)."""
    out = dict(spec)
    out.update(over)
    return out
