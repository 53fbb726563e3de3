"""GPU parity of the four-dimensional perturbed vortex and of the device
1-Wasserstein distance: populations and speed statistics of the harmonic
initial field against the FP64 oracle, and W_1 between two jobs' laws of |u|
against the oracle's own W_1 (and SciPy) on the oracle's fields, plus at the
full resolution pair of the convergence study against SciPy on the library's
own fields."""
import sys

import numpy as np
import pytest

import oracle as O
from helpers import gpu_available, rel_l2
from paper_2508_13867_amd import Job, UQError, tgv_units, wasserstein1
from paper_2508_13867_amd import _abi as A
from paper_2508_13867_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


ZETA = [("zeta00", -0.025, 0.025), ("zeta01", -0.025, 0.025), ("zeta10", -0.025, 0.025),
        ("zeta11", -0.025, 0.025)]


def harmonic(nx, ny, steps, prec="fp64", N=6, seed=7, u0=0.04, nu=0.01, **kw):
    return dict(name=f"tgv4d_{nx}x{ny}", geometry="tgv", init="harmonic", precision=prec, nx=nx, ny=ny,
                steps=steps, u0=u0, nu=nu, dists=ZETA, rule=dict(kind="mc", N=N, seed=seed), **kw)


@pytest.mark.parametrize("layout", ["aa", "ab"])
@pytest.mark.parametrize("steps", [0, 1, 33])
def test_harmonic_init_populations_match_oracle(steps, layout):
    spec = harmonic(72, 40, steps, layout=layout)
    say("case harmonic 72x40 fp64 steps", steps, layout)
    with Job(spec) as job:
        job.run(steps)
        xi, _ = job.samples()
        for s in (0, 3, 5):
            p = O.sample_params(spec, xi[s])
            z = [p["zeta00"], p["zeta01"], p["zeta10"], p["zeta11"]]
            ref = O.tgv_harmonic_run(72, 40, p["nu"], p["u0"], z, steps, want_f=True)["f"]
            got = job.populations(s)
            assert np.abs(got - ref).max() < 1e-13, (s, np.abs(got - ref).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_harmonic_speed_statistics_match_oracle(prec):
    spec = harmonic(48, 48, 120, prec=prec, N=8)
    say("case harmonic 48x48 speed moments", prec)
    ref = O.run_problem(spec, qois=["speed", "ke"])
    tol = 1e-10 if prec == "fp64" else 1e-4
    with Job(spec) as job:
        job.run(spec["steps"])
        sp = job.qoi_samples("speed")
        assert rel_l2(sp, ref["samples"]["speed"].reshape(8, -1)) < tol
        st = job.moments("speed")
        for k in ("mean", "var"):
            assert rel_l2(st[k], ref["stats"]["speed"][k]) < tol, k


def test_wasserstein1_matches_oracle_and_scipy():
    from scipy.stats import wasserstein_distance as wd
    a_spec = harmonic(32, 32, 60, N=5, seed=3)
    b_spec = harmonic(48, 48, 90, N=7, seed=4)
    say("case W1 32^2 vs 48^2 fp64")
    ra = O.run_problem(a_spec, qois=["speed"])["samples"]["speed"].reshape(-1)
    rb = O.run_problem(b_spec, qois=["speed"])["samples"]["speed"].reshape(-1)
    sa, sb = 1 / 0.04, 1 / 0.03
    ref = O.wasserstein1(ra * sa, np.ones(ra.size), rb * sb, np.ones(rb.size))
    assert abs(ref - wd(ra * sa, rb * sb)) < 1e-12
    with Job(a_spec) as A_, Job(b_spec) as B_:
        A_.run(a_spec["steps"])
        B_.run(b_spec["steps"])
        w = wasserstein1(A_, B_, "speed", sa, sb)
        assert abs(w - ref) <= 1e-10 * ref, (w, ref)
        # symmetric, zero on itself, scales linearly
        assert abs(wasserstein1(B_, A_, "speed", sb, sa) - w) <= 1e-12 * w
        assert wasserstein1(A_, A_, "speed", sa, sa) == 0.0
        w2 = wasserstein1(A_, B_, "speed", 2 * sa, 2 * sb)
        assert abs(w2 - 2 * w) <= 1e-12 * w
        # velocity components pooled: the law of (ux, uy) values
        wv = wasserstein1(A_, B_, "vel", 1.0, 1.0)
        va = A_.qoi_samples("vel").reshape(-1)
        vb = B_.qoi_samples("vel").reshape(-1)
        assert abs(wv - wd(va, vb)) <= 1e-10 * wv
        with pytest.raises(UQError) as e:
            wasserstein1(A_, B_, "ke")
        assert e.value.status == A.UQ_EINVAL


def test_wasserstein1_weighted_rule_and_rejected_signed_weights():
    from scipy.stats import wasserstein_distance as wd
    gl = dict(harmonic(24, 24, 40), rule=dict(kind="gl", n=2, order=1))  # 16 weighted samples
    mc = harmonic(24, 24, 40, N=3, seed=9)
    sm = dict(harmonic(24, 24, 40), rule=dict(kind="smolyak", level=2, order=2))
    say("case W1 weighted")
    with Job(gl) as G, Job(mc) as M, Job(sm) as S:
        for j, s in ((G, gl), (M, mc), (S, sm)):
            j.run(s["steps"])
        _, a = G.samples()
        cg, cm = G.qoi_samples("speed"), M.qoi_samples("speed")
        wg = np.repeat(a / cg.shape[1], cg.shape[1])
        ref = wd(cg.reshape(-1), cm.reshape(-1), wg, np.ones(cm.size))
        assert abs(wasserstein1(G, M, "speed") - ref) <= 1e-10 * ref
        _, a_s = S.samples()
        assert (a_s < 0).any()
        with pytest.raises(UQError):
            wasserstein1(S, M, "speed")


def test_wasserstein1_study_pair_fp32_full_size():
    # the largest pair of the convergence study: n = 256 with 256 samples
    # (16.8 M values) against n = 64 with 64 samples, Table
    # tab:simulation_parameters units, after a few hundred steps; the device
    # W_1 against SciPy on the library's own fields.
    from scipy.stats import wasserstein_distance as wd
    jobs, vals, scales = [], [], []
    try:
        for n in (256, 64):
            u = tgv_units(n, 1.6 / n, 40.0 * n)
            spec = harmonic(n, n, 0, prec="fp32", N=n, seed=W.SEED + n, u0=u["u_lat"], nu=u["nu"])
            j = Job(spec)
            jobs.append(j)
            say("case W1 study pair n", n, "steps", 8 * n)
            j.run(8 * n)
            vals.append(j.qoi_samples("speed").reshape(-1))
            scales.append(1.0 / u["u_lat"])
        w = wasserstein1(jobs[0], jobs[1], "speed", scales[0], scales[1])
        ref = wd(vals[0] * scales[0], vals[1] * scales[1])
        say("W1", w, "scipy", ref)
        assert abs(w - ref) <= 1e-9 * ref
    finally:
        for j in jobs:
            j.close()
