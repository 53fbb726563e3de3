"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle on
identical seeded inputs. Tolerances are the relative-L2 bars of the design:
1e-10 for FP64 runs, 1e-4 for FP32, 5e-3 for FP16 storage (BF16 storage is
reported against a looser 5e-2). Sizes are chosen so the oracle finishes in
seconds while the lattices span several 64 x (4 cpt) tiles with ragged edges;
full-size workloads are checked on sampled samples."""
import os
import sys
from math import pi

import numpy as np
import pytest

import oracle as O
from helpers import assert_stats, assert_stats_given_samples, gpu_available, rel_l2, stat_errors
from paper_2508_13867_amd import Job, UQError
from paper_2508_13867_amd import _abi as A
from paper_2508_13867_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = {"fp64": 1e-10, "fp32": 1e-4, "fp16s": 5e-3, "bf16s": 5e-2}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_fields(spec, samples=None):
    return O.run_problem(spec, samples=samples)


# ----------------------------------------------------------------- small TGV, FP64

TGV_RAGGED = dict(name="tgv72x40", geometry="tgv", precision="fp64", nx=72, ny=40, steps=40, u0=0.03, nu=0.02,
                  dists=[("nu", 0.01, 0.03), ("u0", 0.02, 0.04)], rule=dict(kind="gl", n=3, order=2),
                  phase_x=0.3, phase_y=-0.7)


@pytest.mark.parametrize("layout", ["aa", "ab"])
@pytest.mark.parametrize("steps", [0, 1, 2, 7, 40])
def test_tgv_fp64_populations_match_oracle(steps, layout):
    say("case tgv72x40 fp64 steps", steps, layout)
    with Job(W.scaled(TGV_RAGGED, layout=layout)) as job:
        job.run(steps)
        xi, a = job.samples()
        for s in (0, 4, 8):
            p = O.sample_params(TGV_RAGGED, xi[s])
            ref = O.tgv_run(72, 40, p["nu"], p["u0"], steps, p["phase_x"], p["phase_y"], want_f=True)["f"]
            got = job.populations(s)
            assert np.abs(got - ref).max() < 1e-13, (s, np.abs(got - ref).max())


@pytest.mark.parametrize("layout", ["aa", "ab"])
def test_tgv_fp64_moments_match_oracle(layout):
    say("case tgv72x40 fp64 moments", layout)
    ref = O.run_problem(TGV_RAGGED)
    with Job(W.scaled(TGV_RAGGED, layout=layout)) as job:
        job.run(TGV_RAGGED["steps"])
        ke = job.qoi_samples("ke")[:, 0]
        assert rel_l2(ke, ref["samples"]["ke"]) < TOL["fp64"]
        vel = job.qoi_samples("vel")
        assert rel_l2(vel, ref["samples"]["vel"].reshape(9, -1)) < TOL["fp64"]
        for q in ("ke", "vel", "rho"):
            st = job.moments(q)
            rs = ref["stats"][q]
            for k in ("mean", "var", "var_alt", "coeffs"):
                assert rel_l2(st[k], rs[k]) < TOL["fp64"], (q, k, rel_l2(st[k], rs[k]))
            assert_stats(st, rs, TOL["fp64"], q)
            assert np.array_equal(st["alpha"], ref["alpha"])


def test_config1_tgv64_fp64_full():
    # the 64^2 FP64 collocation workload at full size (5 samples, 1000 steps)
    spec = W.TGV_SMALL_FP64
    say("case", spec["name"])
    ref = O.run_problem(spec)
    with Job(spec) as job:
        job.run(spec["steps"])
        for q in ("ke", "vel"):
            st = job.moments(q)
            rs = ref["stats"][q]
            for k in ("mean", "var", "var_alt", "coeffs"):
                assert rel_l2(st[k], rs[k]) < TOL["fp64"], (q, k, rel_l2(st[k], rs[k]))
            assert_stats(st, rs, TOL["fp64"], q)


# ----------------------------------------------------------------- reduced precisions

TGV_4D_SMALL = dict(name="tgv96x80_4d", geometry="tgv", precision="fp32", nx=96, ny=80, steps=300, u0=0.02,
                    nu=0.005, dists=W.FOUR_D_INPUTS, rule=dict(kind="gl", n=2, order=1))


@pytest.fixture(scope="module")
def tgv4d_ref():
    return O.run_problem(TGV_4D_SMALL)


@pytest.mark.parametrize("layout", ["aa", "ab"])
@pytest.mark.parametrize("prec", ["fp32", "fp16s", "bf16s"])
def test_tgv_4d_reduced_precision(prec, layout, tgv4d_ref):
    spec = W.scaled(TGV_4D_SMALL, precision=prec, layout=layout)
    say("case tgv96x80_4d", prec, layout)
    ref = tgv4d_ref
    tol = TOL[prec]
    with Job(spec) as job:
        job.run(spec["steps"])
        ke = job.qoi_samples("ke")[:, 0]
        assert rel_l2(ke, ref["samples"]["ke"]) < tol
        vel = job.qoi_samples("vel")
        vref = ref["samples"]["vel"].reshape(vel.shape)
        assert rel_l2(vel, vref) < tol
        st = job.moments("ke")
        for k in ("mean", "var", "coeffs"):
            assert rel_l2(st[k], ref["stats"]["ke"][k]) < tol, (k, rel_l2(st[k], ref["stats"]["ke"][k]))
        # var, var_alt and the k >= 1 coefficients each on their own norm
        assert_stats(st, ref["stats"]["ke"], tol, "ke " + prec)
        sv = job.moments("vel")
        # the mean velocity under uniform phases is near zero: normalise the
        # field mean by the RMS of the per-sample fields; the variance and
        # the k >= 1 coefficients (which carry it) on their own norms
        rms = np.sqrt(np.mean(vref ** 2)) * np.sqrt(vref.shape[1])
        assert rel_l2(sv["coeffs"], ref["stats"]["vel"]["coeffs"], scale=rms) < tol
        assert_stats(sv, ref["stats"]["vel"], tol, "vel " + prec, mean_scale=rms)
        # storage: FP16S holds the shifted populations times 2^s as halves,
        # BF16S holds them unscaled as bfloat16, FP32 as floats
        inf = job.info()
        w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]
        t = job.populations(1) - w
        t = t[np.abs(t) > 1e-12]  # where w + f~ is exact in double
        if prec == "fp16s":
            assert inf.scale_exp > 0
            v = t * 2.0 ** inf.scale_exp
            assert np.array_equal(v.astype(np.float16).astype(np.float64), v)
        else:
            assert inf.scale_exp == 0
            f32 = t.astype(np.float32)
            assert np.array_equal(f32.astype(np.float64), t)
            if prec == "bf16s":
                assert not (f32.view(np.uint32) & 0xFFFF).any()


def test_tgv_monte_carlo_fp32():
    spec = dict(name="tgv48_mc", geometry="tgv", precision="fp32", nx=48, ny=48, steps=200, u0=0.02, nu=0.005,
                dists=W.FOUR_D_INPUTS, rule=dict(kind="mc", N=32, seed=W.SEED + 7))
    say("case", spec["name"])
    ref = O.run_problem(spec)
    with Job(spec) as job:
        xi, a = job.samples()
        assert np.array_equal(xi, ref["xi"]) and np.array_equal(a, ref["a"])
        job.run(spec["steps"])
        st = job.moments("ke")
        assert_stats(st, ref["stats"]["ke"], TOL["fp32"], "ke mc")
        assert "coeffs" not in st
        # Monte Carlo statistics of a field, formed from the populations
        vel = job.qoi_samples("vel")
        r = dict(ref, samples_q=ref["samples"]["vel"], stats_q=ref["stats"]["vel"])
        assert_stats_given_samples(job.moments("vel"), vel, r, TOL["fp32"], "vel mc")


# ----------------------------------------------------------------- channel

CHANNEL_SMALL = dict(name="chan100x41", geometry="channel", precision="fp64", nx=100, ny=41, steps=401,
                     u_peak=0.05, nu=0.05, D=10, cx=25, cy=18, ramp=200, xbc="zouhe",
                     dists=[("re", 16.0, 24.0), ("u_peak", 0.045, 0.055)], rule=dict(kind="gl", n=2, order=1))


@pytest.mark.parametrize("layout", ["aa", "ab"])
@pytest.mark.parametrize("steps", [0, 1, 2, 201, 401])
def test_channel_fp64_populations(steps, layout):
    say("case chan100x41 fp64 steps", steps, layout)
    with Job(W.scaled(CHANNEL_SMALL, layout=layout)) as job:
        job.run(steps)
        xi, a = job.samples()
        for s in (0, 3):
            p = O.sample_params(CHANNEL_SMALL, xi[s])
            ref = O.channel_run(100, 41, p["nu"], p["u_peak"], steps, D=10, cx=25, cy=18, ramp=200,
                                want_f=True)["f"]
            got = job.populations(s)
            assert np.abs(got - ref).max() < 1e-13, (s, np.abs(got - ref).max())


@pytest.mark.parametrize("layout", ["aa", "ab"])
def test_channel_fp64_drag_lift_moments(layout):
    say("case chan100x41 fp64 moments", layout)
    ref = O.run_problem(CHANNEL_SMALL)
    with Job(W.scaled(CHANNEL_SMALL, layout=layout)) as job:
        job.run(CHANNEL_SMALL["steps"])
        for q in ("cd", "cl"):
            got = job.qoi_samples(q)[:, 0]
            assert rel_l2(got, ref["samples"][q]) < TOL["fp64"], q
            st = job.moments(q)
            for k in ("mean", "var", "coeffs"):
                assert rel_l2(st[k], ref["stats"][q][k]) < TOL["fp64"], (q, k)
            assert_stats(st, ref["stats"][q], TOL["fp64"], q)
        st = job.moments("vel")
        assert rel_l2(st["coeffs"], ref["stats"]["vel"]["coeffs"]) < TOL["fp64"]
        assert_stats(st, ref["stats"]["vel"], TOL["fp64"], "vel")


@pytest.mark.parametrize("n", [2, 3, 4])
@pytest.mark.parametrize("rows", [8, 64])
@pytest.mark.parametrize("steps", [2, 7, 201, 401])
def test_fused_channel_populations_match_oracle(steps, rows, n, monkeypatch):
    # the full-row window on the channel (half-way walls and cylinder, Zou-He
    # ends, the inflow ramp ending at step 200): FP64 against the oracle,
    # counts that leave single steps after the fused blocks, chunks of 8
    # rows (halos next to the walls) and of the whole height
    monkeypatch.setenv("UQ_FUSE", str(n))
    monkeypatch.setenv("UQ_FUSE_TY", str(rows))
    monkeypatch.setenv("UQ_FUSE_WINDOW", "2")
    spec = W.scaled(CHANNEL_SMALL, layout="ab")
    say("case fused channel", n, "steps", steps, "rows", rows)
    with Job(spec) as job:
        assert job.info().fused == n and job.info().fused_window == 2
        job.run(steps)
        xi, _ = job.samples()
        for s in (0, 3):
            p = O.sample_params(CHANNEL_SMALL, xi[s])
            ref = O.channel_run(100, 41, p["nu"], p["u_peak"], steps, D=10, cx=25, cy=18, ramp=200,
                                want_f=True)["f"]
            got = job.populations(s)
            assert np.abs(got - ref).max() < 1e-13, (s, np.abs(got - ref).max())


@pytest.mark.parametrize("xbc", ["walls", "periodic"])
@pytest.mark.parametrize("n", [3, 4])
def test_fused_channel_wall_and_periodic_ends(xbc, n, monkeypatch):
    monkeypatch.setenv("UQ_FUSE", str(n))
    monkeypatch.setenv("UQ_FUSE_TY", "16")
    monkeypatch.setenv("UQ_FUSE_WINDOW", "2")
    spec = W.scaled(CHANNEL_SMALL, layout="ab", xbc=xbc, ramp=0)
    say("case fused channel", xbc, n)
    with Job(spec) as job:
        assert job.info().fused == n
        job.run(37)
        xi, _ = job.samples()
        p = O.sample_params(spec, xi[1])
        code = {"walls": 1, "periodic": 2}[xbc]
        ref = O.channel_run(100, 41, p["nu"], p["u_peak"], 37, D=10, cx=25, cy=18, xbc=code, want_f=True)["f"]
        got = job.populations(1)
        # (a channel without inflow stays at rest: this checks that the end
        # columns and walls bring in nothing from unwritten LDS)
        assert np.all(np.isfinite(got)) and np.abs(got - ref).max() < 1e-13


@pytest.mark.parametrize("nx, ny", [(5, 3), (64, 9), (129, 7)])
def test_fused_channel_small_lattices(nx, ny, monkeypatch):
    # three rows (every row touches a wall), a single wave of columns, and
    # one column past two waves; no cylinder
    monkeypatch.setenv("UQ_FUSE", "3")
    monkeypatch.setenv("UQ_FUSE_TY", "8")
    monkeypatch.setenv("UQ_FUSE_WINDOW", "2")
    spec = W.scaled(CHANNEL_SMALL, nx=nx, ny=ny, D=0, layout="ab", ramp=10,
                    dists=[("nu", 0.04, 0.06), ("u_peak", 0.045, 0.055)])
    say("case fused channel", nx, ny)
    with Job(spec) as job:
        assert job.info().fused == 3
        job.run(29)
        xi, _ = job.samples()
        p = O.sample_params(spec, xi[2])
        ref = O.channel_run(nx, ny, p["nu"], p["u_peak"], 29, ramp=10, want_f=True)["f"]
        assert np.abs(job.populations(2) - ref).max() < 1e-13


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s", "bf16s"])
def test_fused_channel_matches_single_steps(prec, monkeypatch):
    spec = W.scaled(CHANNEL_SMALL, precision=prec, layout="ab", steps=300)
    say("case fused channel vs single", prec)
    res = {}
    for fuse in ("0", "3"):
        monkeypatch.setenv("UQ_FUSE", fuse)
        monkeypatch.setenv("UQ_FUSE_TY", "16")
        monkeypatch.setenv("UQ_FUSE_WINDOW", "2")
        with Job(spec) as job:
            job.run(300)
            res[fuse] = (job.populations(1), job.qoi_samples("cd")[:, 0])
    # the same rules and the same operations in the same order, every fma
    # explicit and no implicit contraction: bit for bit the same populations
    # and drag, also where storage rounds to 16 bits
    assert np.array_equal(res["0"][0], res["3"][0])
    assert np.array_equal(res["0"][1], res["3"][1])


def test_autotune_channel_includes_fused_candidates(tmp_path, monkeypatch):
    # 100 x 41 channel, FP64, layout left to the tuner: 8 AA and 16 AB
    # single-step shapes (64- and 128-wide workgroups), plus the fused channel
    # kernel at 2, 3 and 4 steps on 1, 2, 3 and 4 row chunks (41, 21, 14, 11
    # rows); the job then runs in the chosen shape and matches the oracle
    monkeypatch.setenv("UQ_TUNE_CACHE", str(tmp_path / "tune.txt"))
    for k in ("UQ_FUSE", "UQ_FUSE_TY", "UQ_FUSE_WINDOW", "UQ_NT_STORE", "UQ_LAYOUT"):
        monkeypatch.delenv(k, raising=False)
    spec = W.scaled(CHANNEL_SMALL, name="chan100x41_tuned", steps=121)
    say("case channel autotune")
    r = A.autotune(spec, steps=120)
    assert r["n_candidates"] == 36
    with Job(spec) as job:
        inf = job.info()
        assert (inf.fused, inf.fused_window, inf.fused_rows) == (r["fused"], r["fused_window"], r["fused_rows"])
        job.run(spec["steps"])
        xi, _ = job.samples()
        p = O.sample_params(spec, xi[2])
        ref = O.channel_run(100, 41, p["nu"], p["u_peak"], spec["steps"], D=10, cx=25, cy=18, ramp=200,
                            want_f=True)["f"]
        assert np.abs(job.populations(2) - ref).max() < 1e-13


def test_fused_channel_refused_for_interpolated_rules(monkeypatch):
    # Bouzidi links and finite-difference columns need the boundary-node
    # kernels: such jobs are not fused, whatever the shape asks for
    monkeypatch.setenv("UQ_FUSE", "3")
    monkeypatch.setenv("UQ_FUSE_WINDOW", "2")
    spec = dict(name="chan70x27_interp", geometry="channel", precision="fp64", nx=70, ny=27, steps=20,
                u_peak=0.06, nu=0.04, cyl_bc="bouzidi", cyl_x=17.3, cyl_y=12.6, cyl_d=8.6, ramp=120,
                xbc="interp", force_ref="mean", layout="ab", dists=[("re", 16.0, 24.0)],
                rule=dict(kind="gl", n=2, order=1))
    with Job(spec) as job:
        assert job.info().fused == 0
    monkeypatch.setenv("UQ_FUSE_WINDOW", "1")
    with Job(W.scaled(CHANNEL_SMALL, layout="ab")) as job:
        assert job.info().fused == 0  # strips and tiles are periodic-only


def test_fused_cylinder_config_fp32_sampled(monkeypatch):
    # the 440 x 82 cylinder workload (64 samples), 3 steps per launch over
    # whole rows (4 waves of two columns per lane per step), 600 steps; two
    # samples re-solved by the oracle
    monkeypatch.setenv("UQ_FUSE", "3")
    monkeypatch.setenv("UQ_FUSE_TY", "256")
    monkeypatch.setenv("UQ_FUSE_WINDOW", "2")
    monkeypatch.setenv("UQ_NT_STORE", "0")
    spec = W.scaled(W.CYLINDER_FP32, steps=600, layout="ab")
    say("case", spec["name"], "fused 3, 600 steps")
    with Job(spec) as job:
        assert job.info().fused == 3
        job.run(spec["steps"])
        cd = job.qoi_samples("cd")[:, 0]
        vel = job.qoi_samples("vel")
        ref = O.run_problem(spec, samples=[0, 63])
        assert rel_l2(cd[[0, 63]], ref["samples"]["cd"]) < TOL["fp32"]
        assert rel_l2(vel[[0, 63]], ref["samples"]["vel"].reshape(2, -1)) < TOL["fp32"]


@pytest.mark.parametrize("layout", ["aa", "ab"])
def test_cylinder_config_geometry_fp32_sampled(layout):
    # the 440 x 82 cylinder workload (64 samples) at reduced steps; two
    # samples are re-solved by the oracle one by one
    spec = W.scaled(W.CYLINDER_FP32, steps=600, layout=layout)
    say("case", spec["name"], "600 steps", layout)
    with Job(spec) as job:
        job.run(spec["steps"])
        xi, a = job.samples()
        cd = job.qoi_samples("cd")[:, 0]
        cl = job.qoi_samples("cl")[:, 0]
        vel = job.qoi_samples("vel")
        ref = O.run_problem(spec, samples=[0, 63])
        assert rel_l2(cd[[0, 63]], ref["samples"]["cd"]) < TOL["fp32"]
        assert rel_l2(vel[[0, 63]], ref["samples"]["vel"].reshape(2, -1)) < TOL["fp32"]
        assert np.all(np.isfinite(cl))
        st = job.moments("cd")
        assert st["coeffs"].shape == (36, 1)


# ----------------------------------------------------------------- full-size batched TGV

@pytest.mark.parametrize("layout", ["aa", "ab"])
def test_batched_tgv256_fp32_sampled(layout):
    # 256^2 x 256 samples in the benchmark's launch configuration, 100 steps;
    # three samples re-solved by the oracle
    spec = W.scaled(W.TGV_BATCHED_FP32, steps=100, layout=layout)
    say("case", spec["name"], "100 steps", layout)
    with Job(spec) as job:
        job.run(spec["steps"])
        ke = job.qoi_samples("ke")[:, 0]
        vel = job.qoi_samples("vel")
        pick = [0, 137, 255]
        ref = O.run_problem(spec, samples=pick)
        assert rel_l2(ke[pick], ref["samples"]["ke"]) < TOL["fp32"]
        assert rel_l2(vel[pick], ref["samples"]["vel"].reshape(3, -1)) < TOL["fp32"]


# ----------------------------------------------------------------- engine behaviour

@pytest.mark.parametrize("layout", ["aa", "ab"])
def test_graph_replay_equals_eager(monkeypatch, layout):
    spec = W.scaled(TGV_4D_SMALL, steps=150, layout=layout)
    say("case graph vs eager", layout)
    monkeypatch.setenv("UQ_GRAPH_STEPS", "32")
    with Job(spec) as a:
        a.run(3)
        a.run(147)
        fa = a.populations(5)
        ka = a.qoi_samples("ke")
    monkeypatch.setenv("UQ_GRAPH_STEPS", "0")
    with Job(spec) as b:
        b.run(150)
        fb = b.populations(5)
        kb = b.qoi_samples("ke")
    assert np.array_equal(fa, fb) and np.array_equal(ka, kb)


@pytest.mark.parametrize("bx", [128, 256])
@pytest.mark.parametrize("layout", ["aa", "ab"])
def test_workgroup_shapes_match_oracle(bx, layout, monkeypatch):
    # 128 x 2 and 256 x 1 workgroups (the tuner's other shapes), ragged edges
    monkeypatch.setenv("UQ_BX", str(bx))
    say("case workgroup", bx, layout)
    for spec, steps in ((TGV_RAGGED, 7), (CHANNEL_SMALL, 201)):
        with Job(W.scaled(spec, layout=layout)) as job:
            assert job.info().bx == bx
            job.run(steps)
            xi, a = job.samples()
            p = O.sample_params(spec, xi[-1])
            if spec["geometry"] == "tgv":
                ref = O.tgv_run(72, 40, p["nu"], p["u0"], steps, p["phase_x"], p["phase_y"], want_f=True)["f"]
            else:
                ref = O.channel_run(100, 41, p["nu"], p["u_peak"], steps, D=10, cx=25, cy=18, ramp=200,
                                    want_f=True)["f"]
            assert np.abs(job.populations(job.S - 1) - ref).max() < 1e-13


def test_layouts_agree_fp64():
    # AA and AB perform the same per-node arithmetic (up to the compiler's
    # fused multiply-adds): results agree to rounding
    spec = W.scaled(CHANNEL_SMALL, steps=77)
    say("case layouts agree")
    with Job(W.scaled(spec, layout="aa")) as a, Job(W.scaled(spec, layout="ab")) as b:
        assert a.info().layout == 1 and b.info().layout == 2
        a.run(77)
        b.run(77)
        for s_ in range(4):
            d = float(np.abs(a.populations(s_) - b.populations(s_)).max())
            assert d < 1e-14, d
        assert rel_l2(a.qoi_samples("cd"), b.qoi_samples("cd")) < 1e-12


def test_unstable_sample_is_reported():
    spec = dict(name="tgv_unstable", geometry="tgv", precision="fp32", nx=32, ny=32, steps=400, u0=0.9,
                nu=1e-5, dists=[("u0", 0.8, 0.9)], rule=dict(kind="gl", n=2, order=1))
    say("case unstable")
    with Job(spec) as job:
        job.run(400)
        with pytest.raises(UQError) as e:
            job.moments("ke")
        assert e.value.status == A.UQ_EUNSTABLE


def test_nonpositive_viscosity_rejected():
    spec = W.scaled(TGV_RAGGED, dists=[("nu", -0.01, 0.01)])
    with pytest.raises(UQError) as e:
        Job(spec)
    assert e.value.status == A.UQ_EINVAL


def test_autotune_picks_a_candidate_and_jobs_use_it():
    spec = W.scaled(TGV_4D_SMALL, steps=20)
    say("case autotune")
    r = A.autotune(spec, steps=10)
    # nx = 96: 64- and 128-wide workgroups (256 would leave half the lanes
    # idle), plus 12 fused tile candidates (2, 3, 4 steps x 2 pads x 2 tile
    # heights), 6 sliding-window ones (2, 3, 4 steps x 2 chunk heights) and 12
    # full-row ones (3 to 8 steps x 2 chunk heights)
    assert r["n_candidates"] == 54 and r["layout"] in ("aa", "ab") and r["gbs"] > 0
    with Job(spec) as job:
        inf = job.info()
        assert ({1: "aa", 2: "ab"}[inf.layout], inf.cpt, inf.plane_pad, inf.bx, inf.fused, inf.fused_rows,
                inf.fused_window) == \
            (r["layout"], r["cpt"], r["plane_pad"], r["bx"], r["fused"], r["fused_rows"], r["fused_window"])
        job.run(20)
        ref = O.run_problem(spec, qois=["ke"])
        assert rel_l2(job.qoi_samples("ke")[:, 0], ref["samples"]["ke"]) < TOL["fp32"]


def test_tune_cache_file_carries_the_shape_to_another_process(tmp_path, monkeypatch):
    # uq_autotune appends its choice to the file named by UQ_TUNE_CACHE; a
    # fresh process reads it back and gives the same problem class that shape
    import json
    import subprocess
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("UQ_TUNE_CACHE", str(cache))
    spec = W.scaled(TGV_4D_SMALL, name="tgv96x80_cache", ny=72, steps=20)
    say("case tune cache")
    r = A.autotune(spec, steps=10)
    fields = cache.read_text().split()
    assert len(fields) == 15
    want = {"layout": {1: "aa", 2: "ab"}[int(fields[6])], "cpt": int(fields[7]), "plane_pad": int(fields[9]),
            "bx": int(fields[10]), "fused": int(fields[11]) if int(fields[11]) >= 2 else 0,
            "fused_window": int(fields[13]) if int(fields[11]) >= 2 else 0}
    assert want == {k: r[k] for k in want}
    code = ("import json, sys; from paper_2508_13867_amd import Job; spec = json.loads(sys.argv[1]); "
            "j = Job(spec); i = j.info(); "
            "print(json.dumps(dict(layout={1: 'aa', 2: 'ab'}[i.layout], cpt=i.cpt, plane_pad=i.plane_pad, bx=i.bx, "
            "fused=i.fused, fused_window=i.fused_window))); j.close()")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, UQ_TUNE_CACHE=str(cache), PYTHONPATH=root)
    for k in ("UQ_FUSE", "UQ_FUSE_TY", "UQ_FUSE_WINDOW", "UQ_LAYOUT"):
        env.pop(k, None)
    out = subprocess.run([sys.executable, "-c", code, json.dumps(spec)], env=env, capture_output=True, text=True,
                         timeout=120, cwd=root)
    assert out.returncode == 0, out.stderr[-2000:]
    assert json.loads(out.stdout.strip().splitlines()[-1]) == want


def test_mc4096_full_size_precisions_vs_fp64_and_oracle():
    # the 128^2 x 4096-sample Monte Carlo workload at full size and length:
    # FP64 re-checked on sampled samples by the oracle, FP32 and FP16-storage
    # statistics against FP64 at their bars
    base = W.TGV_MC
    say("case", base["name"], "full")
    ke, st = {}, {}
    for prec in ("fp64", "fp32", "fp16s"):
        with Job(W.scaled(base, precision=prec)) as job:
            job.run(base["steps"])
            ke[prec] = job.qoi_samples("ke")[:, 0]
            st[prec] = job.moments("ke")
    pick = [5, 2222]
    ref = O.run_problem(base, samples=pick, qois=["ke"])
    assert rel_l2(ke["fp64"][pick], ref["samples"]["ke"]) < TOL["fp64"]
    for prec in ("fp32", "fp16s"):
        for k in ("mean", "var"):
            assert rel_l2(st[prec][k], st["fp64"][k]) < TOL[prec], (prec, k, rel_l2(st[prec][k], st["fp64"][k]))
        assert rel_l2(ke[prec], ke["fp64"]) < TOL[prec]


@pytest.mark.parametrize("fuse", ["0", "8"])
def test_fp32_kinetic_energy_does_not_drift(fuse, monkeypatch):
    # The single-precision collision forms its first-order term with axis and
    # diagonal coefficients whose momentum sum is omega exactly. With a
    # rounded omega/3 on both it would scale the momentum by the same
    # 1 + O(1e-8) every step, and the kinetic energy of a decaying vortex
    # would drift by ~1e-4 (a float32 model of that arithmetic: 7e-4 over 3000
    # steps). Per-sample KE of FP32 runs, single steps and 8 fused steps per
    # launch, against the device's FP64 run of the same inputs.
    spec = dict(name="tgv64_drift", geometry="tgv", precision="fp64", nx=64, ny=64, steps=3000, u0=0.02, nu=0.005,
                dists=[("nu", 0.004, 0.006), ("u0", 0.018, 0.022)], rule=dict(kind="gl", n=2, order=1), layout="ab")
    say("case fp32 drift, fuse", fuse)
    ke = {}
    for prec in ("fp64", "fp32"):
        if prec == "fp32" and fuse != "0":
            monkeypatch.setenv("UQ_FUSE", fuse)
            monkeypatch.setenv("UQ_FUSE_TY", "64")
            monkeypatch.setenv("UQ_FUSE_WINDOW", "2")
        with Job(dict(spec, precision=prec)) as job:
            if prec == "fp32":
                assert job.info().fused == int(fuse)
            job.run(spec["steps"])
            ke[prec] = job.qoi_samples("ke")[:, 0]
    err = np.abs(ke["fp32"] / ke["fp64"] - 1.0)
    say("largest relative KE error", err.max())
    assert err.max() < 2e-6, err


@pytest.mark.parametrize("rule", [dict(kind="smolyak", level=2, order=2), dict(kind="halton", N=40),
                                  dict(kind="lhs", N=40, seed=77)])
def test_sparse_grid_qmc_lhs_rules_fp64(rule):
    spec = dict(name="tgv48x40_rules", geometry="tgv", precision="fp64", nx=48, ny=40, steps=61, u0=0.02,
                nu=0.005, dists=W.FOUR_D_INPUTS, rule=rule)
    say("case rule", rule)
    ref = O.run_problem(spec, qois=["ke", "vel"])
    with Job(spec) as job:
        xi, a = job.samples()
        assert np.abs(xi - ref["xi"]).max() < 1e-15 and np.abs(a - ref["a"]).max() < 1e-13
        job.run(spec["steps"])
        for q in ("ke", "vel"):
            st = job.moments(q)
            for k in ("mean", "var", "var_alt") + (("coeffs",) if rule["kind"] == "smolyak" else ()):
                assert rel_l2(st[k], ref["stats"][q][k]) < TOL["fp64"], (q, k)
            assert_stats(st, ref["stats"][q], TOL["fp64"], q)


# ----------------------------------------------------------------- fused steps per launch

@pytest.mark.parametrize("n", [2, 3, 4])
@pytest.mark.parametrize("rows, window", [(4, 0), (8, 0), (8, 1), (16, 1), (8, 2), (16, 2)])
@pytest.mark.parametrize("steps", [4, 7, 41, 130])
def test_fused_kernel_populations_match_oracle(steps, rows, window, n, monkeypatch):
    # FP64 (tile heights 4 and 8; window and full-row chunks of 8 and 16
    # rows) on the ragged 72 x 40 vortex: counts that leave single steps
    # after the fused blocks, and a captured graph
    monkeypatch.setenv("UQ_FUSE", str(n))
    monkeypatch.setenv("UQ_FUSE_TY", str(rows))
    monkeypatch.setenv("UQ_FUSE_WINDOW", str(window))
    spec = W.scaled(TGV_RAGGED, layout="ab")
    say("case fused", n, "fp64 steps", steps, "rows", rows, "window", window)
    with Job(spec) as job:
        assert job.info().fused == n and job.info().fused_rows == rows and job.info().fused_window == window
        job.run(steps)
        xi, a = job.samples()
        for smp in (0, 8):
            p = O.sample_params(TGV_RAGGED, xi[smp])
            ref = O.tgv_run(72, 40, p["nu"], p["u0"], steps, p["phase_x"], p["phase_y"], want_f=True)["f"]
            got = job.populations(smp)
            assert np.abs(got - ref).max() < 1e-13, (smp, np.abs(got - ref).max())


@pytest.mark.parametrize("n", [2, 3, 4])
@pytest.mark.parametrize("window", [0, 1, 2])
@pytest.mark.parametrize("nx, ny", [(20, 12), (3, 5), (2, 4), (130, 17), (58, 9), (59, 9), (192, 6)])
def test_fused_kernel_small_and_wrapping_lattices(nx, ny, window, n, monkeypatch):
    # lattices narrower than a tile and its ring (the ring wraps onto itself);
    # 58 and 59 columns: one window strip at N = 4, then two; two columns
    # and 192 (three waves per row, the widest FP64 full-row lattice at N = 4)
    monkeypatch.setenv("UQ_FUSE", str(n))
    monkeypatch.setenv("UQ_FUSE_WINDOW", str(window))
    spec = W.scaled(TGV_RAGGED, nx=nx, ny=ny, layout="ab", precision="fp64", phase_x=0.0, phase_y=0.0)
    say("case fused", n, "lattice", nx, ny, "window", window)
    with Job(spec) as job:
        assert job.info().fused == n and job.info().fused_window == window
        job.run(24)
        xi, _ = job.samples()
        p = O.sample_params(spec, xi[3])
        ref = O.tgv_run(nx, ny, p["nu"], p["u0"], 24, want_f=True)["f"]
        assert np.abs(job.populations(3) - ref).max() < 1e-13


@pytest.mark.parametrize("n", [5, 6])
@pytest.mark.parametrize("nx, ny, rows", [(72, 40, 16), (72, 40, 256), (20, 12, 8), (3, 5, 8), (2, 4, 8),
                                          (128, 9, 64)])
def test_full_row_kernel_five_and_six_steps(nx, ny, rows, n, monkeypatch):
    # 5 and 6 steps per launch exist only over whole rows (two columns per
    # lane where one would need more than 16 waves); FP64 against the oracle
    # over counts that leave single steps after the fused blocks
    monkeypatch.setenv("UQ_FUSE", str(n))
    monkeypatch.setenv("UQ_FUSE_TY", str(rows))
    monkeypatch.setenv("UQ_FUSE_WINDOW", "2")
    spec = W.scaled(TGV_RAGGED, nx=nx, ny=ny, layout="ab", precision="fp64")
    say("case full rows", n, "lattice", nx, ny, "rows", rows)
    for steps in (n + 1, 4 * n + 3):
        with Job(spec) as job:
            assert job.info().fused == n and job.info().fused_window == 2
            job.run(steps)
            xi, _ = job.samples()
            p = O.sample_params(spec, xi[5])
            ref = O.tgv_run(nx, ny, p["nu"], p["u0"], steps, p["phase_x"], p["phase_y"], want_f=True)["f"]
            assert np.abs(job.populations(5) - ref).max() < 1e-13, steps


@pytest.mark.parametrize("n", [5, 6])
@pytest.mark.parametrize("prec", ["fp32", "bf16s"])
def test_full_row_kernel_five_and_six_steps_full_size(prec, n, monkeypatch):
    # the 256^2 x 256 lattice (two waves of two columns per lane per step),
    # against single steps
    spec = W.scaled(W.TGV_BATCHED_FP32, precision=prec, layout="ab", steps=60)
    say("case full rows", n, "256^2 x 256", prec)
    res = {}
    for fuse in ("0", str(n)):
        monkeypatch.setenv("UQ_FUSE", fuse)
        monkeypatch.setenv("UQ_FUSE_TY", "256")
        monkeypatch.setenv("UQ_FUSE_WINDOW", "2")
        with Job(spec) as job:
            assert job.info().fused == (n if fuse != "0" else 0)
            job.run(60)
            res[fuse] = (job.populations(200), job.qoi_samples("ke")[:, 0])
    assert np.array_equal(res["0"][0], res[str(n)][0])
    assert np.array_equal(res["0"][1], res[str(n)][1])


@pytest.mark.parametrize("n", [2, 3, 4])
@pytest.mark.parametrize("window", [0, 1, 2])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16s", "bf16s"])
def test_fused_kernel_matches_single_steps(prec, window, n, monkeypatch):
    spec = W.scaled(TGV_4D_SMALL, precision=prec, layout="ab", steps=200)
    monkeypatch.setenv("UQ_FUSE_WINDOW", str(window))
    say("case fused", n, "vs single", prec, "window", window)
    res = {}
    for fuse in ("0", str(n)):
        monkeypatch.setenv("UQ_FUSE", fuse)
        with Job(spec) as job:
            job.run(200)
            res[fuse] = (job.populations(7), job.qoi_samples("ke")[:, 0])
    # the same per-node operations in the same order and the same storage
    # rounding: bit for bit the same populations and kinetic energy
    assert np.array_equal(res["0"][0], res[str(n)][0])
    assert np.array_equal(res["0"][1], res[str(n)][1])


@pytest.mark.parametrize("n", [7, 8])
@pytest.mark.parametrize("nx, ny, rows", [(72, 40, 16), (128, 9, 64), (20, 12, 8), (3, 5, 8), (128, 128, 256),
                                           (200, 13, 8), (256, 24, 16)])
@pytest.mark.parametrize("prec", ["fp32", "fp16s", "bf16s"])
def test_full_row_kernel_seven_and_eight_steps(prec, nx, ny, rows, n, monkeypatch):
    # 7 and 8 steps per launch: whole rows of up to 128 columns at one
    # column per lane and of 129..256 columns at two (14 or 16 waves; 200
    # leaves lanes past the lattice), single precision and 16-bit storage;
    # bit for bit the single-step result, over counts that leave single
    # steps after the fused blocks
    monkeypatch.setenv("UQ_FUSE_TY", str(rows))
    monkeypatch.setenv("UQ_FUSE_WINDOW", "2")
    spec = W.scaled(TGV_RAGGED, nx=nx, ny=ny, layout="ab", precision=prec)
    say("case full rows", n, prec, "lattice", nx, ny, "rows", rows)
    for steps in (n + 1, 3 * n + 5):
        res = {}
        for fuse in ("0", str(n)):
            monkeypatch.setenv("UQ_FUSE", fuse)
            with Job(spec) as job:
                assert job.info().fused == (n if fuse != "0" else 0)
                job.run(steps)
                res[fuse] = job.populations(5)
        assert np.array_equal(res["0"], res[str(n)]), steps
    if prec == "fp32":
        with Job(spec) as job:
            xi, _ = job.samples()
        p = O.sample_params(spec, xi[5])
        ref = O.tgv_run(nx, ny, p["nu"], p["u0"], steps, p["phase_x"], p["phase_y"], want_f=True)["f"]
        assert np.abs(res[str(n)] - ref).max() < 1e-6


@pytest.mark.parametrize("nx, ny", [(384, 12), (512, 9), (450, 20)])
@pytest.mark.parametrize("prec", ["fp32", "bf16s"])
def test_full_row_kernel_wide_rows(prec, nx, ny, monkeypatch):
    # rows of 384..512 columns: three or four waves of two columns per lane
    # per level, 4 steps per launch (16 waves); 450 leaves lanes past the
    # lattice. Bit for bit the single-step result; FP32 also against the
    # oracle on one sample
    monkeypatch.setenv("UQ_FUSE_TY", "8")
    monkeypatch.setenv("UQ_FUSE_WINDOW", "2")
    spec = W.scaled(TGV_RAGGED, nx=nx, ny=ny, layout="ab", precision=prec)
    say("case wide rows", prec, nx, ny)
    steps = 4 * 3 + 3
    res = {}
    for fuse in ("0", "4"):
        monkeypatch.setenv("UQ_FUSE", fuse)
        with Job(spec) as job:
            assert job.info().fused == (4 if fuse == "4" else 0)
            assert fuse == "0" or job.info().fused_window == 2
            job.run(steps)
            res[fuse] = job.populations(3)
    assert np.array_equal(res["0"], res["4"])
    if prec == "fp32":
        with Job(spec) as job:
            xi, _ = job.samples()
        p = O.sample_params(spec, xi[3])
        ref = O.tgv_run(nx, ny, p["nu"], p["u0"], steps, p["phase_x"], p["phase_y"], want_f=True)["f"]
        assert np.abs(res["4"] - ref).max() < 1e-6


@pytest.mark.parametrize("nx, ny, n", [(640, 9, 3), (600, 11, 3), (768, 7, 2), (700, 5, 2)])
@pytest.mark.parametrize("prec", ["fp32", "bf16s"])
def test_full_row_kernel_widest_rows(prec, nx, ny, n, monkeypatch):
    # rows of 600..768 columns: five or six waves of two columns per lane per
    # level, 3 or 2 steps per launch; 600 and 700 leave lanes past the
    # lattice. Bit for bit the single-step result; FP32 also against the
    # oracle on one sample
    monkeypatch.setenv("UQ_FUSE_TY", "8")
    monkeypatch.setenv("UQ_FUSE_WINDOW", "2")
    spec = W.scaled(TGV_RAGGED, nx=nx, ny=ny, layout="ab", precision=prec)
    say("case widest rows", prec, nx, ny, n)
    steps = 2 * n * 2 + 1
    res = {}
    for fuse in ("0", str(n)):
        monkeypatch.setenv("UQ_FUSE", fuse)
        with Job(spec) as job:
            assert job.info().fused == (n if fuse != "0" else 0)
            assert fuse == "0" or job.info().fused_window == 2
            job.run(steps)
            res[fuse] = job.populations(2)
    assert np.array_equal(res["0"], res[str(n)])
    if prec == "fp32":
        with Job(spec) as job:
            xi, _ = job.samples()
        p = O.sample_params(spec, xi[2])
        ref = O.tgv_run(nx, ny, p["nu"], p["u0"], steps, p["phase_x"], p["phase_y"], want_f=True)["f"]
        assert np.abs(res[str(n)] - ref).max() < 1e-6


@pytest.mark.parametrize("prec", ["fp32", "fp16s", "bf16s"])
def test_fused_channel_widest_rows(prec, monkeypatch):
    # a 616-column channel (five waves of two columns per level, 2 steps per
    # launch) with walls, cylinder and Zou-He ends: bit for bit the single
    # steps (populations and drag); FP32 single steps against the oracle
    spec = W.scaled(CHANNEL_SMALL, nx=616, ny=23, D=8, cx=60, cy=11, precision=prec, layout="ab", ramp=10,
                    steps=25)
    say("case fused channel widest rows", prec)
    res = {}
    for fuse in ("0", "2"):
        monkeypatch.setenv("UQ_FUSE", fuse)
        monkeypatch.setenv("UQ_FUSE_TY", "8")
        monkeypatch.setenv("UQ_FUSE_WINDOW", "2")
        with Job(spec) as job:
            assert job.info().fused == (2 if fuse == "2" else 0)
            job.run(25)
            res[fuse] = (job.populations(1), job.qoi_samples("cd")[:, 0])
            if prec == "fp32" and fuse == "0":
                xi, _ = job.samples()
    assert np.array_equal(res["0"][0], res["2"][0])
    assert np.array_equal(res["0"][1], res["2"][1])
    if prec == "fp32":
        p = O.sample_params(spec, xi[1])
        ref = O.channel_run(616, 23, p["nu"], p["u_peak"], 25, D=8, cx=60, cy=11, ramp=10, want_f=True)["f"]
        assert np.abs(res["2"][0] - ref).max() < 1e-5


@pytest.mark.parametrize("steps, launches", [(3, 1), (5, 1), (7, 3), (8, 2), (13, 3), (20, 4), (25, 5)])
def test_steps_left_over_run_as_odd_fused_launches(steps, launches, monkeypatch):
    # 6 steps per launch in pairs (12); what is left goes in odd fused
    # launches of 5 or 3 steps, then single steps (7 = 5 + 1 + 1,
    # 8 = 5 + 3, 13 = 12 + 1, 20 = 12 + 5 + 3, 25 = 24 + 1): bit for bit the
    # single-step result, and the launch count says which kernels ran
    monkeypatch.setenv("UQ_FUSE_TY", "16")
    monkeypatch.setenv("UQ_FUSE_WINDOW", "2")
    monkeypatch.setenv("UQ_GRAPH_STEPS", "0")
    spec = W.scaled(TGV_RAGGED, layout="ab", precision="fp32")
    say("case leftover steps", steps)
    res = {}
    for fuse in ("0", "6"):
        monkeypatch.setenv("UQ_FUSE", fuse)
        with Job(spec) as job:
            job.run(steps)
            res[fuse] = (job.populations(4), job.info().step_launches)
    assert np.array_equal(res["0"][0], res["6"][0])
    assert res["0"][1] == steps and res["6"][1] == launches


def test_full_row_kernel_eight_steps_refused_where_rows_are_too_wide(monkeypatch):
    # 320 columns need three waves of two columns per lane per level: 24
    # waves for 8 levels, more than a workgroup holds, so 8 steps over whole
    # rows fall back to single steps (256 columns fit: 16 waves)
    monkeypatch.setenv("UQ_FUSE", "8")
    monkeypatch.setenv("UQ_FUSE_WINDOW", "2")
    spec = W.scaled(TGV_RAGGED, nx=320, ny=16, layout="ab", precision="fp32")
    with Job(spec) as job:
        assert job.info().fused == 0
    with Job(W.scaled(spec, nx=256)) as job:
        assert job.info().fused == 8


@pytest.mark.parametrize("n, window, rows, nt", [(2, 0, 8, 1), (3, 0, 8, 1), (4, 1, 64, 0), (4, 2, 256, 0),
                                                 (3, 2, 256, 0), (5, 2, 256, 0), (6, 2, 256, 0), (7, 2, 256, 0),
                                                 (8, 2, 256, 0)])
def test_fused_kernel_full_size_sampled(n, window, rows, nt, monkeypatch):
    # the 256^2 x 256 benchmark lattice, fused, 120 steps, two samples
    # re-solved by the oracle
    monkeypatch.setenv("UQ_FUSE", str(n))
    monkeypatch.setenv("UQ_FUSE_WINDOW", str(window))
    monkeypatch.setenv("UQ_FUSE_TY", str(rows))
    monkeypatch.setenv("UQ_NT_STORE", str(nt))
    spec = W.scaled(W.TGV_BATCHED_FP32, steps=120, layout="ab")
    say("case fused", n, "window", window, "rows", rows, "256^2 x 256")
    with Job(spec) as job:
        assert job.info().fused == n and job.info().fused_window == window
        job.run(spec["steps"])
        ke = job.qoi_samples("ke")[:, 0]
        pick = [0, 200]
        ref = O.run_problem(spec, samples=pick, qois=["ke", "vel"])
        assert rel_l2(ke[pick], ref["samples"]["ke"]) < TOL["fp32"]
        vel = job.qoi_samples("vel")
        assert rel_l2(vel[pick], ref["samples"]["vel"].reshape(2, -1)) < TOL["fp32"]


def test_benchmark_workload_in_its_tuned_launch_shape(tmp_path, monkeypatch):
    # the benchmark's own path: tune the 256^2 x 256 FP32 job as bench.py
    # does, then run it in the chosen shape (graph replay included) and
    # re-solve sampled samples with the oracle
    monkeypatch.setenv("UQ_TUNE_CACHE", str(tmp_path / "tune.txt"))
    for k in ("UQ_FUSE", "UQ_FUSE_TY", "UQ_FUSE_WINDOW", "UQ_NT_STORE", "UQ_LAYOUT"):
        monkeypatch.delenv(k, raising=False)
    spec = W.scaled(W.TGV_BATCHED_FP32, steps=250)
    say("case benchmark shape: tuning")
    r = A.autotune(spec, steps=120)
    say("tuned", r)
    with Job(spec) as job:
        inf = job.info()
        assert (inf.fused, inf.fused_window, inf.fused_rows) == (r["fused"], r["fused_window"], r["fused_rows"])
        job.run(spec["steps"])
        ke = job.qoi_samples("ke")[:, 0]
        vel = job.qoi_samples("vel")
        pick = [3, 129, 255]
        ref = O.run_problem(spec, samples=pick, qois=["ke", "vel"])
        assert rel_l2(ke[pick], ref["samples"]["ke"]) < TOL["fp32"]
        assert rel_l2(vel[pick], ref["samples"]["vel"].reshape(3, -1)) < TOL["fp32"]
        st = job.moments("ke")
        assert abs(st["mean"][0] - float(np.dot(job.samples()[1], ke))) <= 1e-12 * abs(st["mean"][0])


def test_benchmark_workload_full_length(monkeypatch):
    # tgv256_fp32_gl4x4 over its full 5000 steps. FP32 in the launch shape
    # the benchmark times (6 fused steps per launch over whole rows, chunks
    # of 256 rows, AB) against the same job in FP64 on the device; three
    # samples of the FP64 run re-solved by the oracle (in threads while the
    # device works) pin that reference at the FP64 bar. Statistics of KE and
    # of the velocity field: mean, variance and all 35 gPC coefficients, the
    # k >= 1 terms on their own norm, at the FP32 bar.
    from concurrent.futures import ThreadPoolExecutor

    for k, v in (("UQ_FUSE", "6"), ("UQ_FUSE_WINDOW", "2"), ("UQ_FUSE_TY", "256"), ("UQ_NT_STORE", "0"),
                 ("UQ_PLANE_PAD", "64")):
        monkeypatch.setenv(k, v)
    base = W.TGV_BATCHED_FP32
    pick = [0, 77, 255]
    say("case benchmark workload, 5000 steps: oracle on samples", pick)
    with ThreadPoolExecutor(len(pick)) as ex:
        futs = [ex.submit(O.run_problem, base, [j], ["ke", "vel"]) for j in pick]
        res = {}
        with Job(W.scaled(base, layout="ab")) as job:
            inf = job.info()
            assert (inf.fused, inf.fused_window, inf.fused_rows) == (6, 2, 256)
            job.run(base["steps"])
            res["fp32"] = (job.qoi_samples("ke")[:, 0], job.qoi_samples("vel"), job.moments("ke"),
                           job.moments("vel"))
            assert job.info().steps_done == 5000
        monkeypatch.setenv("UQ_FUSE", "0")
        with Job(W.scaled(base, precision="fp64")) as job:
            job.run(base["steps"])
            res["fp64"] = (job.qoi_samples("ke")[:, 0], job.qoi_samples("vel"), job.moments("ke"),
                           job.moments("vel"))
        refs = [f.result() for f in futs]
    ke64, vel64, st64, sv64 = res["fp64"]
    for j, r in zip(pick, refs):
        assert rel_l2(ke64[j], r["samples"]["ke"]) < TOL["fp64"], j
        assert rel_l2(vel64[j], r["samples"]["vel"].ravel()) < TOL["fp64"], j
    ke32, vel32, st32, sv32 = res["fp32"]
    assert rel_l2(ke32, ke64) < TOL["fp32"] and rel_l2(vel32, vel64) < TOL["fp32"]
    assert_stats(st32, st64, TOL["fp32"], "ke")
    # the mean velocity under uniform phases is near zero (a few 1e-6 of the
    # amplitude from the 4-node phase rule): over the per-sample field RMS
    rms = np.sqrt(np.mean(vel64 ** 2)) * np.sqrt(vel64.shape[1])
    assert_stats(sv32, sv64, TOL["fp32"], "vel", mean_scale=rms)
    errs = {"ke": stat_errors(st32, st64), "vel": stat_errors(sv32, sv64, mean_scale=rms)}
    say("fp32 vs fp64 after 5000 steps:", errs)


def test_fused_graph_replay_equals_eager(monkeypatch):
    monkeypatch.setenv("UQ_FUSE", "3")
    spec = W.scaled(TGV_4D_SMALL, steps=150, layout="ab")
    say("case fused graph vs eager")
    monkeypatch.setenv("UQ_GRAPH_STEPS", "24")
    with Job(spec) as a:
        a.run(5)
        a.run(145)
        fa = a.populations(5)
    monkeypatch.setenv("UQ_GRAPH_STEPS", "0")
    with Job(spec) as b:
        b.run(150)
        fb = b.populations(5)
    assert np.array_equal(fa, fb)


@pytest.mark.parametrize("nx, ny, steps, fused", [(4096, 4096, 9, True), (8192, 7300, 3, False)])
def test_fused_kernels_at_the_buffer_range_limit(nx, ny, steps, fused, monkeypatch):
    # one FP32 sample: 4096^2 (604 MB per slab) runs the window kernel;
    # 8192 x 7300 (2.15 GB per slab, beyond the 2^31-byte range of a buffer
    # descriptor) falls back to single steps; both against the oracle
    monkeypatch.setenv("UQ_FUSE", "4")
    monkeypatch.setenv("UQ_FUSE_TY", "64")
    monkeypatch.setenv("UQ_FUSE_WINDOW", "1")
    spec = dict(name=f"tgv{nx}x{ny}_single", geometry="tgv", precision="fp32", nx=nx, ny=ny, steps=steps, u0=0.03,
                nu=0.02, dists=[("nu", 0.015, 0.025)], rule=dict(kind="gl", n=1, order=0), layout="ab")
    say("case buffer range", nx, ny)
    with Job(spec) as job:
        assert (job.info().fused == 4) == fused
        job.run(spec["steps"])
        ke = job.qoi_samples("ke")[:, 0]
        ref = O.run_problem(spec, qois=["ke"])
        assert rel_l2(ke, ref["samples"]["ke"]) < TOL["fp32"]


@pytest.mark.parametrize("layout, fuse", [("aa", "0"), ("ab", "0"), ("ab", "4")])
def test_more_samples_than_a_grid_dimension(layout, fuse, monkeypatch):
    # 70,000 samples (> 65,535, the largest grid y extent) on an 8 x 8 lattice:
    # every per-sample loop must reach the last samples
    monkeypatch.setenv("UQ_FUSE", fuse)
    spec = dict(name="tgv8_mc70000", geometry="tgv", precision="fp32", nx=8, ny=8, steps=12, u0=0.02, nu=0.02,
                dists=[("nu", 0.01, 0.03), ("u0", 0.015, 0.025)], rule=dict(kind="mc", N=70000, seed=5),
                layout=layout)
    say("case S = 70000", layout, fuse)
    with Job(spec) as job:
        job.run(spec["steps"])
        ke = job.qoi_samples("ke")[:, 0]
        vel = job.qoi_samples("vel")
        pick = [0, 65535, 65536, 69999]
        ref = O.run_problem(spec, samples=pick, qois=["ke", "vel"])
        assert rel_l2(ke[pick], ref["samples"]["ke"]) < TOL["fp32"]
        assert rel_l2(vel[pick], ref["samples"]["vel"].reshape(4, -1)) < TOL["fp32"]
        st = job.moments("ke")
        assert abs(st["mean"][0] - ke.mean()) <= 1e-12 * abs(ke.mean())
