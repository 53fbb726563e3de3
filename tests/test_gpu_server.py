"""GPU tests of the continuous-batching server: served results equal the
standalone job path and the FP64 oracle within the stated tolerances, a job's
result is the same alone and in a mix of concurrently running jobs, the plain
(one sample per launch) mode agrees with the batched one, admission respects
the memory budget, and a failing job does not disturb the others."""
import sys
import time

import numpy as np
import pytest

import oracle as O
from helpers import gpu_available, rel_l2
from paper_2508_13867_amd import Job, Server, UQError
from paper_2508_13867_amd import _abi as A
from paper_2508_13867_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


TGV_A = dict(name="tgv_a", geometry="tgv", precision="fp32", nx=80, ny=72, steps=301, u0=0.02, nu=0.005,
             dists=W.FOUR_D_INPUTS, rule=dict(kind="gl", n=2, order=1))
TGV_B = dict(name="tgv_b", geometry="tgv", precision="fp32", nx=128, ny=128, steps=500, u0=0.02, nu=0.006,
             dists=[("nu", 0.004, 0.008)], rule=dict(kind="mc", N=64, seed=W.SEED + 3))
CYL_C = dict(name="cyl_c", geometry="channel", precision="fp32", nx=220, ny=41, steps=800, u_peak=0.05, nu=0.05,
             D=10, cx=20, cy=20, ramp=300, xbc="zouhe", dists=[("re", 16.0, 24.0), ("u_peak", 0.045, 0.055)],
             rule=dict(kind="gl", n=3, order=2))
TGV_D = dict(name="tgv_d", geometry="tgv", precision="fp32", nx=64, ny=64, steps=150, u0=0.01, nu=0.01,
             dists=[("nu", 0.008, 0.012)], rule=dict(kind="gl", n=5, order=4))


def standalone(spec, qoi):
    with Job(W.scaled(spec, layout="aa")) as j:
        j.run(spec["steps"])
        return j.moments(qoi)


def test_served_results_match_job_path_and_oracle():
    say("case server vs job path")
    with Server(memory_budget_gb=4, max_jobs=8, steps_per_tick=32) as srv:
        ta = srv.submit(TGV_A)
        tc = srv.submit(CYL_C)
        ra = srv.wait(ta, 120)
        rc = srv.wait(tc, 120)
    assert ra["status"] == A.UQ_OK and rc["status"] == A.UQ_OK
    sa = standalone(TGV_A, "ke")
    sc = standalone(CYL_C, "cd")
    # the same per-node arithmetic (fused and single steps agree bit for
    # bit) and the same reduction: bitwise the standalone job's statistics
    for r, s in ((ra, sa), (rc, sc)):
        assert r["mean"] == s["mean"][0] and r["var"] == s["var"][0] and r["var_alt"] == s["var_alt"][0]
        assert np.array_equal(r["coeffs"], s["coeffs"][:, 0])
    ref = O.run_problem(TGV_A, qois=["ke"])["stats"]["ke"]
    assert rel_l2(ra["mean"], ref["mean"]) < 1e-4 and rel_l2(ra["var"], ref["var"]) < 1e-4


def test_result_same_alone_and_in_mix():
    say("case alone vs mix")
    with Server(memory_budget_gb=4, max_jobs=8, steps_per_tick=32) as srv:
        alone = srv.wait(srv.submit(CYL_C), 120)
    with Server(memory_budget_gb=4, max_jobs=8, steps_per_tick=32) as srv:
        t_b = srv.submit(W.scaled(TGV_B, steps=4000))  # long enough to be running when C arrives
        t_d = srv.submit(TGV_D)
        time.sleep(0.01)  # C arrives while B and D are on the GPU
        t_c = srv.submit(CYL_C)
        t_a = srv.submit(TGV_A)
        mix = srv.wait(t_c, 120)
        others = [srv.wait(t, 120) for t in (t_b, t_d, t_a)]
        st = srv.stats()
    assert all(o["status"] == A.UQ_OK for o in others)
    assert mix["status"] == A.UQ_OK
    assert st["completed"] == 4
    # C really shared the GPU: its time on the server overlaps another job's
    assert any(max(mix["t_admit"], o["t_admit"]) < min(mix["t_done"], o["t_done"]) for o in others)
    # same kernels, same per-node arithmetic, fixed per-job reduction order
    assert mix["mean"] == alone["mean"] and mix["var"] == alone["var"]
    assert np.array_equal(mix["coeffs"], alone["coeffs"])


def test_plain_mode_agrees_with_batched():
    say("case plain vs batched")
    res = {}
    for mode in ("batched", "plain"):
        with Server(memory_budget_gb=4, max_jobs=8, steps_per_tick=16, mode=mode) as srv:
            ts = [srv.submit(s) for s in (TGV_D, TGV_A)]
            res[mode] = [srv.wait(t, 180) for t in ts]
    for b, p in zip(res["batched"], res["plain"]):
        assert b["status"] == p["status"] == A.UQ_OK
        assert p["mean"] == b["mean"] and p["var"] == b["var"] and np.array_equal(p["coeffs"], b["coeffs"])


@pytest.mark.parametrize("prec", ["fp32", "fp16s", "bf16s"])
def test_batched_instances_equal_standalone_single_steps(prec):
    # jobs that land in different batched instances (vortex rows of 64, 200,
    # 256 and 384 columns: one or two columns per lane, 8 or 4 steps per
    # launch; a 640-column vortex in strips of 4 steps; channels of 220, 440
    # and 616 columns: 4, 3 or 2 steps, the last with five waves of two
    # columns per level) and one that runs the single-step AA launch (an
    # 880-column channel), with step counts that leave the last steps to
    # each job's own launches: every result is bitwise that of the job
    # alone, one step per launch
    say("case batched instances", prec)
    tgv = dict(geometry="tgv", precision=prec, u0=0.02, nu=0.005, dists=[("nu", 0.004, 0.006), ("u0", 0.018, 0.022)],
               rule=dict(kind="gl", n=2, order=1))
    specs = [dict(tgv, name=f"v{n}", nx=n, ny=n // 2 + 3, steps=steps) for n, steps in
             ((64, 211), (200, 157), (256, 130), (384, 101), (640, 53))]
    specs += [dict(CYL_C, name="c220", precision=prec, steps=233),
              dict(CYL_C, name="c440", precision=prec, nx=440, ny=82, D=20, cx=40, cy=41, steps=149, ramp=60),
              dict(CYL_C, name="c616", precision=prec, nx=616, ny=115, D=28, cx=56, cy=57, nu=0.07, steps=61,
                   ramp=30),
              dict(CYL_C, name="c880", precision=prec, nx=880, ny=164, D=40, cx=80, cy=82, nu=0.1, steps=53,
                   ramp=30)]
    with Server(memory_budget_gb=4, max_jobs=16, steps_per_tick=48, precision=prec) as srv:
        ts = [srv.submit(s) for s in specs]
        rs = [srv.wait(t, 120) for t in ts]
    for spec, r in zip(specs, rs):
        assert r["status"] == A.UQ_OK, spec["name"]
        q = "ke" if spec["geometry"] == "tgv" else "cd"
        s = standalone(spec, q)
        assert r["mean"] == s["mean"][0] and r["var"] == s["var"][0], spec["name"]
        assert np.array_equal(r["coeffs"][:r["K"]], s["coeffs"][:, 0]), spec["name"]


def test_admission_by_memory_budget():
    say("case admission")
    big = W.scaled(TGV_B, rule=dict(kind="mc", N=4096, seed=1))  # 4096 x 128^2 x 36 B = 2.5 GB
    with Server(memory_budget_gb=0.05, max_jobs=4, steps_per_tick=16) as srv:
        with pytest.raises(UQError) as e:
            srv.submit(big)
        assert e.value.status == A.UQ_ENOMEM
        # six jobs of ~19 MB each through a 51 MB arena: at most two resident
        spec = W.scaled(TGV_B, rule=dict(kind="mc", N=32, seed=5), steps=200)
        ts = [srv.submit(spec) for _ in range(6)]
        peak_live = 0
        while True:
            s = srv.stats()
            peak_live = max(peak_live, s["live"])
            if s["completed"] + s["failed"] == 6:
                break
            time.sleep(0.002)
        rs = [srv.wait(t, 60) for t in ts]
        st = srv.stats()
    assert all(r["status"] == A.UQ_OK for r in rs)
    assert peak_live <= 2 and st["arena_peak_bytes"] <= st["arena_bytes"]
    # identical problems give identical results whatever was resident beside them
    assert len({(r["mean"], r["var"]) for r in rs}) == 1


def test_unstable_job_is_isolated():
    say("case failure isolation")
    bad = dict(name="bad", geometry="tgv", precision="fp32", nx=32, ny=32, steps=400, u0=0.9, nu=1e-5,
               dists=[("u0", 0.8, 0.9)], rule=dict(kind="gl", n=2, order=1))
    with Server(memory_budget_gb=2, max_jobs=8, steps_per_tick=32) as srv:
        tb = srv.submit(bad)
        tg = srv.submit(TGV_A)
        rb = srv.wait(tb, 60)
        rg = srv.wait(tg, 60)
    assert rb["status"] == A.UQ_EUNSTABLE
    assert rg["status"] == A.UQ_OK
    assert rel_l2(rg["mean"], standalone(TGV_A, "ke")["mean"]) < 1e-6
