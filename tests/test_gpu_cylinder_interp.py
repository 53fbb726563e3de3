"""GPU parity of the paper's cylinder variant: interpolated (Bouzidi) bounce-
back on the exact circle and the finite-difference (interpolated) inlet and
outlet, in the AB layout, against the FP64 oracle on the same seeded
samples; plus the full-size 22D x 4D channel on sampled samples, graph
replay, and the rejections (AA layout, circle too close to a boundary,
the server)."""
import sys

import numpy as np
import pytest

import oracle as O
from helpers import assert_stats, assert_stats_given_samples, gpu_available, rel_l2
from paper_2508_13867_amd import Job, Server, UQError
from paper_2508_13867_amd import _abi as A
from paper_2508_13867_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = {"fp64": 1e-10, "fp32": 1e-4}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# an off-centre circle (both interpolation branches, no symmetry), ragged
# against the 64-wide tiles
SMALL = dict(name="chan70x27_interp", geometry="channel", precision="fp64", nx=70, ny=27, steps=301,
             u_peak=0.06, nu=0.04, cyl_bc="bouzidi", cyl_x=17.3, cyl_y=12.6, cyl_d=8.6, ramp=120, xbc="interp",
             force_ref="mean", layout="ab", dists=[("re", 16.0, 24.0), ("u_peak", 0.054, 0.066)],
             rule=dict(kind="gl", n=2, order=1))

VARIANTS = {
    "bouzidi+fd": {},
    "bouzidi+zouhe": {"xbc": "zouhe"},
    "halfway+fd": {"cyl_bc": "halfway", "D": 8, "cx": 17, "cy": 12},  # off the mid-line: nonzero lift
}


def oracle_f(spec, params, steps):
    xbc = {"zouhe": 0, "interp": 3}[spec["xbc"]]
    fref = 1 if spec.get("force_ref") == "mean" else 0
    if spec.get("cyl_bc") == "bouzidi":
        kw = dict(cyl=1, ccx=spec["cyl_x"], ccy=spec["cyl_y"], R=0.5 * spec["cyl_d"])
    else:
        kw = dict(D=spec["D"], cx=spec["cx"], cy=spec["cy"])
    return O.channel_run_opts(spec["nx"], spec["ny"], params["nu"], params["u_peak"], steps, xbc=xbc,
                              ramp=spec["ramp"], force_ref=fref, want_f=True, **kw)


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("steps", [1, 2, 7, 130])
def test_populations_match_oracle(variant, steps):
    spec = W.scaled(SMALL, **VARIANTS[variant])
    say("case", spec["name"], variant, "steps", steps)
    with Job(spec) as job:
        job.run(steps)
        xi, _ = job.samples()
        for s in (0, 3):
            p = O.sample_params(spec, xi[s])
            ref = oracle_f(spec, p, steps)["f"]
            got = job.populations(s)
            assert np.abs(got - ref).max() < 1e-13, (s, np.abs(got - ref).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", list(VARIANTS))
def test_drag_lift_moments_match_oracle(variant, prec):
    spec = W.scaled(SMALL, precision=prec, **VARIANTS[variant])
    say("case", spec["name"], variant, prec, "moments")
    ref = O.run_problem(spec, qois=["cd", "cl", "vel"])
    with Job(spec) as job:
        job.run(spec["steps"])
        for q in ("cd", "cl"):
            got = job.qoi_samples(q)[:, 0]
            assert rel_l2(got, ref["samples"][q]) < TOL[prec], (q, rel_l2(got, ref["samples"][q]))
            st = job.moments(q)
            for k in ("mean", "coeffs"):
                assert rel_l2(st[k], ref["stats"][q][k]) < TOL[prec], (q, k)
            if prec == "fp64":
                # mean, var, var_alt and the k >= 1 coefficients (which carry
                # the variance) each on their own norm
                assert_stats(st, ref["stats"][q], TOL[prec], q + " " + prec)
            else:
                # FP32: the reduction of the device's own samples pinned at
                # FP64, and the statistics within what the per-sample
                # errors allow (bounds in the helper)
                r = dict(ref, samples_q=ref["samples"][q], stats_q=ref["stats"][q])
                assert_stats_given_samples(st, got, r, TOL[prec], q + " " + prec)
        vel = job.qoi_samples("vel")
        assert rel_l2(vel, ref["samples"]["vel"].reshape(4, -1)) < TOL[prec]


def test_paper_channel_full_size_sampled():
    # 22D x 4D at D = 20 (440 x 80), 16 Gauss-Legendre samples of the inflow,
    # 1500 steps, FP32 in the benchmarked AB launch; two samples re-solved by
    # the oracle
    spec = W.scaled(W.CYLINDER_PAPER_FP32, steps=1500, rule=dict(kind="gl", n=16, order=15))
    say("case", spec["name"], "1500 steps")
    with Job(spec) as job:
        job.run(spec["steps"])
        cd = job.qoi_samples("cd")[:, 0]
        cl = job.qoi_samples("cl")[:, 0]
        pick = [0, 11]
        ref = O.run_problem(spec, samples=pick, qois=["cd", "cl", "vel"])
        assert rel_l2(cd[pick], ref["samples"]["cd"]) < TOL["fp32"]
        assert np.abs(cl[pick] - ref["samples"]["cl"]).max() < 1e-5
        vel = job.qoi_samples("vel")
        assert rel_l2(vel[pick], ref["samples"]["vel"].reshape(2, -1)) < TOL["fp32"]


def test_graph_replay_equals_eager(monkeypatch):
    spec = W.scaled(SMALL, precision="fp32")
    say("case interp graph vs eager")
    monkeypatch.setenv("UQ_GRAPH_STEPS", "32")
    with Job(spec) as a:
        a.run(5)
        a.run(140)
        fa = a.populations(2)
        ca = a.qoi_samples("cd")
    monkeypatch.setenv("UQ_GRAPH_STEPS", "0")
    with Job(spec) as b:
        b.run(145)
        fb = b.populations(2)
        cb = b.qoi_samples("cd")
    assert np.array_equal(fa, fb) and np.array_equal(ca, cb)


def test_rejections():
    say("case interp rejections")
    for bad in (dict(layout="aa"),                       # interpolated rules need AB
                dict(cyl_y=4.0),                         # circle touches the wall band
                dict(cyl_x=5.0),                         # too close to the inlet column
                dict(xbc="interp", nx=3)):               # no room for the difference stencil
        with pytest.raises(UQError) as e:
            Job(W.scaled(SMALL, **bad)).close()
        assert e.value.status == A.UQ_EINVAL, bad
    with Server(memory_budget_gb=1, max_jobs=2, steps_per_tick=16, precision="fp64") as srv:
        with pytest.raises(UQError) as e:
            srv.submit(SMALL, qoi="cd")
        assert e.value.status == A.UQ_EINVAL
