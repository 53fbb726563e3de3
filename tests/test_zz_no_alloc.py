"""GPU tests of uq_moments_noalloc, the allocation-free variant of uq_moments:
through the C-ABI it gives bit for bit the results of uq_moments on two calls
in a row (the second on a smaller job, so stale scratch contents of the
first would show), allocates no device memory (the job's device bytes and
torch's allocated bytes are unchanged), serialises concurrent callers, fits
the benchmark workload's velocity-field statistics, and refuses a request
larger than its fixed scratch array with a clear error."""
import sys
import threading

import numpy as np
import pytest

from helpers import gpu_available
from paper_2508_13867_amd import Job, UQError
from paper_2508_13867_amd import _abi as A
from paper_2508_13867_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

SCRATCH_BYTES = 64 << 20  # UQ_NOALLOC_SCRATCH_BYTES

LARGE = dict(name="noalloc_large", geometry="tgv", precision="fp64", nx=72, ny=40, steps=37, u0=0.02, nu=0.005,
             dists=[("nu", 0.004, 0.006), ("u0", 0.018, 0.022), ("phase_x", 0.0, 6.283185307179586)],
             rule=dict(kind="gl", n=3, order=2))
SMALL = dict(name="noalloc_small", geometry="tgv", precision="fp32", nx=24, ny=16, steps=21, u0=0.02, nu=0.006,
             dists=[("nu", 0.004, 0.008), ("u0", 0.018, 0.022)], rule=dict(kind="mc", N=5, seed=W.SEED + 7))
CHANNEL = dict(name="noalloc_channel", geometry="channel", precision="fp32", nx=66, ny=21, steps=120, u_peak=0.05,
               nu=0.05, D=6, cx=12, cy=10, ramp=40, xbc="zouhe", dists=[("re", 16.0, 24.0), ("u_peak", 0.045, 0.055)],
               rule=dict(kind="gl", n=3, order=2))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same(a, b):
    assert set(a) == set(b)
    for k in a:
        assert a[k].shape == b[k].shape, k
        assert np.array_equal(a[k], b[k]), (k, np.max(np.abs(a[k] - b[k])))


def noalloc_unallocating(job, qoi):
    """uq_moments_noalloc, checking that neither the job nor torch allocates."""
    import torch

    torch.cuda.synchronize()
    held, torch_bytes = job.info().device_bytes, torch.cuda.memory_allocated()
    res = job.moments(qoi, noalloc=True)
    torch.cuda.synchronize()
    assert job.info().device_bytes == held
    assert torch.cuda.memory_allocated() == torch_bytes
    return res


def test_noalloc_equals_moments_on_two_calls_in_a_row():
    say("case noalloc: large FP64 job then small FP32 job, vel and ke")
    with Job(LARGE) as big, Job(SMALL) as small:
        big.run(LARGE["steps"])
        small.run(SMALL["steps"])
        first = {q: noalloc_unallocating(big, q) for q in ("vel", "ke")}
        second = {q: noalloc_unallocating(small, q) for q in ("vel", "ke")}
        for q in ("vel", "ke"):
            same(first[q], big.moments(q))
            same(second[q], small.moments(q))
        # and once more in the other order, now that the job buffers exist
        same(noalloc_unallocating(small, "speed"), small.moments("speed"))
        same(noalloc_unallocating(big, "rho"), big.moments("rho"))


def test_noalloc_drag_of_a_channel_job():
    say("case noalloc: channel cd/cl")
    with Job(CHANNEL) as j:
        j.run(CHANNEL["steps"])
        got = {q: noalloc_unallocating(j, q) for q in ("cd", "cl")}
        for q in ("cd", "cl"):
            same(got[q], j.moments(q))


def test_noalloc_concurrent_callers_are_serialised():
    say("case noalloc: two threads on one GPU")
    with Job(LARGE) as big, Job(SMALL) as small:
        big.run(LARGE["steps"])
        small.run(SMALL["steps"])
        ref = {"big": big.moments("vel"), "small": small.moments("vel")}
        out, errs = {}, []

        def work(name, job):
            try:
                for _ in range(4):
                    out[name] = job.moments("vel", noalloc=True)
            except Exception as e:  # reported below
                errs.append(e)

        ts = [threading.Thread(target=work, args=("big", big)), threading.Thread(target=work, args=("small", small))]
        for t in ts:
            t.start()
        for t in ts:
            t.join(120)
        assert not errs, errs
        same(out["big"], ref["big"])
        same(out["small"], ref["small"])


def test_noalloc_benchmark_velocity_field():
    # 256^2 x 256 samples, K = 35: (35 + 3) x 131072 doubles = 39.8 MB of
    # outputs in the scratch array, no per-sample field buffer
    say("case noalloc: benchmark workload velocity field")
    spec = W.scaled(W.TGV_BATCHED_FP32, steps=12)
    with Job(spec) as j:
        j.run(spec["steps"])
        same(noalloc_unallocating(j, "vel"), j.moments("vel"))


def test_noalloc_refuses_more_than_its_scratch():
    say("case noalloc: request above the scratch size")
    # the velocity field of a 1024^2 lattice with K = 6 gPC terms: (K + 3)
    # outputs of 2 * 1024^2 doubles, 151 MB
    spec = dict(name="noalloc_too_big", geometry="tgv", precision="fp32", nx=1024, ny=1024, steps=2, u0=0.02,
                nu=0.005, dists=[("nu", 0.004, 0.006), ("u0", 0.018, 0.022)], rule=dict(kind="gl", n=3, order=2))
    need = 8 * (6 + 3) * 2 * 1024 * 1024
    assert need > SCRATCH_BYTES
    with Job(spec) as j:
        j.run(2)
        held = j.info().device_bytes
        with pytest.raises(UQError) as e:
            j.moments("vel", noalloc=True)
        assert e.value.status == A.UQ_EINVAL
        assert "scratch" in str(e.value) and str(SCRATCH_BYTES) in str(e.value)
        assert j.info().device_bytes == held
        # a scalar QoI of the same job fits
        same(j.moments("ke", noalloc=True), j.moments("ke"))
