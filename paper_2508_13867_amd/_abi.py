"""ctypes binding of include/uq.h (argument marshalling only).

Every computation happens in libuqlbm.so; this module only converts Python
values to the C structs, hands torch-allocated device memory and torch's
current stream to the library, and copies results into numpy arrays. If the
library is missing it raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libuqlbm.so")

UQ_OK, UQ_EINVAL, UQ_ENOMEM, UQ_EAGAIN, UQ_EUNSTABLE, UQ_EDEVICE, UQ_ESTATE = range(7)
STATUS_NAMES = {0: "UQ_OK", 1: "UQ_EINVAL", 2: "UQ_ENOMEM", 3: "UQ_EAGAIN", 4: "UQ_EUNSTABLE",
                5: "UQ_EDEVICE", 6: "UQ_ESTATE"}
PRECISION = {"fp64": 0, "fp32": 1, "fp16s": 2, "bf16s": 3}
GEOMETRY = {"tgv": 0, "channel": 1}
XBC = {0: 0, 1: 1, 2: 2, 3: 3, "zouhe": 0, "walls": 1, "periodic": 2, "interp": 3}
CYL_BC = {"halfway": 0, "bouzidi": 1}
FORCE_REF = {"peak": 0, "mean": 1}
TARGET = {"nu": 0, "u0": 1, "phase_x": 2, "phase_y": 3, "re": 4, "u_peak": 5, "zeta00": 6, "zeta01": 7,
          "zeta10": 8, "zeta11": 9}
INIT = {"tgv": 0, "harmonic": 1}
RULE = {"gl": 0, "mc": 1, "smolyak": 2, "halton": 3, "lhs": 4}
LAYOUT = {"auto": 0, "aa": 1, "ab": 2}
QOI = {"ke": 0, "vel": 1, "cd": 2, "cl": 3, "rho": 4, "speed": 5}
MAX_DIMS = 8


class UQError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Dist(C.Structure):
    _fields_ = [("target", C.c_int32), ("lo", C.c_double), ("hi", C.c_double)]


class Problem(C.Structure):
    _fields_ = [
        ("geometry", C.c_int32), ("precision", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
        ("nu", C.c_double), ("u0", C.c_double), ("phase_x", C.c_double), ("phase_y", C.c_double),
        ("u_peak", C.c_double), ("D", C.c_int32), ("cx", C.c_int32), ("cy", C.c_int32), ("xbc", C.c_int32),
        ("ramp", C.c_int64), ("n_dists", C.c_int32), ("dists", Dist * MAX_DIMS), ("rule", C.c_int32),
        ("n_per_dim", C.c_int32), ("order", C.c_int32), ("mc_n", C.c_int64), ("seed", C.c_uint64),
        ("layout", C.c_int32), ("level", C.c_int32), ("init", C.c_int32),
        ("cyl_bc", C.c_int32), ("force_ref", C.c_int32),
        ("cyl_x", C.c_double), ("cyl_y", C.c_double), ("cyl_d", C.c_double),
    ]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Device(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("ctx", C.c_void_p)]


class MomentsOut(C.Structure):
    _fields_ = [("n_out", C.c_int64), ("K", C.c_int32), ("d", C.c_int32), ("mean", C.c_void_p),
                ("var", C.c_void_p), ("var_alt", C.c_void_p), ("coeffs", C.c_void_p), ("alpha", C.c_void_p)]


class JobInfo(C.Structure):
    _fields_ = [("S", C.c_int64), ("d", C.c_int32), ("K", C.c_int32), ("steps_done", C.c_int64),
                ("pitch", C.c_int64), ("device_bytes", C.c_int64), ("scale_exp", C.c_int32),
                ("fluid_nodes", C.c_int32), ("layout", C.c_int32), ("cpt", C.c_int32), ("nt_store", C.c_int32),
                ("plane_pad", C.c_int32), ("bx", C.c_int32), ("fused", C.c_int32), ("fused_rows", C.c_int32),
                ("step_launches", C.c_int64), ("fused_window", C.c_int32), ("pad3", C.c_int32)]


class TuneResult(C.Structure):
    _fields_ = [("layout", C.c_int32), ("cpt", C.c_int32), ("nt_store", C.c_int32), ("plane_pad", C.c_int32),
                ("bx", C.c_int32), ("gbs", C.c_double), ("ms_per_step", C.c_double), ("n_candidates", C.c_int32),
                ("fused", C.c_int32), ("fused_rows", C.c_int32), ("fused_window", C.c_int32)]


RESULT_MAX_COEFFS = 256
SERVE = {"batched": 0, "plain": 1}


class ServerConfig(C.Structure):
    _fields_ = [("memory_budget", C.c_int64), ("max_jobs", C.c_int32), ("steps_per_tick", C.c_int32),
                ("mode", C.c_int32), ("use_graph", C.c_int32), ("precision", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("status", C.c_int32), ("qoi", C.c_int32), ("S", C.c_int64),
                ("K", C.c_int32), ("pad0", C.c_int32), ("mean", C.c_double), ("var", C.c_double),
                ("var_alt", C.c_double), ("coeffs", C.c_double * RESULT_MAX_COEFFS), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("node_updates", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64), ("pending", C.c_int64),
                ("live", C.c_int64), ("elapsed_s", C.c_double), ("busy_s", C.c_double),
                ("node_updates", C.c_double), ("solves_per_hour", C.c_double), ("mlups", C.c_double),
                ("latency_p50_s", C.c_double), ("latency_p99_s", C.c_double), ("latency_mean_s", C.c_double),
                ("arena_bytes", C.c_int64), ("arena_peak_bytes", C.c_int64)]


# every symbol the header declares, with its signature
_P = C.c_void_p
SIGNATURES = {
    "uq_create": (C.c_int, [C.POINTER(Problem), C.POINTER(Device), C.POINTER(_P)]),
    "uq_samples": (C.c_int, [_P, _P, _P, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "uq_run": (C.c_int, [_P, C.c_int64]),
    "uq_run_timed": (C.c_int, [_P, C.c_int64, C.POINTER(C.c_double)]),
    "uq_sync": (C.c_int, [_P]),
    "uq_qoi_samples": (C.c_int, [_P, C.c_int32, _P, C.POINTER(C.c_int64)]),
    "uq_moments": (C.c_int, [_P, C.c_int32, C.POINTER(MomentsOut)]),
    "uq_moments_noalloc": (C.c_int, [_P, C.c_int32, C.POINTER(MomentsOut)]),
    "uq_populations": (C.c_int, [_P, C.c_int64, _P]),
    "uq_job_get_info": (C.c_int, [_P, C.POINTER(JobInfo)]),
    "uq_destroy": (None, [_P]),
    "uq_last_error": (C.c_char_p, []),
    "uq_autotune": (C.c_int, [C.POINTER(Problem), C.POINTER(Device), C.c_int64, C.POINTER(TuneResult)]),
    "uq_server_create": (C.c_int, [C.POINTER(ServerConfig), C.POINTER(Device), C.POINTER(_P)]),
    "uq_server_submit": (C.c_int, [_P, C.POINTER(Problem), C.c_int64, C.c_int32, C.POINTER(C.c_uint64)]),
    "uq_server_poll": (C.c_int, [_P, C.c_uint64, C.POINTER(Result)]),
    "uq_server_wait": (C.c_int, [_P, C.c_uint64, C.c_double, C.POINTER(Result)]),
    "uq_server_get_stats": (C.c_int, [_P, C.POINTER(ServerStats)]),
    "uq_server_destroy": (None, [_P]),
    "uq_wasserstein1": (C.c_int, [_P, _P, C.c_int32, C.c_double, C.c_double, C.POINTER(C.c_double)]),
    "uq_tgv_units": (C.c_int, [C.c_int32, C.c_double, C.c_double] + [C.POINTER(C.c_double)] * 5),
    "uq_rule_size": (C.c_int, [C.POINTER(Problem), C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "uq_rule_points": (C.c_int, [C.POINTER(Problem), _P, _P, _P, _P]),
}

_lib = None


def lib():
    """Load libuqlbm.so (built in-tree by paper_2508_13867_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                              "python paper_2508_13867_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != UQ_OK:
        raise UQError(status, lib().uq_last_error().decode())


def make_problem(spec: dict) -> Problem:
    """Marshal a problem dict (keys as in workloads.py) into the C struct."""
    p = Problem()
    p.geometry = GEOMETRY[spec["geometry"]]
    p.precision = PRECISION[spec.get("precision", "fp32")]
    p.nx, p.ny = int(spec["nx"]), int(spec["ny"])
    p.nu = float(spec.get("nu", 0.0))
    p.u0 = float(spec.get("u0", 0.0))
    p.phase_x = float(spec.get("phase_x", 0.0))
    p.phase_y = float(spec.get("phase_y", 0.0))
    p.u_peak = float(spec.get("u_peak", 0.0))
    p.D = int(spec.get("D", 0))
    p.cx = int(spec.get("cx", 0))
    p.cy = int(spec.get("cy", 0))
    p.xbc = XBC[spec.get("xbc", 0)]
    p.ramp = int(spec.get("ramp", 0))
    dists = spec.get("dists", [])
    if len(dists) > MAX_DIMS:
        raise ValueError("too many uncertain inputs")
    p.n_dists = len(dists)
    for k, (t, lo, hi) in enumerate(dists):
        p.dists[k].target = TARGET[t]
        p.dists[k].lo = float(lo)
        p.dists[k].hi = float(hi)
    r = spec["rule"]
    p.rule = RULE[r["kind"]]
    p.n_per_dim = int(r.get("n", 0))
    p.order = int(r.get("order", 0))
    p.mc_n = int(r.get("N", 0))
    p.seed = int(r.get("seed", 123456))
    p.layout = LAYOUT[spec.get("layout", "auto")]
    p.level = int(r.get("level", 0))
    p.init = INIT[spec.get("init", "tgv")]
    p.cyl_bc = CYL_BC[spec.get("cyl_bc", "halfway")]
    p.force_ref = FORCE_REF[spec.get("force_ref", "peak")]
    p.cyl_x = float(spec.get("cyl_x", 0.0))
    p.cyl_y = float(spec.get("cyl_y", 0.0))
    p.cyl_d = float(spec.get("cyl_d", 0.0))
    return p


def rule_points(spec: dict):
    """Host-only: the sample set (xi, a) and, for collocation, alpha and Phi."""
    p = make_problem(spec)
    S, K = C.c_int64(), C.c_int32()
    check(lib().uq_rule_size(C.byref(p), C.byref(S), C.byref(K)))
    d = p.n_dists
    xi = np.zeros((S.value, d))
    a = np.zeros(S.value)
    alpha = np.zeros((K.value, d), np.int32)
    phi = np.zeros((S.value, K.value))
    check(lib().uq_rule_points(C.byref(p), xi.ctypes.data, a.ctypes.data, alpha.ctypes.data, phi.ctypes.data))
    return xi, a, alpha, phi


class TorchAllocator:
    """Device memory for the library from torch's caching allocator."""

    def __init__(self, device: int):
        import torch

        self.torch = torch
        self.device = device
        self.live = {}
        self._alloc = ALLOC_FN(self.alloc)
        self._free = FREE_FN(self.free)

    def alloc(self, nbytes, ctx):
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=f"cuda:{self.device}")
        except Exception:
            return None
        ptr = t.data_ptr()
        self.live[ptr] = t
        return ptr

    def free(self, ptr, ctx):
        self.live.pop(ptr, None)


def _pinned(shape):
    """An uninitialised float64 host array in page-locked memory (torch's
    caching host allocator: blocks are reused across calls); the array keeps
    its tensor, and so the memory, alive."""
    import torch

    return torch.empty(shape, dtype=torch.float64, pin_memory=True).numpy()


def torch_device(device: int = 0, stream=None, allocator=True):
    """uq_device for `device`, torch's current stream and torch memory."""
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the library runs only on an MI355X (gfx950)")
    dev = Device()
    dev.device = device
    s = stream if stream is not None else torch.cuda.current_stream(device)
    dev.stream = C.c_void_p(s.cuda_stream)
    keep = None
    if allocator:
        keep = TorchAllocator(device)
        dev.alloc = keep._alloc
        dev.free = keep._free
    else:
        dev.alloc = ALLOC_FN()
        dev.free = FREE_FN()
    dev.ctx = None
    return dev, keep


def tgv_units(n: int, Ma: float, Re: float) -> dict:
    """Lattice units of the four-dimensional vortex case (uq_tgv_units)."""
    v = [C.c_double() for _ in range(5)]
    check(lib().uq_tgv_units(int(n), float(Ma), float(Re), *[C.byref(x) for x in v]))
    return dict(zip(("nu", "u_lat", "dx", "dt", "tau"), (x.value for x in v)))


def wasserstein1(a: "Job", b: "Job", qoi: str = "speed", scale_a: float = 1.0, scale_b: float = 1.0) -> float:
    """uq_wasserstein1: W_1 between the laws of a field QoI of two jobs."""
    w = C.c_double()
    check(lib().uq_wasserstein1(a.h, b.h, QOI[qoi], float(scale_a), float(scale_b), C.byref(w)))
    return w.value


def autotune(spec: dict, steps: int = 40, device: int = 0) -> dict:
    """uq_autotune: measure every launch-shape candidate of the problem class
    and make the fastest the shape of later jobs of that class."""
    dev, keep = torch_device(device, None, True)
    p = make_problem(spec)
    r = TuneResult()
    check(lib().uq_autotune(C.byref(p), C.byref(dev), int(steps), C.byref(r)))
    del keep
    return {"layout": {1: "aa", 2: "ab"}[r.layout], "cpt": r.cpt, "nt_store": r.nt_store,
            "plane_pad": r.plane_pad, "bx": r.bx, "gbs": r.gbs, "ms_per_step": r.ms_per_step,
            "n_candidates": r.n_candidates, "fused": r.fused, "fused_rows": r.fused_rows,
            "fused_window": r.fused_window}


class Job:
    """One UQ job (uq_create ... uq_destroy)."""

    def __init__(self, spec: dict, device: int = 0, stream=None, torch_memory: bool = True):
        self.spec = dict(spec)
        self._dev, self._keep = torch_device(device, stream, torch_memory)
        p = make_problem(spec)
        h = C.c_void_p()
        check(lib().uq_create(C.byref(p), C.byref(self._dev), C.byref(h)))
        self.h = h
        info = self.info()
        self.S, self.d, self.K = info.S, info.d, info.K

    def info(self) -> JobInfo:
        inf = JobInfo()
        check(lib().uq_job_get_info(self.h, C.byref(inf)))
        return inf

    def samples(self):
        xi = np.zeros((self.S, self.d))
        a = np.zeros(self.S)
        check(lib().uq_samples(self.h, xi.ctypes.data, a.ctypes.data, None, None))
        return xi, a

    def run(self, steps: int):
        check(lib().uq_run(self.h, int(steps)))

    def run_timed(self, steps: int) -> float:
        """Run and wait; returns the device time of the step launches in ms."""
        ms = C.c_double()
        check(lib().uq_run_timed(self.h, int(steps), C.byref(ms)))
        return ms.value

    def sync(self):
        check(lib().uq_sync(self.h))

    def qoi_samples(self, qoi: str) -> np.ndarray:
        n = C.c_int64()
        check(lib().uq_qoi_samples(self.h, QOI[qoi], None, C.byref(n)))
        out = np.zeros((self.S, n.value))
        check(lib().uq_qoi_samples(self.h, QOI[qoi], out.ctypes.data, C.byref(n)))
        return out

    def moments(self, qoi: str, noalloc: bool = False) -> dict:
        """uq_moments, or uq_moments_noalloc (no device allocation) if asked.
        The result arrays are page-locked host memory (every entry is written
        by the library), so that its device-to-host copies of field moments
        (tens of MB) run at the link's rate."""
        n = C.c_int64()
        check(lib().uq_qoi_samples(self.h, QOI[qoi], None, C.byref(n)))
        n = n.value
        mean, var, alt = _pinned(n), _pinned(n), _pinned(n)
        res = {"mean": mean, "var": var, "var_alt": alt}
        m = MomentsOut()
        m.mean, m.var, m.var_alt = mean.ctypes.data, var.ctypes.data, alt.ctypes.data
        if self.K > 0:
            coeffs = _pinned((self.K, n))
            alpha = np.zeros((self.K, self.d), np.int32)
            m.coeffs, m.alpha = coeffs.ctypes.data, alpha.ctypes.data
            res["coeffs"], res["alpha"] = coeffs, alpha
        fn = lib().uq_moments_noalloc if noalloc else lib().uq_moments
        check(fn(self.h, QOI[qoi], C.byref(m)))
        return res

    def populations(self, sample: int) -> np.ndarray:
        nx, ny = self.spec["nx"], self.spec["ny"]
        out = np.zeros((9, ny, nx))
        check(lib().uq_populations(self.h, int(sample), out.ctypes.data))
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().uq_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _result_dict(r: Result) -> dict:
    K = r.K
    return {"ticket": r.ticket, "status": r.status, "qoi": r.qoi, "S": r.S, "K": K, "mean": r.mean,
            "var": r.var, "var_alt": r.var_alt, "coeffs": np.array(r.coeffs[:min(K, RESULT_MAX_COEFFS)]),
            "t_submit": r.t_submit, "t_admit": r.t_admit, "t_done": r.t_done, "node_updates": r.node_updates,
            "latency_s": r.t_done - r.t_submit}


class Server:
    """A continuous-batching UQ server (uq_server_*) on one GPU."""

    def __init__(self, memory_budget_gb: float = 16.0, max_jobs: int = 64, steps_per_tick: int = 64,
                 mode: str = "batched", use_graph: bool = True, precision: str = "fp32", device: int = 0,
                 stream=None, torch_memory: bool = True):
        # the arena comes from torch's caching allocator (or hipMalloc), and
        # torch's current stream orders the server against the caller
        self._dev, self._keep = torch_device(device, stream, torch_memory)
        cfg = ServerConfig()
        cfg.memory_budget = int(memory_budget_gb * (1 << 30))
        cfg.max_jobs = max_jobs
        cfg.steps_per_tick = steps_per_tick
        cfg.mode = SERVE[mode]
        cfg.use_graph = 1 if use_graph else 0
        cfg.precision = PRECISION[precision]
        h = C.c_void_p()
        check(lib().uq_server_create(C.byref(cfg), C.byref(self._dev), C.byref(h)))
        self.h = h

    def submit(self, spec: dict, steps: int | None = None, qoi: str | None = None) -> int:
        p = make_problem(spec)
        if qoi is None:
            qoi = "ke" if spec["geometry"] == "tgv" else "cd"
        t = C.c_uint64()
        check(lib().uq_server_submit(self.h, C.byref(p), int(spec["steps"] if steps is None else steps), QOI[qoi],
                                     C.byref(t)))
        return t.value

    def poll(self, ticket: int):
        r = Result()
        st = lib().uq_server_poll(self.h, ticket, C.byref(r))
        if st == UQ_EAGAIN:
            return None
        check(st)
        return _result_dict(r)

    def wait(self, ticket: int, timeout_s: float = -1.0) -> dict:
        r = Result()
        check(lib().uq_server_wait(self.h, ticket, float(timeout_s), C.byref(r)))
        return _result_dict(r)

    def stats(self) -> dict:
        st = ServerStats()
        check(lib().uq_server_get_stats(self.h, C.byref(st)))
        return {name: getattr(st, name) for name, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            lib().uq_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
