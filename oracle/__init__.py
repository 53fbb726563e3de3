"""FP64 CPU oracle for the batched LBM-UQ path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package. It is a plain, slow, single-threaded double-precision
implementation written from the paper (OpenLB-UQ, arXiv 2508.13867):

* the lattice Boltzmann solve per sample (Sec. "Lattice Boltzmann methods":
  Eqs. deterministicLBE, bgkCollision, equilibrium, the D2Q9 set and weights,
  and the collide/stream split) lives in ``oracle.c``;
* the non-intrusive UQ algorithm (Algorithm alg:uq_openlb: generate samples,
  solve each one in turn, then Monte Carlo or stochastic-collocation
  statistics) is ``run_problem`` below, looping over samples one at a time.

It shares no code with the GPU library and imports nothing from it. Problems
are plain dicts (keys documented in ``run_problem``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from math import comb

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _declare(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_u64p = C.POINTER(C.c_uint64)


def _declare(L):
    L.oracle_d2q9.argtypes = [_ip, _ip, _dp, _ip]
    L.oracle_feq.argtypes = [C.c_double, C.c_double, C.c_double, _dp]
    L.oracle_collide.argtypes = [_dp, C.c_double, _dp]
    L.oracle_table1_units.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp, _dp]
    L.oracle_legendre_orthonormal.argtypes = [C.c_int, C.c_double]
    L.oracle_legendre_orthonormal.restype = C.c_double
    L.oracle_gauss_legendre.argtypes = [C.c_int, _dp, _dp]
    L.oracle_gl_tensor.argtypes = [C.c_int, C.c_int, _dp, _dp]
    L.oracle_multi_indices.argtypes = [C.c_int, C.c_int, _ip]
    L.oracle_multi_indices.restype = C.c_int
    L.oracle_phi_table.argtypes = [C.c_long, C.c_int, _dp, C.c_int, _ip, _dp]
    L.oracle_splitmix64_stream.argtypes = [C.c_uint64, C.c_long, _u64p]
    L.oracle_mc_points.argtypes = [C.c_uint64, C.c_long, C.c_int, _dp, _dp]
    L.oracle_mc_stats.argtypes = [C.c_long, C.c_long, _dp, _dp, _dp, _dp]
    L.oracle_gpc_stats.argtypes = [C.c_long, C.c_long, _dp, _dp, C.c_int, _dp, _dp, _dp, _dp, _dp]
    L.oracle_tgv_run.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, C.c_long,
                                 C.c_double, _dp, _dp, _dp, _dp, _dp]
    L.oracle_channel_run.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                     C.c_double, C.c_long, C.c_long, C.c_double, _dp, _dp, _dp, _dp, _dp, _dp,
                                     _dp]
    L.oracle_channel_run_opts.argtypes = [C.POINTER(ChannelOpts), _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.oracle_cylinder_nodes.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]
    L.oracle_cylinder_nodes.restype = C.c_long
    L.oracle_tgv_harmonic_run.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, _dp, C.c_long, C.c_double,
                                          _dp, _dp, _dp, _dp, _dp, _dp]
    L.oracle_cc_points.argtypes = [C.c_int]
    L.oracle_cc_rule.argtypes = [C.c_int, _dp, _dp]
    L.oracle_smolyak.argtypes = [C.c_int, C.c_int, _dp, _dp]
    L.oracle_smolyak.restype = C.c_long
    L.oracle_halton.argtypes = [C.c_long, C.c_int, _dp, _dp]
    L.oracle_lhs.argtypes = [C.c_uint64, C.c_long, C.c_int, _dp, _dp]


def _p(a):
    return None if a is None else a.ctypes.data_as(_dp)


# --------------------------------------------------------------------------
# lattice constants and single-node operators


def d2q9():
    cx = np.zeros(9, np.int32)
    cy = np.zeros(9, np.int32)
    w = np.zeros(9)
    opp = np.zeros(9, np.int32)
    lib().oracle_d2q9(cx.ctypes.data_as(_ip), cy.ctypes.data_as(_ip), _p(w), opp.ctypes.data_as(_ip))
    return cx, cy, w, opp


def feq(rho, ux, uy):
    out = np.zeros(9)
    lib().oracle_feq(rho, ux, uy, _p(out))
    return out


def collide(f, tau):
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(9)
    lib().oracle_collide(_p(f), tau, _p(out))
    return out


def table1_units(n, Ma, Re):
    t, dx, dt = C.c_double(), C.c_double(), C.c_double()
    lib().oracle_table1_units(n, Ma, Re, C.byref(t), C.byref(dx), C.byref(dt))
    return t.value, dx.value, dt.value


# --------------------------------------------------------------------------
# quadrature, basis and sampling


def legendre_orthonormal(n, x):
    return lib().oracle_legendre_orthonormal(int(n), float(x))


def gauss_legendre(n):
    x = np.zeros(n)
    w = np.zeros(n)
    if lib().oracle_gauss_legendre(n, _p(x), _p(w)) != 0:
        raise ValueError("n must be >= 1")
    return x, w


def gl_tensor(d, n):
    S = n ** d
    xi = np.zeros((S, d))
    a = np.zeros(S)
    lib().oracle_gl_tensor(d, n, _p(xi), _p(a))
    return xi, a


def multi_indices(d, P):
    K = comb(d + P, P)
    al = np.zeros((K, d), np.int32)
    k = lib().oracle_multi_indices(d, P, al.ctypes.data_as(_ip))
    assert k == K
    return al


def phi_table(xi, alpha):
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    alpha = np.ascontiguousarray(alpha, dtype=np.int32)
    S, d = xi.shape
    K = alpha.shape[0]
    phi = np.zeros((S, K))
    lib().oracle_phi_table(S, d, _p(xi), K, alpha.ctypes.data_as(_ip), _p(phi))
    return phi


def splitmix64_stream(seed, n):
    out = np.zeros(n, np.uint64)
    lib().oracle_splitmix64_stream(C.c_uint64(seed), n, out.ctypes.data_as(_u64p))
    return out


def mc_points(seed, N, d):
    xi = np.zeros((N, d))
    a = np.zeros(N)
    lib().oracle_mc_points(C.c_uint64(seed), N, d, _p(xi), _p(a))
    return xi, a


def cc_rule(i):
    m = lib().oracle_cc_points(i)
    x, w = np.zeros(m), np.zeros(m)
    lib().oracle_cc_rule(i, _p(x), _p(w))
    return x, w


def smolyak(d, level):
    S = lib().oracle_smolyak(d, level, None, None)
    xi, a = np.zeros((S, d)), np.zeros(S)
    lib().oracle_smolyak(d, level, _p(xi), _p(a))
    return xi, a


def halton(N, d):
    xi, a = np.zeros((N, d)), np.zeros(N)
    lib().oracle_halton(N, d, _p(xi), _p(a))
    return xi, a


def lhs(seed, N, d):
    xi, a = np.zeros((N, d)), np.zeros(N)
    lib().oracle_lhs(C.c_uint64(seed), N, d, _p(xi), _p(a))
    return xi, a


# --------------------------------------------------------------------------
# statistics


def mc_stats(M):
    M = np.ascontiguousarray(M, dtype=np.float64)
    S = M.shape[0]
    n_out = int(np.prod(M.shape[1:])) if M.ndim > 1 else 1
    mean, var, var_n = (np.zeros(n_out) for _ in range(3))
    lib().oracle_mc_stats(S, n_out, _p(M), _p(mean), _p(var), _p(var_n))
    return {"mean": mean, "var": var, "var_alt": var_n}


def gpc_stats(M, a, phi):
    M = np.ascontiguousarray(M, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.float64)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    S = M.shape[0]
    n_out = int(np.prod(M.shape[1:])) if M.ndim > 1 else 1
    K = phi.shape[1]
    coeffs = np.zeros((K, n_out))
    mean, var, vq = (np.zeros(n_out) for _ in range(3))
    lib().oracle_gpc_stats(S, n_out, _p(M), _p(a), K, _p(phi), _p(coeffs), _p(mean), _p(var), _p(vq))
    return {"mean": mean, "var": var, "var_alt": vq, "coeffs": coeffs}


# --------------------------------------------------------------------------
# one deterministic solve


def tgv_run(nx, ny, nu, u0, steps, phase_x=0.0, phase_y=0.0, ke_u0=None, want_f=False):
    n = nx * ny
    rho, ux, uy = np.zeros(n), np.zeros(n), np.zeros(n)
    f = np.zeros(9 * n) if want_f else None
    ke = C.c_double()
    rc = lib().oracle_tgv_run(nx, ny, nu, u0, phase_x, phase_y, steps, u0 if ke_u0 is None else ke_u0,
                              _p(f), _p(rho), _p(ux), _p(uy), C.byref(ke))
    if rc != 0:
        raise ValueError("invalid TGV parameters (tau must exceed 1/2)")
    out = {"ke": ke.value, "rho": rho.reshape(ny, nx), "ux": ux.reshape(ny, nx), "uy": uy.reshape(ny, nx)}
    if want_f:
        out["f"] = f.reshape(9, ny, nx)
    return out


def tgv_harmonic_run(nx, ny, nu, u0, zeta, steps, ke_u0=None, want_f=False):
    n = nx * ny
    rho, ux, uy, sp = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n)
    f = np.zeros(9 * n) if want_f else None
    z = np.ascontiguousarray(zeta, dtype=np.float64)
    ke = C.c_double()
    rc = lib().oracle_tgv_harmonic_run(nx, ny, nu, u0, _p(z), steps, u0 if ke_u0 is None else ke_u0, _p(f),
                                       _p(rho), _p(ux), _p(uy), _p(sp), C.byref(ke))
    if rc != 0:
        raise ValueError("invalid TGV parameters (tau must exceed 1/2)")
    out = {"ke": ke.value, "rho": rho.reshape(ny, nx), "ux": ux.reshape(ny, nx), "uy": uy.reshape(ny, nx),
           "speed": sp.reshape(ny, nx)}
    if want_f:
        out["f"] = f.reshape(9, ny, nx)
    return out


def wasserstein1(xa, wa, xb, wb):
    """W_1 between two weighted empirical measures on the real line, as the
    integral over p in [0, 1] of |Q_a(p) - Q_b(p)| (Q the quantile functions):
    sort each, walk both piecewise-constant quantile functions together."""
    xa, wa, xb, wb = (np.asarray(v, dtype=np.float64).ravel() for v in (xa, wa, xb, wb))
    ia, ib = np.argsort(xa, kind="stable"), np.argsort(xb, kind="stable")
    xa, wa, xb, wb = xa[ia], wa[ia] / wa.sum(), xb[ib], wb[ib] / wb.sum()
    Pa, Pb = np.cumsum(wa), np.cumsum(wb)
    Pa[-1] = Pb[-1] = 1.0
    edges = np.union1d(Pa, Pb)
    lo = np.concatenate([[0.0], edges[:-1]])
    mid = 0.5 * (lo + edges)
    qa = xa[np.minimum(np.searchsorted(Pa, mid, side="left"), len(xa) - 1)]
    qb = xb[np.minimum(np.searchsorted(Pb, mid, side="left"), len(xb) - 1)]
    return float(np.sum(np.abs(qa - qb) * (edges - lo)))


def channel_run(nx, ny, nu, u_peak, steps, D=0, cx=0, cy=0, ramp=0, xbc=0, want_f=False, ux_init=0.0):
    n = nx * ny
    rho, ux, uy = np.zeros(n), np.zeros(n), np.zeros(n)
    f = np.zeros(9 * n) if want_f else None
    force, cdcl, wall = np.zeros(2), np.zeros(2), np.zeros(2)
    rc = lib().oracle_channel_run(nx, ny, xbc, D, cx, cy, nu, u_peak, ramp, steps, ux_init, _p(f), _p(rho), _p(ux),
                                  _p(uy), _p(force), _p(cdcl), _p(wall))
    if rc != 0:
        raise ValueError("invalid channel parameters")
    out = {"rho": rho.reshape(ny, nx), "ux": ux.reshape(ny, nx), "uy": uy.reshape(ny, nx),
           "force": force, "cd": cdcl[0], "cl": cdcl[1], "wall_force": wall}
    if want_f:
        out["f"] = f.reshape(9, ny, nx)
    return out


class ChannelOpts(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("xbc", C.c_int), ("cyl", C.c_int), ("D", C.c_int),
                ("cx", C.c_int), ("cy", C.c_int), ("ccx", C.c_double), ("ccy", C.c_double), ("R", C.c_double),
                ("q_lo", C.c_double), ("q_hi", C.c_double), ("q_fix", C.c_double), ("nu", C.c_double),
                ("u_peak", C.c_double), ("ramp", C.c_long), ("steps", C.c_long), ("ux_init", C.c_double),
                ("force_ref", C.c_int)]


def channel_run_opts(nx, ny, nu, u_peak, steps, xbc=0, cyl=0, D=0, cx=0, cy=0, ccx=0.0, ccy=0.0, R=0.0,
                     q_lo=-1.0, q_hi=-1.0, q_fix=-1.0, ramp=0, ux_init=0.0, force_ref=0, want_f=False, want_q=False):
    """Channel run with every option of the oracle: cyl = 1 is the exact
    circle (ccx, ccy, R) with interpolated bounce-back; q_lo / q_hi >= 0
    place the straight walls at y = -q_lo and y = ny - 1 + q_hi with the
    same interpolated rule; xbc = 3 is the finite-difference inlet/outlet."""
    o = ChannelOpts(nx=nx, ny=ny, xbc=xbc, cyl=cyl, D=D, cx=cx, cy=cy, ccx=ccx, ccy=ccy, R=R, q_lo=q_lo,
                    q_hi=q_hi, q_fix=q_fix, nu=nu, u_peak=u_peak, ramp=ramp, steps=steps, ux_init=ux_init,
                    force_ref=force_ref)
    n = nx * ny
    rho, ux, uy = np.zeros(n), np.zeros(n), np.zeros(n)
    f = np.zeros(9 * n) if want_f else None
    q = np.zeros(9 * n) if want_q else None
    force, cdcl, wall = np.zeros(2), np.zeros(2), np.zeros(2)
    rc = lib().oracle_channel_run_opts(C.byref(o), _p(f), _p(rho), _p(ux), _p(uy), _p(force), _p(cdcl), _p(wall),
                                       _p(q))
    if rc != 0:
        raise ValueError("invalid channel parameters")
    out = {"rho": rho.reshape(ny, nx), "ux": ux.reshape(ny, nx), "uy": uy.reshape(ny, nx),
           "force": force, "cd": cdcl[0], "cl": cdcl[1], "wall_force": wall}
    if want_f:
        out["f"] = f.reshape(9, ny, nx)
    if want_q:
        out["q"] = q.reshape(9, ny, nx)
    return out


def cylinder_nodes(nx, ny, D, cx, cy):
    return lib().oracle_cylinder_nodes(nx, ny, D, cx, cy)


# --------------------------------------------------------------------------
# the non-intrusive UQ algorithm, one sample after the other

_TARGETS = ("nu", "u0", "phase_x", "phase_y", "re", "u_peak", "zeta00", "zeta01", "zeta10", "zeta11")


def sample_set(problem):
    """Step 1 of the SC-gPC procedure / MC sample generation: (xi, a)."""
    d = len(problem["dists"])
    r = problem["rule"]
    if r["kind"] == "gl":
        return gl_tensor(d, r["n"])
    if r["kind"] == "mc":
        return mc_points(r.get("seed", 123456), r["N"], d)
    if r["kind"] == "smolyak":
        return smolyak(d, r["level"])
    if r["kind"] == "halton":
        return halton(r["N"], d)
    if r["kind"] == "lhs":
        return lhs(r.get("seed", 123456), r["N"], d)
    raise ValueError(r["kind"])


def sample_params(problem, xi_row):
    """Deterministic inputs of one sample: each uncertain input is the affine
    image (lo+hi)/2 + (hi-lo)/2 xi of its reference variable; a Reynolds-number
    input sets nu = U D / Re (the cylinder section's definition of Re), U the
    nominal peak inflow velocity or, with force_ref 'mean', its mean 2/3 of
    it, D the diameter."""
    p = {k: problem.get(k, 0.0) for k in _TARGETS}
    p["u_peak"] = problem.get("u_peak", 0.0)
    for (target, lo, hi), z in zip(problem["dists"], xi_row):
        if target not in _TARGETS:
            raise ValueError(target)
        p[target] = 0.5 * (lo + hi) + 0.5 * (hi - lo) * z
    if any(t == "re" for t, _, _ in problem["dists"]):
        U = problem["u_peak"] * (2.0 / 3.0 if problem.get("force_ref", "peak") == "mean" else 1.0)
        dia = problem["cyl_d"] if problem.get("cyl_bc", "halfway") == "bouzidi" else problem["D"]
        p["nu"] = U * dia / p["re"]
    return p


def solve_sample(problem, params, steps=None):
    """One deterministic LBM run of the given sample; returns its QoIs."""
    steps = problem["steps"] if steps is None else steps
    nx, ny = problem["nx"], problem["ny"]
    if problem["geometry"] == "tgv" and problem.get("init", "tgv") == "harmonic":
        zeta = [params["zeta00"], params["zeta01"], params["zeta10"], params["zeta11"]]
        r = tgv_harmonic_run(nx, ny, params["nu"], params["u0"], zeta, steps, ke_u0=problem["u0"])
        return {"ke": r["ke"], "vel": np.stack([r["ux"], r["uy"]]), "rho": r["rho"], "speed": r["speed"]}
    if problem["geometry"] == "tgv":
        r = tgv_run(nx, ny, params["nu"], params["u0"], steps, params["phase_x"], params["phase_y"],
                    ke_u0=problem["u0"])
        return {"ke": r["ke"], "vel": np.stack([r["ux"], r["uy"]]), "rho": r["rho"],
                "speed": np.sqrt(r["ux"] ** 2 + r["uy"] ** 2)}
    if problem["geometry"] == "channel":
        xbc = {"zouhe": 0, "walls": 1, "periodic": 2, "interp": 3}.get(problem.get("xbc", 0), problem.get("xbc", 0))
        fref = 1 if problem.get("force_ref", "peak") == "mean" else 0
        if problem.get("cyl_bc", "halfway") == "bouzidi":
            r = channel_run_opts(nx, ny, params["nu"], params["u_peak"], steps, xbc=xbc, cyl=1,
                                 ccx=problem["cyl_x"], ccy=problem["cyl_y"], R=0.5 * problem["cyl_d"],
                                 ramp=problem.get("ramp", 0), force_ref=fref)
        else:
            r = channel_run_opts(nx, ny, params["nu"], params["u_peak"], steps, xbc=xbc, D=problem.get("D", 0),
                                 cx=problem.get("cx", 0), cy=problem.get("cy", 0), ramp=problem.get("ramp", 0),
                                 force_ref=fref)
        return {"cd": r["cd"], "cl": r["cl"], "fx": r["force"][0], "fy": r["force"][1],
                "vel": np.stack([r["ux"], r["uy"]]), "rho": r["rho"], "speed": np.sqrt(r["ux"] ** 2 + r["uy"] ** 2)}
    raise ValueError(problem["geometry"])


def run_problem(problem, samples=None, qois=None, steps=None):
    """Algorithm alg:uq_openlb, sequentially.

    problem keys: geometry ('tgv' | 'channel'), nx, ny, steps, nominal inputs
    (nu, u0, phase_x, phase_y for the vortex; u_peak, D, cx, cy, ramp, xbc for
    the channel), dists = [(target, lo, hi), ...] with target in nu, u0,
    phase_x, phase_y, re, u_peak, and rule = {'kind': 'gl', 'n': points per
    dimension, 'order': P}, {'kind': 'smolyak', 'level': l, 'order': P},
    {'kind': 'mc' | 'halton' | 'lhs', 'N': samples, 'seed': s}.

    samples: optional subset of sample indices to solve (statistics are then
    not computed). Returns per-sample QoIs and, for the full set, statistics.
    """
    xi, a = sample_set(problem)
    S = xi.shape[0]
    idxs = range(S) if samples is None else samples
    per = [solve_sample(problem, sample_params(problem, xi[j]), steps) for j in idxs]
    names = qois or [k for k in per[0].keys()]
    out = {"xi": xi, "a": a, "samples": {k: np.array([p[k] for p in per]) for k in names}}
    if samples is not None:
        return out
    d = xi.shape[1]
    r = problem["rule"]
    stats = {}
    if r["kind"] in ("gl", "smolyak"):
        alpha = multi_indices(d, r["order"])
        phi = phi_table(xi, alpha)
        out["alpha"], out["phi"] = alpha, phi
        for k in names:
            stats[k] = gpc_stats(out["samples"][k].reshape(S, -1), a, phi)
    else:
        for k in names:
            stats[k] = mc_stats(out["samples"][k].reshape(S, -1))
    out["stats"] = stats
    return out
