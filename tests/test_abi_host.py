"""C-ABI library: loads, exports every declared symbol, and its host-only
logic (sample sets, basis, validation) agrees with the oracle. No GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2508_13867_amd import _abi as A
from paper_2508_13867_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "uq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(uq_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = A.lib()
    names = declared_functions()
    assert "uq_create" in names and "uq_moments" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) <= set(A.SIGNATURES), set(names) - set(A.SIGNATURES)


def declared_signatures():
    """{name: (return type, [parameter types])} of every function in uq.h."""
    text = open(os.path.join(ROOT, "include", "uq.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for m in re.finditer(r"^\s*((?:const\s+)?[a-z_0-9]+\s*\*?)\s*(uq_[a-z_0-9]+)\s*\(([^)]*)\)\s*;", text,
                         flags=re.M):
        params = [p.strip() for p in m.group(3).split(",") if p.strip() and p.strip() != "void"]
        # drop each parameter's name (the identifier after the type)
        types = [re.sub(r"\s+", " ", re.sub(r"(?<=[\s*])[A-Za-z_][A-Za-z_0-9]*$", "", p).strip()).replace(" *", "*")
                 for p in params]
        out[m.group(2)] = (m.group(1).strip(), types)
    return out


def test_binding_signatures_match_header():
    # every parameter of every declared function has the C type the ctypes
    # binding passes: structs by pointer to their mirror (or an untyped
    # pointer for caller buffers), opaque handles as pointers, integers at
    # their width, doubles as doubles
    mirrors = {"uq_problem": A.Problem, "uq_device": A.Device, "uq_moments_out": A.MomentsOut,
               "uq_job_info": A.JobInfo, "uq_tune_result": A.TuneResult, "uq_server_config": A.ServerConfig,
               "uq_result": A.Result, "uq_server_stats": A.ServerStats}
    scalars = {"int32_t": C.c_int32, "int64_t": C.c_int64, "uint64_t": C.c_uint64, "double": C.c_double}
    opaque = {"uq_job", "uq_server"}

    def ok(ctype, arg):
        base = ctype.replace("const ", "").rstrip("*").strip()
        if ctype.endswith("**"):
            return arg in (C.c_void_p, C.POINTER(C.c_void_p))
        if ctype.endswith("*"):
            if base in opaque:
                return arg is C.c_void_p
            if base in mirrors:
                return arg is C.POINTER(mirrors[base])
            return arg is C.c_void_p or arg is C.POINTER(scalars[base])
        return arg is scalars[base] or (base == "int32_t" and arg is C.c_int32)

    sigs = declared_signatures()
    assert "uq_server_create" in sigs and sigs["uq_server_create"][1][1] == "const uq_device*"
    for name, (_, params) in sigs.items():
        _, args = A.SIGNATURES[name]
        assert len(args) == len(params), name
        for k, (ctype, arg) in enumerate(zip(params, args)):
            assert ok(ctype, arg), (name, k, ctype, arg)


def test_struct_layout_matches_header(tmp_path):
    # the ctypes mirrors must have the C compiler's layout of uq.h
    import subprocess

    structs = {"uq_dist": A.Dist, "uq_problem": A.Problem, "uq_device": A.Device,
               "uq_moments_out": A.MomentsOut, "uq_job_info": A.JobInfo, "uq_tune_result": A.TuneResult,
               "uq_server_config": A.ServerConfig, "uq_result": A.Result, "uq_server_stats": A.ServerStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "uq.h"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    for line in out:
        if not line:
            continue
        cname, field, val = line.split()
        py = structs[cname]
        got = C.sizeof(py) if field == "sizeof" else getattr(py, field).offset
        assert got == int(val), (cname, field, got, val)


@pytest.mark.parametrize("spec", [W.TGV_SMALL_FP64, W.TGV_BATCHED_FP32, W.CYLINDER_FP32])
def test_collocation_rule_matches_oracle(spec):
    xi, a, alpha, phi = A.rule_points(spec)
    d, n, P = len(spec["dists"]), spec["rule"]["n"], spec["rule"]["order"]
    xo, ao = O.gl_tensor(d, n)
    assert np.abs(xi - xo).max() < 1e-15 and np.abs(a - ao).max() < 1e-15
    assert np.array_equal(alpha, O.multi_indices(d, P))
    assert np.abs(phi - O.phi_table(xo, alpha)).max() < 1e-12


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_smolyak_rule_matches_oracle(level):
    spec = W.scaled(W.TGV_BATCHED_FP32, rule=dict(kind="smolyak", level=level, order=min(level, 3)))
    xi, a, alpha, phi = A.rule_points(spec)
    xo, ao = O.smolyak(4, level)
    assert xi.shape == xo.shape and np.abs(xi - xo).max() < 1e-15 and np.abs(a - ao).max() < 1e-13
    assert np.abs(phi - O.phi_table(xo, alpha)).max() < 1e-12


def test_halton_and_lhs_match_oracle():
    xi, a, _, _ = A.rule_points(W.scaled(W.TGV_MC, rule=dict(kind="halton", N=1000)))
    xo, ao = O.halton(1000, 4)
    assert np.abs(xi - xo).max() < 1e-15 and np.array_equal(a, ao)
    xi, a, _, _ = A.rule_points(W.scaled(W.TGV_MC, rule=dict(kind="lhs", N=777, seed=9)))
    xo, ao = O.lhs(9, 777, 4)
    assert np.array_equal(xi, xo) and np.array_equal(a, ao)


def test_monte_carlo_points_bit_exact_with_oracle():
    xi, a, alpha, phi = A.rule_points(W.TGV_MC)
    xo, ao = O.mc_points(W.SEED, 4096, 4)
    assert np.array_equal(xi, xo) and np.array_equal(a, ao)
    assert alpha.shape == (0, 4)


@pytest.mark.parametrize("bad", [
    dict(nx=1), dict(ny=1), dict(precision="fp64", rule=dict(kind="gl", n=0, order=1)),
    dict(rule=dict(kind="mc", N=1, seed=1)), dict(dists=[("re", 10, 20)]),
    dict(dists=[("nu", 0.02, 0.01)]), dict(dists=[("nu", 0.1, 0.2), ("nu", 0.1, 0.2)]),
])
def test_invalid_problems_are_rejected(bad):
    spec = W.scaled(W.TGV_SMALL_FP64, **bad)
    with pytest.raises(A.UQError) as e:
        A.rule_points(spec)
    assert e.value.status == A.UQ_EINVAL
    assert A.lib().uq_last_error().decode()


def test_tgv_units_match_the_papers_table():
    # Table tab:simulation_parameters (values as printed, 6 decimals)
    rows = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "table1_tgv_units.txt"), comments="#")
    for N, n, Ma, Re, tau, dx, dt in rows:
        u = A.tgv_units(int(n), Ma, Re)
        assert abs(u["tau"] - tau) < 1e-6 and abs(u["dx"] - dx) < 1e-6 and abs(u["dt"] - dt) < 1e-6, n
        assert abs(u["u_lat"] - Ma / np.sqrt(3.0)) < 1e-16
        assert abs(u["tau"] - (3 * u["nu"] + 0.5)) < 1e-15
    with pytest.raises(A.UQError):
        A.tgv_units(1, 0.1, 100)
