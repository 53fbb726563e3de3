"""Shared test utilities (comparison metrics and GPU availability)."""
import numpy as np


def rel_l2(got, ref, scale=None):
    """||got - ref||_2 / ||ref||_2 over the whole output, or / scale."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = np.linalg.norm(ref) if scale is None else scale
    num = np.linalg.norm(got - ref)
    if den == 0:
        return num
    return num / den


def gpu_available():
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False


def stat_errors(st, ref, mean_scale=None):
    """Relative-L2 errors of a statistics result against a reference: mean
    (over mean_scale where the reference mean is near zero), var, var_alt,
    and for gPC the coefficients of degree >= 1 on their own norm (a norm
    over all coefficients is dominated by the mean's c_0, so it would hide
    errors in the terms that carry the variance)."""
    e = {"mean": rel_l2(st["mean"], ref["mean"], scale=mean_scale), "var": rel_l2(st["var"], ref["var"])}
    if "var_alt" in st and "var_alt" in ref:
        e["var_alt"] = rel_l2(st["var_alt"], ref["var_alt"])
    if "coeffs" in ref and np.asarray(ref["coeffs"]).shape[0] > 1:
        e["coeffs_k>=1"] = rel_l2(np.asarray(st["coeffs"])[1:], np.asarray(ref["coeffs"])[1:])
    return e


def assert_stats(st, ref, tol, label="", mean_scale=None):
    for k, e in stat_errors(st, ref, mean_scale).items():
        assert e < tol, (label, k, e, tol)


def assert_stats_given_samples(st, gpu_samples, ref, tol, label=""):
    """Statistics of a reduced-precision run, checked in two parts.

    (1) The device's reduction of its own per-sample values equals the
    oracle's reduction of the same values (oracle.gpc_stats / mc_stats) to
    1e-12: every moment and every gPC coefficient, so the projection itself
    is pinned at FP64 whatever the solve's rounding.
    (2) Against the oracle's own solve (ref = oracle.run_problem output for
    the same QoI), the statistics may differ only by what the per-sample
    errors e_j = M_gpu,j - M_ref,j allow, output by output, with
    E = sum_j a_j e_j^2 (weights a_j; 1/(N-1) and 1/N for Monte Carlo):
      mean:                 |d mean| <= sqrt(E)        (Cauchy-Schwarz)
      k >= 1 coefficients:  ||d c_k>=1|| <= sqrt(E)    (Bessel: the basis is
                            orthonormal under the rule's discrete measure)
      variance:             |d var| <= 2 sigma sqrt(E) + E
    and the per-sample values must meet the bar themselves: rel. L2 < tol.
    (A relative bar on the variance alone would amplify the solve's
    rounding by 2 |mean| / sigma, 44x for a drag of 22 +- 1.)"""
    import oracle as O

    gpu = np.asarray(gpu_samples, dtype=np.float64)
    S = gpu.shape[0]
    gpu = gpu.reshape(S, -1)
    refM = np.asarray(ref["samples_q"], dtype=np.float64).reshape(S, -1)
    assert rel_l2(gpu, refM) < tol, (label, "samples", rel_l2(gpu, refM))
    if "phi" in ref:
        own = O.gpc_stats(gpu, ref["a"], ref["phi"])
        w = np.asarray(ref["a"], dtype=np.float64)
    else:
        own = O.mc_stats(gpu)
        w = np.full(S, 1.0 / max(S - 1, 1))
    for k in own:
        assert rel_l2(st[k], own[k]) < 1e-12, (label, "reduction", k, rel_l2(st[k], own[k]))
    rs = ref["stats_q"]
    e = gpu - refM
    E = (w[:, None] * e * e).sum(axis=0)
    slack = 1 + 1e-9
    dm = np.abs(np.asarray(st["mean"]) - rs["mean"])
    assert np.all(dm <= np.sqrt(E) * slack + 1e-300), (label, "mean", dm.max())
    sig = np.sqrt(np.maximum(rs["var"], 0.0))
    dv = np.abs(np.asarray(st["var"]) - rs["var"])
    assert np.all(dv <= (2 * sig * np.sqrt(E) + E) * slack + 1e-300), (label, "var", dv.max())
    if "coeffs" in rs and np.asarray(rs["coeffs"]).shape[0] > 1:
        dc = np.sqrt(((np.asarray(st["coeffs"])[1:] - rs["coeffs"][1:]) ** 2).sum(axis=0))
        assert np.all(dc <= np.sqrt(E) * slack + 1e-300), (label, "coeffs_k>=1", dc.max())
