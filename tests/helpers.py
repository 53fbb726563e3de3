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
