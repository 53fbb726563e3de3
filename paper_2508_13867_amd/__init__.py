"""MI355X-native batched lattice-Boltzmann uncertainty quantification.

The HIP library libuqlbm.so (C-ABI in include/uq.h) runs the whole hot path:
an ensemble of D2Q9 BGK solves, one per sample of the uncertain inputs,
advanced together on the GPU, then Monte Carlo or stochastic-collocation gPC
statistics in compensated FP64 (OpenLB-UQ, arXiv 2508.13867). This package is
the thin Python binding.
"""
from ._abi import (QOI, Job, Server, UQError, autotune, lib, make_problem, rule_points,  # noqa: F401
                   tgv_units, wasserstein1)
from . import workloads  # noqa: F401
