"""MI355X-native weighted mean curvature (Gong & Goksel, arXiv 1903.07189).

The hot path -- the Half Laplace Operator (Sec. 4.2) and the WMC-driven
Jacobi iterations (Sec. 3.5, Sec. 5.2) -- runs in hand-written HIP kernels for
gfx950 behind the C ABI of include/wmc.h (libwmc.so).  This package is the
thin Python binding of that ABI; see :mod:`paper_1903_07189_amd.wmc`.
"""
from . import nn
from .wmc import (WMCError, WMCKernelLayer, WMCSolve, WMCSolve3, SolveBatchedPlan, SolvePlan,
                  autotune, backward, backward3, bw_probe, compute, compute3, fd_compute, fd_flow,
                  layer_backward, layer_forward, lib, release, selftest, shape_of, solve, solve3,
                  solve_batched, solve_l1, solve_noalloc, solve_tuning, step, step3)

__all__ = ["WMCError", "WMCKernelLayer", "WMCSolve", "WMCSolve3", "SolveBatchedPlan", "SolvePlan",
           "autotune", "backward", "backward3", "bw_probe", "compute", "compute3", "fd_compute",
           "fd_flow", "layer_backward", "layer_forward", "lib", "nn", "release", "selftest", "shape_of",
           "solve", "solve3", "solve_batched", "solve_l1", "solve_noalloc", "solve_tuning", "step",
           "step3"]
