"""FP64 CPU oracle for the discrete weighted mean curvature and its iterations.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU baseline
leg of the benchmark may import this package; the product library and its
Python binding never do.  It shares no code with the HIP implementation: the
arithmetic lives in ``wmc_oracle.c`` (plain C, FP64, single threaded) and this
module only marshals numpy arrays through ctypes.

What each function computes follows the paper (Gong & Goksel, "Weighted Mean
Curvature", arXiv 1903.07189):

* :func:`compute`   -- Sec. 4.2, eqs. (conv) and (act): eight half-window
  responses, minimum-magnitude selection (first index on ties), replicate
  (Neumann) border.
* :func:`step` / :func:`solve` -- Sec. 3.5 eq. (MCF) (``f is None``) and the
  gradient-descent iteration of Sec. 5.2 with A = I (data mode).
* :func:`energy_wmc` / :func:`energy_area` -- eq. (wmcr) with q = 1 and
  eq. (areaReg), each plus the quadratic data term.
* :func:`l1_step` / :func:`l1_solve` -- the l1-fidelity primal-dual
  iteration of Sec. 5.3 (A = I).
* :func:`fd_compute` / :func:`fd_flow` -- the conventional finite-difference
  discretisation of eq. (rhs) and its curvature flow (Sec. 5.4 comparator).
* :func:`layer_forward` / :func:`layer_backward` -- the learnable half-window
  layer of Sec. 4.3 (K learned 3x3 kernels, minimum-magnitude activation) and
  its derivative with the selection held fixed.
* :func:`kernels3` / :func:`compute3` / :func:`solve3` -- the 3-D extension
  mentioned in the conclusion, built like Sec. 4.1 builds the 2-D kernels
  (18 half windows of the tensor-product Laplacian, see O13).
* :func:`listing` -- the Appendix A function's semantics (zero padding, true
  convolution, its candidate order).
* :func:`step_adjoint` / :func:`solve_adjoint` -- derivative of the update map
  with the selection held fixed (the paper leaves this gradient open).

Where the paper is silent the readings are: correlation with the printed
kernels, first index in printed order on exact ties, replicate border,
default step delta = 1/(1+lam) (data) or 1 (MCF), U^0 = f.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wmc_oracle.c")
_LIB = os.path.join(_HERE, "libwmc_oracle.so")

GCC_CMD = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c99", "-fPIC", "-shared",
           _SRC, "-o", _LIB, "-lm"]


def build() -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no FMA contraction)."""
    subprocess.run(GCC_CMD, check=True)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        # WMC_ORACLE_LIB: another build of wmc_oracle.c (e.g. with sanitizers)
        path = os.environ.get("WMC_ORACLE_LIB")
        if not path:
            path = _LIB
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        I = ctypes.c_int
        lib.wmco_kernel_table.argtypes = [P]
        lib.wmco_candidates.argtypes = [P, I64, I64, P]
        lib.wmco_compute.argtypes = [P, I64, I64, P, P]
        lib.wmco_step.argtypes = [P, P, I64, I64, D, D, P, P, P]
        lib.wmco_solve.argtypes = [P, P, I64, I64, D, D, I, P, P]
        lib.wmco_energy_wmc.argtypes = [P, P, I64, I64, D]
        lib.wmco_energy_wmc.restype = D
        lib.wmco_energy_area.argtypes = [P, P, I64, I64, D]
        lib.wmco_energy_area.restype = D
        lib.wmco_listing_kernels.argtypes = [P]
        lib.wmco_listing.argtypes = [P, I64, I64, P, P]
        lib.wmco_step_adjoint.argtypes = [P, P, I64, I64, D, D, I, P, P, P, P, P]
        lib.wmco_solve_adjoint.argtypes = [P, P, I64, I64, D, D, I, I, P, P, P, P, P, P]
        lib.wmco_l1_step.argtypes = [P, P, P, I64, I64, D, D, D, P, P, P, P]
        lib.wmco_l1_solve.argtypes = [P, P, P, I64, I64, D, D, D, I, P, P]
        lib.wmco_fd_compute.argtypes = [P, I64, I64, D, P]
        lib.wmco_fd_flow.argtypes = [P, I64, I64, D, D, I, P]
        lib.wmco_layer_forward.argtypes = [P, I64, I64, I, P, P, P]
        lib.wmco_layer_backward.argtypes = [P, I64, I64, I, P, P, P, P, P]
        lib.wmco3_kernels.argtypes = [P]
        lib.wmco3_compute.argtypes = [P, I64, I64, I64, P, P]
        lib.wmco3_solve.argtypes = [P, P, I64, I64, I64, D, D, I, P]
        lib.wmco3_step.argtypes = [P, P, I64, I64, I64, D, D, P, P, P]
        lib.wmco3_step_adjoint.argtypes = [P, P, I64, I64, I64, D, D, I, P, P, P, P, P]
        lib.wmco3_solve_adjoint.argtypes = [P, P, I64, I64, I64, D, D, I, I, P, P, P, P, P, P]
        _lib = lib
    return _lib


def _d(a):
    """C-contiguous float64 copy/view of a 2-D array."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 2:
        raise ValueError("oracle functions take one 2-D plane")
    return a


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _m8(m, shape):
    if m is None:
        return None
    m = np.ascontiguousarray(m, dtype=np.int8)
    if m.shape != shape:
        raise ValueError("selection map shape mismatch")
    return m


def default_delta(lam: float, mcf: bool) -> float:
    """Step size when none is given: 1 for MCF, 1/(1+lam) with a data term."""
    return 1.0 if mcf else 1.0 / (1.0 + lam)


def kernel_table() -> np.ndarray:
    """The eight printed kernels times 12, shape (8, 3, 3), int."""
    out = np.zeros((8, 3, 3), dtype=np.int32)
    _load().wmco_kernel_table(_p(out))
    return out


def candidates(U) -> np.ndarray:
    """All eight responses S_i = 12 d_i, shape (H, W, 8)."""
    U = _d(U)
    H, W = U.shape
    S = np.empty((H, W, 8), dtype=np.float64)
    _load().wmco_candidates(_p(U), H, W, _p(S))
    return S


def compute(U, return_argmin: bool = False):
    """H_d(U) (Sec. 4.2); optionally the 0-based selection map."""
    U = _d(U)
    H, W = U.shape
    Hd = np.empty_like(U)
    m = np.empty((H, W), dtype=np.int8)
    _load().wmco_compute(_p(U), H, W, _p(Hd), _p(m))
    return (Hd, m) if return_argmin else Hd


def step(U, f=None, lam: float = 1.0, delta: float | None = None, m_forced=None,
         return_argmin: bool = False):
    """One Jacobi update; f=None is MCF mode.  m_forced replays a selection
    (entries < 0 fall back to the minimum rule)."""
    U = _d(U)
    H, W = U.shape
    f = None if f is None else _d(f)
    if delta is None:
        delta = default_delta(lam, f is None)
    mf = _m8(m_forced, (H, W))
    out = np.empty_like(U)
    m = np.empty((H, W), dtype=np.int8)
    _load().wmco_step(_p(U), _p(f), H, W, float(lam), float(delta), _p(mf), _p(out), _p(m))
    return (out, m) if return_argmin else out


def solve(f=None, lam: float = 1.0, iters: int = 1, delta: float | None = None, u0=None,
          m_forced_all=None):
    """iters Jacobi updates from u0 (default f).  f=None is MCF from u0."""
    if f is None and u0 is None:
        raise ValueError("MCF mode needs u0")
    f = None if f is None else _d(f)
    u0 = None if u0 is None else _d(u0)
    ref = f if f is not None else u0
    H, W = ref.shape
    if delta is None:
        delta = default_delta(lam, f is None)
    mf = None
    if m_forced_all is not None:
        mf = np.ascontiguousarray(m_forced_all, dtype=np.int8)
        if mf.shape != (iters, H, W):
            raise ValueError("m_forced_all must be (iters, H, W)")
    out = np.empty((H, W), dtype=np.float64)
    _load().wmco_solve(_p(f), _p(u0), H, W, float(lam), float(delta), int(iters), _p(mf), _p(out))
    return out


def energy_wmc(U, f=None, lam: float = 1.0) -> float:
    U = _d(U)
    f = None if f is None else _d(f)
    return float(_load().wmco_energy_wmc(_p(U), _p(f), U.shape[0], U.shape[1], float(lam)))


def energy_area(U, f=None, lam: float = 1.0) -> float:
    U = _d(U)
    f = None if f is None else _d(f)
    return float(_load().wmco_energy_area(_p(U), _p(f), U.shape[0], U.shape[1], float(lam)))


def listing_kernels() -> np.ndarray:
    out = np.zeros((8, 3, 3), dtype=np.float64)
    _load().wmco_listing_kernels(_p(out))
    return out


def listing(U, return_argmin: bool = False):
    U = _d(U)
    H, W = U.shape
    Hd = np.empty_like(U)
    m = np.empty((H, W), dtype=np.int8)
    _load().wmco_listing(_p(U), H, W, _p(Hd), _p(m))
    return (Hd, m) if return_argmin else Hd


def step_adjoint(U, gbar, f=None, lam: float = 1.0, delta: float | None = None,
                 delta_from_lam: bool | None = None, m_forced=None):
    """Returns (gU, gf, glam) for one step; gf is None in MCF mode."""
    U = _d(U)
    H, W = U.shape
    f = None if f is None else _d(f)
    gbar = _d(gbar)
    if delta is None:
        delta = default_delta(lam, f is None)
        if delta_from_lam is None:
            delta_from_lam = f is not None
    delta_from_lam = bool(delta_from_lam)
    mf = _m8(m_forced, (H, W))
    gU = np.empty_like(U)
    gf = np.zeros_like(U) if f is not None else None
    gl = ctypes.c_double(0.0)
    _load().wmco_step_adjoint(_p(U), _p(f), H, W, float(lam), float(delta), int(delta_from_lam),
                              _p(mf), _p(gbar), _p(gU), _p(gf), ctypes.byref(gl))
    return gU, gf, float(gl.value)


def solve_adjoint(gK, f=None, lam: float = 1.0, K: int = 1, delta: float | None = None,
                  u0=None, delta_from_lam: bool | None = None, m_forced_all=None):
    """Adjoint of a K-step solve.  Returns dict with gu0, gf (data term only),
    glam and UK."""
    if f is None and u0 is None:
        raise ValueError("MCF mode needs u0")
    f = None if f is None else _d(f)
    u0 = None if u0 is None else _d(u0)
    ref = f if f is not None else u0
    H, W = ref.shape
    gK = _d(gK)
    if delta is None:
        delta = default_delta(lam, f is None)
        if delta_from_lam is None:
            delta_from_lam = f is not None
    delta_from_lam = bool(delta_from_lam)
    mf = None
    if m_forced_all is not None:
        mf = np.ascontiguousarray(m_forced_all, dtype=np.int8)
        if mf.shape != (K, H, W):
            raise ValueError("m_forced_all must be (K, H, W)")
    gu0 = np.empty((H, W))
    gf = np.empty((H, W)) if f is not None else None
    UK = np.empty((H, W))
    gl = ctypes.c_double(0.0)
    _load().wmco_solve_adjoint(_p(f), _p(u0), H, W, float(lam), float(delta), int(delta_from_lam),
                               int(K), _p(mf), _p(gK), _p(gu0), _p(gf), ctypes.byref(gl), _p(UK))
    return {"gu0": gu0, "gf": gf, "glam": float(gl.value), "UK": UK}


def near_tie_mask(U, tau: float):
    """Pixels where some candidate of the opposite sign to the selected one
    lies within tau (x12 units) of the minimum magnitude: the set where an
    FP32 evaluation may legitimately select differently (the selection of
    eq. (act) is discontinuous there)."""
    S = candidates(U)
    mag = np.abs(S)
    mn = mag.min(axis=2)
    m = np.argmin(mag, axis=2)
    sel = np.take_along_axis(S, m[..., None], axis=2)[..., 0]
    close = mag <= (mn + tau)[..., None]
    opp = np.sign(S) != np.sign(sel)[..., None]
    return np.any(close & opp, axis=2)


def allowed_values(U, tau: float):
    """For each pixel, the H_d values (S_i/12) of every candidate within tau
    (x12 units) of the minimum magnitude, as an (H, W, 8) array with NaN for
    candidates that are not allowed."""
    S = candidates(U)
    mag = np.abs(S)
    mn = mag.min(axis=2)
    ok = mag <= (mn + tau)[..., None]
    return np.where(ok, S / 12.0, np.nan)


def step_window(U, f, y: int, x: int, k: int, lam: float = 1.0, delta: float | None = None):
    """U^{t+k}(y, x) computed from U^t alone, one sample at a time: the
    in-image (2k+1)^2 neighbourhood is iterated k times with the oracle's
    own replicate border.  Where the window is cut by the image border the
    border rule is the true one; elsewhere the cut is >= k pixels away from
    (y, x), so the sample is exact.  f=None is MCF mode."""
    U = np.asarray(U)
    H, W = U.shape
    y0, y1 = max(0, y - k), min(H, y + k + 1)
    x0, x1 = max(0, x - k), min(W, x + k + 1)
    u = _d(U[y0:y1, x0:x1])
    ff = None if f is None else _d(np.asarray(f)[y0:y1, x0:x1])
    if delta is None:
        delta = default_delta(lam, f is None)
    for _ in range(k):
        u = step(u, ff, lam, delta)
    return float(u[y - y0, x - x0])


def l1_default_delta(lam: float, alpha: float) -> float:
    """Step for the l1 iteration when none is given: 1/(lam + 2/alpha), the
    largest step for which the update is a convex combination while the dual
    is unclipped."""
    return 1.0 / (lam + 2.0 / alpha)


def l1_step(U, d, f, lam: float = 1.0, alpha: float = 0.05, delta: float | None = None,
            m_forced=None, return_argmin: bool = False):
    """One primal-dual step of Sec. 5.3; returns (U', d').  m_forced replays a
    selection as in :func:`step`."""
    U, d, f = _d(U), _d(d), _d(f)
    H, W = U.shape
    if delta is None:
        delta = l1_default_delta(lam, alpha)
    mf = _m8(m_forced, (H, W))
    uo, do = np.empty_like(U), np.empty_like(U)
    m = np.empty((H, W), dtype=np.int8)
    _load().wmco_l1_step(_p(U), _p(d), _p(f), H, W, float(lam), float(alpha), float(delta),
                         _p(mf), _p(uo), _p(do), _p(m))
    return (uo, do, m) if return_argmin else (uo, do)


def l1_solve(f, lam: float = 1.0, alpha: float = 0.05, iters: int = 1, delta: float | None = None,
             u0=None, d0=None):
    """iters primal-dual steps from (u0 or f, d0 or 0); returns (U, d)."""
    f = _d(f)
    H, W = f.shape
    u0 = None if u0 is None else _d(u0)
    d0 = None if d0 is None else _d(d0)
    if delta is None:
        delta = l1_default_delta(lam, alpha)
    uo, do = np.empty_like(f), np.empty_like(f)
    _load().wmco_l1_solve(_p(f), _p(u0), _p(d0), H, W, float(lam), float(alpha), float(delta),
                          int(iters), _p(uo), _p(do))
    return uo, do


def fd_compute(U, eps: float = 1e-12) -> np.ndarray:
    """Central-difference H^w of eq. (rhs) with the guard eps (see O11)."""
    U = _d(U)
    H, W = U.shape
    out = np.empty_like(U)
    _load().wmco_fd_compute(_p(U), H, W, float(eps), _p(out))
    return out


def fd_flow(u0, delta: float = 0.1, iters: int = 1, eps: float = 1e-12) -> np.ndarray:
    u0 = _d(u0)
    H, W = u0.shape
    out = np.empty_like(u0)
    _load().wmco_fd_flow(_p(u0), H, W, float(delta), float(eps), int(iters), _p(out))
    return out


def layer_forward(U, w, return_argmin: bool = False):
    """Learnable half-window layer (O12): K kernels w (K, 3, 3), min-|.|
    activation.  Returns out (and the 0-based selection)."""
    U = _d(U)
    H, W = U.shape
    w = np.ascontiguousarray(w, dtype=np.float64)
    K = w.shape[0]
    if w.shape != (K, 3, 3) or not (1 <= K <= 127):
        raise ValueError("w must be (K, 3, 3) with 1 <= K <= 127")
    out = np.empty_like(U)
    m = np.empty((H, W), dtype=np.int8)
    _load().wmco_layer_forward(_p(U), H, W, K, _p(w), _p(out), _p(m))
    return (out, m) if return_argmin else out


def layer_backward(U, w, m, g):
    """(gU, gW) of the layer with the selection m held fixed (O12)."""
    U = _d(U)
    H, W = U.shape
    w = np.ascontiguousarray(w, dtype=np.float64)
    K = w.shape[0]
    m = np.ascontiguousarray(m, dtype=np.int8)
    g = _d(g)
    gU = np.empty_like(U)
    gW = np.empty((K, 3, 3))
    _load().wmco_layer_backward(_p(U), H, W, K, _p(w), _p(m), _p(g), _p(gU), _p(gW))
    return gU, gW


def _d3(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 3:
        raise ValueError("3-D functions take one (D, H, W) volume")
    return a


def kernels3() -> np.ndarray:
    """The 18 half-window kernels of the 3-D extension, x56, shape (18, 3, 3, 3)
    indexed [i][dz+1][dy+1][dx+1] (O13)."""
    out = np.empty(18 * 27, dtype=np.int32)
    _load().wmco3_kernels(out.ctypes.data_as(ctypes.c_void_p))
    return out.reshape(18, 3, 3, 3)


def compute3(U, return_argmin: bool = False):
    U = _d3(U)
    D, H, W = U.shape
    Hd = np.empty_like(U)
    m = np.empty(U.shape, dtype=np.int8)
    _load().wmco3_compute(_p(U), D, H, W, _p(Hd), _p(m))
    return (Hd, m) if return_argmin else Hd


def solve3(f=None, lam: float = 1.0, iters: int = 1, delta: float | None = None, u0=None):
    if f is None and u0 is None:
        raise ValueError("flow mode needs u0")
    f = None if f is None else _d3(f)
    u0 = None if u0 is None else _d3(u0)
    ref = f if f is not None else u0
    D, H, W = ref.shape
    if delta is None:
        delta = default_delta(lam, f is None)
    out = np.empty_like(ref)
    _load().wmco3_solve(_p(f), _p(u0), D, H, W, float(lam), float(delta), int(iters), _p(out))
    return out


def step3(U, f=None, lam: float = 1.0, delta: float | None = None, m_forced=None,
          return_argmin: bool = False):
    """One 3-D Jacobi step (O14 with O13's operator); m_forced replays a
    selection (entries < 0: the first-minimum rule)."""
    U = _d3(U)
    D, H, W = U.shape
    f = None if f is None else _d3(f)
    if delta is None:
        delta = default_delta(lam, f is None)
    mf = None
    if m_forced is not None:
        mf = np.ascontiguousarray(m_forced, dtype=np.int8)
        if mf.shape != U.shape:
            raise ValueError("selection map shape mismatch")
    out = np.empty_like(U)
    m = np.empty(U.shape, dtype=np.int8)
    _load().wmco3_step(_p(U), _p(f), D, H, W, float(lam), float(delta), _p(mf), _p(out), _p(m))
    return (out, m) if return_argmin else out


def step3_adjoint(U, gbar, f=None, lam: float = 1.0, delta: float | None = None,
                  delta_from_lam: bool | None = None, m_forced=None):
    """Adjoint of one 3-D step (O14).  Returns (gU, gf, glam); gf is None in
    flow mode."""
    U = _d3(U)
    D, H, W = U.shape
    f = None if f is None else _d3(f)
    gbar = _d3(gbar)
    if delta is None:
        delta = default_delta(lam, f is None)
        if delta_from_lam is None:
            delta_from_lam = f is not None
    delta_from_lam = bool(delta_from_lam)
    mf = None
    if m_forced is not None:
        mf = np.ascontiguousarray(m_forced, dtype=np.int8)
        if mf.shape != U.shape:
            raise ValueError("selection map shape mismatch")
    gU = np.empty_like(U)
    gf = np.zeros_like(U) if f is not None else None
    gl = ctypes.c_double(0.0)
    _load().wmco3_step_adjoint(_p(U), _p(f), D, H, W, float(lam), float(delta), int(delta_from_lam),
                               _p(mf), _p(gbar), _p(gU), _p(gf), ctypes.byref(gl))
    return gU, gf, float(gl.value)


def solve3_adjoint(gK, f=None, lam: float = 1.0, K: int = 1, delta: float | None = None,
                   u0=None, delta_from_lam: bool | None = None, m_forced_all=None):
    """Adjoint of a K-step 3-D solve (O14).  Returns dict with gu0, gf (data
    term only), glam and UK."""
    if f is None and u0 is None:
        raise ValueError("flow mode needs u0")
    f = None if f is None else _d3(f)
    u0 = None if u0 is None else _d3(u0)
    ref = f if f is not None else u0
    D, H, W = ref.shape
    gK = _d3(gK)
    if delta is None:
        delta = default_delta(lam, f is None)
        if delta_from_lam is None:
            delta_from_lam = f is not None
    delta_from_lam = bool(delta_from_lam)
    mf = None
    if m_forced_all is not None:
        mf = np.ascontiguousarray(m_forced_all, dtype=np.int8)
        if mf.shape != (K, D, H, W):
            raise ValueError("m_forced_all must be (K, D, H, W)")
    gu0 = np.empty((D, H, W))
    gf = np.empty((D, H, W)) if f is not None else None
    UK = np.empty((D, H, W))
    gl = ctypes.c_double(0.0)
    _load().wmco3_solve_adjoint(_p(f), _p(u0), D, H, W, float(lam), float(delta),
                                int(delta_from_lam), int(K), _p(mf), _p(gK), _p(gu0), _p(gf),
                                ctypes.byref(gl), _p(UK))
    return {"gu0": gu0, "gf": gf, "glam": float(gl.value), "UK": UK}
