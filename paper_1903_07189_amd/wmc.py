"""ctypes binding of libwmc (include/wmc.h): argument marshalling only.

Every computation runs in the HIP kernels of libwmc.so; this module converts
torch tensors (device memory owned by PyTorch) into the plain pointers, sizes
and stream handle of the C ABI and raises on a non-zero status.  There is no
fallback: if the library is missing or the device is not gfx950 the calls
raise.

Tensors are float32 CUDA tensors shaped (H, W) or (N, H, W) with unit stride
along W; N planes are independent (colour channels or batch items).
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# WMC_LIB names another build of the same library (for instance one whose host
# code is compiled with sanitizers); by default the in-tree libwmc.so.
LIB_PATH = os.environ.get("WMC_LIB") or os.path.join(_HERE, "libwmc.so")

WMC_OK, WMC_EINVAL, WMC_EHIP, WMC_ENOMEM, WMC_EUNSUPPORTED = 0, -1, -2, -3, -4
WMC_OP_SOLVE, WMC_OP_SOLVE_L1, WMC_OP_BACKWARD, WMC_OP_FD_FLOW, WMC_OP_LAYER_BACKWARD = 0, 1, 2, 3, 4


class WMCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libwmc status {code}: {msg}")
        self.code = code


class Shape(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("h", ctypes.c_int64), ("w", ctypes.c_int64),
                ("ld", ctypes.c_int64), ("ps", ctypes.c_int64)]


class Shape3(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int64), ("h", ctypes.c_int64),
                ("w", ctypes.c_int64), ("ld", ctypes.c_int64), ("ss", ctypes.c_int64),
                ("vs", ctypes.c_int64)]


class Image(ctypes.Structure):
    _fields_ = [("u0", ctypes.c_void_p), ("f", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("h", ctypes.c_int64), ("w", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("ps", ctypes.c_int64), ("channels", ctypes.c_int32), ("lam_index", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("cols", ctypes.c_int32), ("tsteps", ctypes.c_int32),
                ("seg_rows", ctypes.c_int32), ("use_graph", ctypes.c_int32)]


_lib = None
EXPORTS = ["wmc_compute", "wmc_step", "wmc_solve_workspace", "wmc_set_stride",
           "wmc_num_checkpoints", "wmc_solve", "wmc_solve_noalloc", "wmc_solve_tuning", "wmc_l1_workspace",
           "wmc_solve_l1", "wmc_fd_compute", "wmc_fd_flow", "wmc_layer_workspace",
           "wmc_layer_forward", "wmc_layer_backward", "wmc_workspace_bytes",
           "wmc3_compute", "wmc3_step", "wmc3_solve_workspace", "wmc3_set_stride", "wmc3_solve",
           "wmc3_backward_workspace", "wmc3_backward",
           "wmc_batched_workspace", "wmc_solve_batched", "wmc_autotune", "wmc_backward_workspace",
           "wmc_backward", "wmc_bw_probe", "wmc_selftest", "wmc_last_error", "wmc_release"]


def lib():
    """Loads libwmc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                           "(or python paper_1903_07189_amd/_build.py) first")
    L = ctypes.CDLL(LIB_PATH)
    P, I, I64, F, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_float, ctypes.c_size_t
    L.wmc_compute.argtypes = [P, P, Shape, P]
    L.wmc_step.argtypes = [P, P, P, P, F, P, Shape, P]
    L.wmc_solve_workspace.argtypes = [Shape]
    L.wmc_solve_workspace.restype = SZ
    L.wmc_set_stride.argtypes = [Shape]
    L.wmc_set_stride.restype = I64
    L.wmc_num_checkpoints.argtypes = [I, I]
    L.wmc_num_checkpoints.restype = I64
    L.wmc_solve.argtypes = [P, P, P, P, I, F, P, I, ctypes.POINTER(Tuning), P, SZ, Shape, P]
    L.wmc_solve_noalloc.argtypes = [P, P, P, P, I, F, ctypes.POINTER(Tuning), Shape, P]
    L.wmc_solve_tuning.argtypes = [P, P, P, F, P, SZ, Shape, ctypes.POINTER(Tuning), P]
    L.wmc_l1_workspace.argtypes = [Shape]
    L.wmc_l1_workspace.restype = SZ
    L.wmc_solve_l1.argtypes = [P, P, P, P, P, P, F, I, F, ctypes.POINTER(Tuning), P, SZ, Shape, P]
    L.wmc_fd_compute.argtypes = [P, P, F, Shape, P]
    L.wmc_fd_flow.argtypes = [P, P, I, F, F, P, SZ, Shape, P]
    L.wmc3_compute.argtypes = [P, P, Shape3, P]
    L.wmc3_step.argtypes = [P, P, P, P, F, P, Shape3, P]
    L.wmc3_solve_workspace.argtypes = [Shape3]
    L.wmc3_solve_workspace.restype = SZ
    L.wmc3_set_stride.argtypes = [Shape3]
    L.wmc3_set_stride.restype = I64
    L.wmc3_solve.argtypes = [P, P, P, P, I, F, P, I, P, SZ, Shape3, P]
    L.wmc3_backward_workspace.argtypes = [Shape3, I, I]
    L.wmc3_backward_workspace.restype = SZ
    L.wmc3_backward.argtypes = [P, P, P, I, F, P, I, P, P, P, P, P, SZ, Shape3, P]
    L.wmc_workspace_bytes.argtypes = [I, Shape, I, I]
    L.wmc_workspace_bytes.restype = SZ
    L.wmc_layer_workspace.argtypes = [Shape, I]
    L.wmc_layer_workspace.restype = SZ
    L.wmc_layer_forward.argtypes = [P, P, I, P, P, Shape, P]
    L.wmc_layer_backward.argtypes = [P, P, I, P, P, P, P, P, SZ, Shape, P]
    L.wmc_batched_workspace.argtypes = [ctypes.POINTER(Image), I]
    L.wmc_batched_workspace.restype = SZ
    L.wmc_solve_batched.argtypes = [ctypes.POINTER(Image), I, P, I, F, ctypes.POINTER(Tuning), P,
                                    SZ, P]
    L.wmc_autotune.argtypes = [ctypes.POINTER(Image), I, I, ctypes.POINTER(Tuning), P, SZ, P]
    L.wmc_backward_workspace.argtypes = [Shape, I, I]
    L.wmc_backward_workspace.restype = SZ
    L.wmc_backward.argtypes = [P, P, P, I, F, P, I, P, P, P, P, P, SZ, Shape, P]
    L.wmc_bw_probe.argtypes = [I, P, P, P, I64, I, P]
    L.wmc_selftest.argtypes = []
    L.wmc_last_error.argtypes = []
    L.wmc_last_error.restype = ctypes.c_char_p
    L.wmc_release.argtypes = []
    L.wmc_release.restype = None
    for name in ("wmc_compute", "wmc_step", "wmc_solve", "wmc_solve_noalloc", "wmc_solve_tuning",
                 "wmc_solve_l1",
                 "wmc_fd_compute", "wmc_fd_flow", "wmc_layer_forward", "wmc_layer_backward",
                 "wmc3_compute", "wmc3_step", "wmc3_solve", "wmc3_backward",
                 "wmc_solve_batched",
                 "wmc_autotune",
                 "wmc_backward", "wmc_bw_probe", "wmc_selftest"):
        getattr(L, name).restype = I
    _lib = L
    return L


def check(code: int):
    if code != WMC_OK:
        raise WMCError(code, lib().wmc_last_error().decode(errors="replace"))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _planes(t: torch.Tensor) -> torch.Tensor:
    if t.dim() == 2:
        t = t.unsqueeze(0)
    if t.dim() != 3:
        raise ValueError("expected an (H, W) or (N, H, W) tensor")
    if t.dtype != torch.float32 or not t.is_cuda:
        raise TypeError("expected a float32 CUDA tensor")
    if t.stride(2) != 1:
        t = t.contiguous()
    return t


def shape_of(t: torch.Tensor) -> Shape:
    t = _planes(t)
    n, h, w = t.shape
    return Shape(n, h, w, t.stride(1), t.stride(0) if n > 1 else h * t.stride(1))


def require_shape(t: torch.Tensor | None, want, name: str) -> None:
    """Raises ValueError unless t (if given) has exactly the shape `want`.
    Every array passed with one wmc_shape must cover that shape: a tensor with
    fewer planes or rows would be read past its end by the kernels."""
    if t is not None and tuple(t.shape) != tuple(want):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(want)}")


def checkpoint_sets(iters: int, ckpt_every: int) -> int:
    """Plane sets a solve(..., ckpt_every=c) of iters steps returns (at least one)."""
    if int(ckpt_every) < 1:
        raise ValueError("ckpt_every must be >= 1")
    return max(1, int(lib().wmc_num_checkpoints(int(iters), int(ckpt_every))))


def _like(t: torch.Tensor) -> torch.Tensor:
    """Uninitialised tensor with exactly t's strides (the ABI shares one layout)."""
    return torch.empty_strided(t.shape, t.stride(), dtype=t.dtype, device=t.device)


def _lam_tensor(lam, n: int, device) -> torch.Tensor:
    if isinstance(lam, torch.Tensor):
        lt = lam.detach().to(device=device, dtype=torch.float32).reshape(-1)
        if lt.numel() == 1 and n > 1:
            lt = lt.expand(n)
        if lt.numel() != n:
            raise ValueError(f"lam must hold 1 or {n} values")
        return lt.contiguous()
    return torch.full((n,), float(lam), dtype=torch.float32, device=device)


def _tuning(tuning) -> Tuning | None:
    if tuning is None:
        return None
    if isinstance(tuning, Tuning):
        return tuning
    d = dict(tuning)
    return Tuning(int(d.get("cols", 0)), int(d.get("tsteps", 0)), int(d.get("seg_rows", 0)),
                  int(d.get("use_graph", 1)))


def compute(u: torch.Tensor) -> torch.Tensor:
    """H_d(u): the Half Laplace Operator (Sec. 4.2)."""
    squeeze = u.dim() == 2
    u = _planes(u)
    out = _like(u)
    check(lib().wmc_compute(_ptr(u), _ptr(out), shape_of(u), _stream()))
    return out[0] if squeeze else out


def step(u: torch.Tensor, f: torch.Tensor | None = None, lam=1.0, dt: float = 0.0,
         return_argmin: bool = False):
    """One Jacobi update (data term if f is given, curvature flow otherwise)."""
    squeeze = u.dim() == 2
    u = _planes(u)
    if f is not None:
        f = _planes(f)
        require_shape(f, u.shape, "f")
        if f.stride() != u.stride():
            f = f.contiguous() if u.is_contiguous() else f
            if f.stride() != u.stride():
                raise ValueError("u and f must share shape and layout")
    out = _like(u)
    lt = _lam_tensor(lam, u.shape[0], u.device) if f is not None else None
    amap = torch.empty(u.shape, dtype=torch.uint8, device=u.device) if return_argmin else None
    if amap is not None and (u.stride() != amap.stride()):
        raise ValueError("argmin output needs a contiguous input")
    check(lib().wmc_step(_ptr(u), _ptr(f), _ptr(out), _ptr(lt), float(dt), _ptr(amap),
                         shape_of(u), _stream()))
    if squeeze:
        out = out[0]
        amap = amap[0] if amap is not None else None
    return (out, amap) if return_argmin else out


def solve(f: torch.Tensor | None, lam=1.0, iters: int = 1, dt: float = 0.0,
          u0: torch.Tensor | None = None, ckpt_every: int | None = None, tuning=None):
    """iters Jacobi updates from u0 (default f).  With ckpt_every also returns
    the checkpoint tensor (num_ckpt, N, H, W) that backward() restarts from."""
    ref = f if f is not None else u0
    if ref is None:
        raise ValueError("need f or u0")
    squeeze = ref.dim() == 2
    ref = _planes(ref).contiguous()
    f = None if f is None else _planes(f).contiguous()
    u0 = None if u0 is None else _planes(u0).contiguous()
    require_shape(u0, ref.shape, "u0")
    s = shape_of(ref)
    L = lib()
    out = torch.empty_like(ref)
    ws = torch.empty(max(1, L.wmc_solve_workspace(s) // 4), dtype=torch.float32, device=ref.device)
    lt = _lam_tensor(lam, ref.shape[0], ref.device) if f is not None else None
    ck = None
    if ckpt_every:
        nck = L.wmc_num_checkpoints(int(iters), int(ckpt_every))
        if L.wmc_set_stride(s) != ref.numel():
            raise ValueError("checkpointing needs a contiguous plane set")
        ck = torch.empty((max(nck, 1),) + tuple(ref.shape), dtype=torch.float32, device=ref.device)
    tn = _tuning(tuning)
    check(L.wmc_solve(_ptr(f), _ptr(u0), _ptr(out), _ptr(lt), int(iters), float(dt), _ptr(ck),
                      int(ckpt_every or 0), ctypes.byref(tn) if tn else None, _ptr(ws),
                      ws.numel() * 4, s, _stream()))
    if squeeze:
        out = out[0]
    return (out, ck) if ckpt_every else out


def solve_noalloc(f: torch.Tensor | None, lam, iters: int, out: torch.Tensor, dt: float = 0.0,
                  u0: torch.Tensor | None = None, tuning=None) -> torch.Tensor:
    """solve() through wmc_solve_noalloc: no workspace and no checkpoints; the
    library keeps the intermediate state in its static device scratch.  The
    caller passes the output tensor `out` (f's shape), so nothing here
    allocates device memory as long as lam is a device tensor of one value per
    plane."""
    ref = f if f is not None else u0
    if ref is None:
        raise ValueError("need f or u0")
    for name, t in (("f", f), ("u0", u0), ("out", out)):
        if t is not None and (t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    require_shape(u0, ref.shape, "u0")
    require_shape(out, ref.shape, "out")
    r3 = ref if ref.dim() == 3 else ref.unsqueeze(0)
    s = shape_of(r3)
    lt = _lam_tensor(lam, r3.shape[0], ref.device) if f is not None else None
    tn = _tuning(tuning)
    check(lib().wmc_solve_noalloc(_ptr(f), _ptr(u0), _ptr(out), _ptr(lt), int(iters), float(dt),
                                  ctypes.byref(tn) if tn else None, s, _stream()))
    return out


def solve_l1(f: torch.Tensor, lam=1.0, alpha: float = 0.05, iters: int = 1, dt: float = 0.0,
             u0: torch.Tensor | None = None, d0: torch.Tensor | None = None, tuning=None):
    """The l1-fidelity primal-dual iteration of Sec. 5.3; returns (U, d)."""
    squeeze = f.dim() == 2
    f = _planes(f).contiguous()
    u0 = None if u0 is None else _planes(u0).contiguous()
    d0 = None if d0 is None else _planes(d0).contiguous()
    require_shape(u0, f.shape, "u0")
    require_shape(d0, f.shape, "d0")
    s = shape_of(f)
    L = lib()
    out, dout = torch.empty_like(f), torch.empty_like(f)
    ws = torch.empty(max(1, L.wmc_l1_workspace(s) // 4), dtype=torch.float32, device=f.device)
    lt = _lam_tensor(lam, f.shape[0], f.device)
    tn = _tuning(tuning)
    check(L.wmc_solve_l1(_ptr(f), _ptr(u0), _ptr(d0), _ptr(out), _ptr(dout), _ptr(lt),
                         float(alpha), int(iters), float(dt), ctypes.byref(tn) if tn else None,
                         _ptr(ws), ws.numel() * 4, s, _stream()))
    if squeeze:
        return out[0], dout[0]
    return out, dout


def fd_compute(u: torch.Tensor, eps: float = 1e-12) -> torch.Tensor:
    """Conventional central-difference H^w of eq. (rhs) (Sec. 5.4 comparator)."""
    squeeze = u.dim() == 2
    u = _planes(u).contiguous()
    out = torch.empty_like(u)
    check(lib().wmc_fd_compute(_ptr(u), _ptr(out), float(eps), shape_of(u), _stream()))
    return out[0] if squeeze else out


def fd_flow(u0: torch.Tensor, iters: int, dt: float = 0.1, eps: float = 1e-12) -> torch.Tensor:
    """iters explicit curvature-flow steps with the conventional discretisation."""
    squeeze = u0.dim() == 2
    u0 = _planes(u0).contiguous()
    s = shape_of(u0)
    L = lib()
    out = torch.empty_like(u0)
    ws = torch.empty(max(1, L.wmc_solve_workspace(s) // 4), dtype=torch.float32, device=u0.device)
    check(L.wmc_fd_flow(_ptr(u0), _ptr(out), int(iters), float(dt), float(eps), _ptr(ws),
                        ws.numel() * 4, s, _stream()))
    return out[0] if squeeze else out


def _weights(w: torch.Tensor) -> torch.Tensor:
    if w.dim() != 3 or tuple(w.shape[1:]) != (3, 3):
        raise ValueError("kernels must be a (K, 3, 3) tensor")
    if not (1 <= w.shape[0] <= 16):
        raise ValueError("1 <= K <= 16 kernels")
    return w.detach().to(dtype=torch.float32).contiguous()


def layer_forward(u: torch.Tensor, w: torch.Tensor):
    """Learnable half-window layer (Sec. 4.3): K kernels w (K, 3, 3), then the
    minimum-magnitude activation.  Returns (out, sel) with sel uint8."""
    squeeze = u.dim() == 2
    u = _planes(u).contiguous()
    wt = _weights(w)
    out = torch.empty_like(u)
    sel = torch.empty(u.shape, dtype=torch.uint8, device=u.device)
    check(lib().wmc_layer_forward(_ptr(u), _ptr(wt), wt.shape[0], _ptr(out), _ptr(sel),
                                  shape_of(u), _stream()))
    return (out[0], sel[0]) if squeeze else (out, sel)


def layer_backward(u: torch.Tensor, w: torch.Tensor, sel: torch.Tensor, g: torch.Tensor,
                   need_u: bool = True, need_w: bool = True):
    """(g_u, g_w) of the layer with the selection held fixed."""
    squeeze = u.dim() == 2
    u = _planes(u).contiguous()
    sel = (sel.unsqueeze(0) if sel.dim() == 2 else sel).contiguous()
    g = _planes(g).contiguous()
    if sel.shape != u.shape or g.shape != u.shape or sel.dtype != torch.uint8:
        raise ValueError("sel (uint8) and g must have u's shape")
    wt = _weights(w)
    K = wt.shape[0]
    s = shape_of(u)
    L = lib()
    g_u = torch.empty_like(u) if need_u else None
    g_w = torch.empty((K, 3, 3), dtype=torch.float32, device=u.device) if need_w else None
    ws = torch.empty(max(1, L.wmc_layer_workspace(s, K) // 4), dtype=torch.float32,
                     device=u.device) if need_w else None
    check(L.wmc_layer_backward(_ptr(u), _ptr(wt), K, _ptr(sel), _ptr(g), _ptr(g_u), _ptr(g_w),
                               _ptr(ws), 0 if ws is None else ws.numel() * 4, s, _stream()))
    if squeeze and g_u is not None:
        g_u = g_u[0]
    return g_u, g_w


class WMCKernelLayer(torch.autograd.Function):
    """out = layer(u; w) as a differentiable op: gradients to u (N, H, W) and to
    the kernels w (K, 3, 3), with the forward's selection held fixed."""

    @staticmethod
    def forward(ctx, u, w):
        out, sel = layer_forward(u.detach(), w)
        ctx.save_for_backward(u.detach(), w.detach(), sel)
        return out

    @staticmethod
    def backward(ctx, g):
        u, w, sel = ctx.saved_tensors
        g_u, g_w = layer_backward(u, w, sel, g.contiguous(), need_u=ctx.needs_input_grad[0],
                                  need_w=ctx.needs_input_grad[1])
        if g_w is not None:
            g_w = g_w.to(w.dtype)
        return g_u, g_w


def _volumes(t: torch.Tensor) -> torch.Tensor:
    if t.dim() == 3:
        t = t.unsqueeze(0)
    if t.dim() != 4:
        raise ValueError("expected a (D, H, W) or (N, D, H, W) tensor")
    if t.dtype != torch.float32 or not t.is_cuda:
        raise TypeError("expected a float32 CUDA tensor")
    return t.contiguous()


def shape3_of(t: torch.Tensor) -> Shape3:
    n, d, h, w = t.shape
    return Shape3(n, d, h, w, t.stride(2), t.stride(1), t.stride(0) if n > 1 else d * t.stride(1))


def compute3(u: torch.Tensor) -> torch.Tensor:
    """3-D half-window operator (18 half windows of the tensor-product
    Laplacian; the extension the conclusion mentions)."""
    squeeze = u.dim() == 3
    u = _volumes(u)
    out = torch.empty_like(u)
    check(lib().wmc3_compute(_ptr(u), _ptr(out), shape3_of(u), _stream()))
    return out[0] if squeeze else out


def step3(u: torch.Tensor, f: torch.Tensor | None = None, lam=1.0, dt: float = 0.0,
          return_argmin: bool = False):
    """One Jacobi update on volumes (f given: data term, else the flow); with
    return_argmin also the selected half window of every voxel (uint8)."""
    squeeze = u.dim() == 3
    u = _volumes(u)
    f = None if f is None else _volumes(f)
    require_shape(f, u.shape, "f")
    out = torch.empty_like(u)
    am = torch.empty(u.shape, dtype=torch.uint8, device=u.device) if return_argmin else None
    lt = _lam_tensor(lam, u.shape[0], u.device) if f is not None else None
    check(lib().wmc3_step(_ptr(u), _ptr(f), _ptr(out), _ptr(lt), float(dt), _ptr(am), shape3_of(u),
                          _stream()))
    if squeeze:
        out = out[0]
        am = None if am is None else am[0]
    return (out, am) if return_argmin else out


def solve3(f: torch.Tensor | None, lam=1.0, iters: int = 1, dt: float = 0.0,
           u0: torch.Tensor | None = None, ckpt_every: int | None = None):
    """iters Jacobi updates of the data (f given) or flow iteration on volumes.
    With ckpt_every also returns the checkpoints (num_ckpt, N, D, H, W) that
    backward3() restarts from."""
    ref = f if f is not None else u0
    if ref is None:
        raise ValueError("need f or u0")
    squeeze = ref.dim() == 3
    ref = _volumes(ref)
    f = None if f is None else _volumes(f)
    u0 = None if u0 is None else _volumes(u0)
    require_shape(u0, ref.shape, "u0")
    require_shape(f, ref.shape, "f")
    s = shape3_of(ref)
    L = lib()
    out = torch.empty_like(ref)
    ws = torch.empty(max(1, L.wmc3_solve_workspace(s) // 4), dtype=torch.float32, device=ref.device)
    lt = _lam_tensor(lam, ref.shape[0], ref.device) if f is not None else None
    ck = None
    if ckpt_every:
        if L.wmc3_set_stride(s) != ref.numel():
            raise ValueError("checkpointing needs a contiguous volume set")
        ck = torch.empty((checkpoint_sets(iters, ckpt_every),) + tuple(ref.shape),
                         dtype=torch.float32, device=ref.device)
    check(L.wmc3_solve(_ptr(f), _ptr(u0), _ptr(out), _ptr(lt), int(iters), float(dt), _ptr(ck),
                       int(ckpt_every or 0), _ptr(ws), ws.numel() * 4, s, _stream()))
    if squeeze:
        out = out[0]
    return (out, ck) if ckpt_every else out


def backward3(g_out: torch.Tensor, f: torch.Tensor | None, lam, iters: int, ckpt: torch.Tensor,
              ckpt_every: int, dt: float = 0.0, u0: torch.Tensor | None = None):
    """Reverse-mode derivative of L(U^iters) through solve3(); returns
    (g_f, g_u0, g_lam) for (N, D, H, W) volumes.  g_f includes the path
    through U^0 = f when u0 is None."""
    ref = f if f is not None else u0
    if ref is None:
        raise ValueError("need f or u0")
    ref = _volumes(ref)
    f = None if f is None else _volumes(f)
    u0 = None if u0 is None else _volumes(u0)
    g_out = _volumes(g_out)
    require_shape(u0, ref.shape, "u0")
    require_shape(g_out, ref.shape, "g_out")
    if ckpt is None:
        raise ValueError("backward3 needs the checkpoints of the forward solve")
    if ckpt.dtype != torch.float32 or not ckpt.is_cuda or not ckpt.is_contiguous():
        raise ValueError("ckpt must be a contiguous float32 CUDA tensor")
    require_shape(ckpt, (checkpoint_sets(iters, ckpt_every),) + tuple(ref.shape), "ckpt")
    s = shape3_of(ref)
    L = lib()
    n = ref.shape[0]
    lt = _lam_tensor(lam, n, ref.device) if f is not None else None
    ws = torch.empty(max(1, L.wmc3_backward_workspace(s, int(iters), int(ckpt_every)) // 4 + 64),
                     dtype=torch.float32, device=ref.device)
    g_f = torch.empty_like(ref) if f is not None else None
    g_u0 = torch.empty_like(ref)
    g_lam = torch.empty(n, dtype=torch.float32, device=ref.device) if f is not None else None
    check(L.wmc3_backward(_ptr(f), _ptr(u0), _ptr(lt), int(iters), float(dt), _ptr(ckpt),
                          int(ckpt_every), _ptr(g_out), _ptr(g_f), _ptr(g_u0), _ptr(g_lam),
                          _ptr(ws), ws.numel() * 4, s, _stream()))
    return g_f, g_u0, g_lam


def solve_tuning(f: torch.Tensor | None, lam=1.0, dt: float = 0.0, u0: torch.Tensor | None = None):
    """The launch shape solve() picks for this input (autotuned, cached)."""
    ref = f if f is not None else u0
    ref = _planes(ref).contiguous()
    f = None if f is None else _planes(f).contiguous()
    u0 = None if u0 is None else _planes(u0).contiguous()
    require_shape(u0, ref.shape, "u0")
    s = shape_of(ref)
    L = lib()
    # two plane sets: the search then ping-pongs between them as the solve does
    ws = torch.empty(max(1, (2 * L.wmc_solve_workspace(s) + 256) // 4), dtype=torch.float32,
                     device=ref.device)
    lt = _lam_tensor(lam, ref.shape[0], ref.device) if f is not None else None
    t = Tuning()
    check(L.wmc_solve_tuning(_ptr(f), _ptr(u0), _ptr(lt), float(dt), _ptr(ws), ws.numel() * 4, s,
                             ctypes.byref(t), _stream()))
    return {"cols": t.cols, "tsteps": t.tsteps, "seg_rows": t.seg_rows, "use_graph": t.use_graph}


class SolvePlan:
    """Pre-marshalled solve() for repeated calls on fixed buffers, so that the
    library replays one cached graph (its cache is keyed by the pointers)."""

    def __init__(self, f: torch.Tensor, lam, iters: int, dt: float = 0.0, tuning=None):
        self.f = _planes(f).contiguous()
        self.s = shape_of(self.f)
        L = lib()
        self.out = torch.empty_like(self.f)
        self.ws = torch.empty(max(1, L.wmc_solve_workspace(self.s) // 4), dtype=torch.float32,
                              device=self.f.device)
        self.lam = _lam_tensor(lam, self.f.shape[0], self.f.device)
        self.iters, self.dt = int(iters), float(dt)
        self.tuning = _tuning(tuning)

    def __call__(self):
        check(lib().wmc_solve(_ptr(self.f), None, _ptr(self.out), _ptr(self.lam), self.iters,
                              self.dt, None, 0, ctypes.byref(self.tuning) if self.tuning else None,
                              _ptr(self.ws), self.ws.numel() * 4, self.s, _stream()))
        return self.out


def backward(g_out: torch.Tensor, f: torch.Tensor | None, lam, iters: int, ckpt: torch.Tensor,
             ckpt_every: int, dt: float = 0.0, u0: torch.Tensor | None = None):
    """Reverse-mode derivative of L(U^iters) through solve(); returns
    (g_f, g_u0, g_lam).  g_f includes the path through U^0 = f when u0 is None."""
    ref = f if f is not None else u0
    if ref is None:
        raise ValueError("need f or u0")
    ref = _planes(ref).contiguous()
    f = None if f is None else _planes(f).contiguous()
    u0 = None if u0 is None else _planes(u0).contiguous()
    g_out = _planes(g_out).contiguous()
    require_shape(u0, ref.shape, "u0")
    require_shape(g_out, ref.shape, "g_out")
    if ckpt is None:
        raise ValueError("backward needs the checkpoints of the forward solve")
    if ckpt.dtype != torch.float32 or not ckpt.is_cuda or not ckpt.is_contiguous():
        raise ValueError("ckpt must be a contiguous float32 CUDA tensor")
    require_shape(ckpt, (checkpoint_sets(iters, ckpt_every),) + tuple(ref.shape), "ckpt")
    s = shape_of(ref)
    L = lib()
    n = ref.shape[0]
    lt = _lam_tensor(lam, n, ref.device) if f is not None else None
    ws = torch.empty(max(1, L.wmc_backward_workspace(s, int(iters), int(ckpt_every)) // 4 + 64),
                     dtype=torch.float32, device=ref.device)
    g_f = torch.empty_like(ref) if f is not None else None
    g_u0 = torch.empty_like(ref)
    g_lam = torch.empty(n, dtype=torch.float32, device=ref.device) if f is not None else None
    check(L.wmc_backward(_ptr(f), _ptr(u0), _ptr(lt), int(iters), float(dt), _ptr(ckpt),
                         int(ckpt_every), _ptr(g_out), _ptr(g_f), _ptr(g_u0), _ptr(g_lam),
                         _ptr(ws), ws.numel() * 4, s, _stream()))
    return g_f, g_u0, g_lam


def _images(fs, u0s, outs, lam_index):
    arr = (Image * len(fs))()
    for i, (f, u0, o) in enumerate(zip(fs, u0s, outs)):
        ref = f if f is not None else u0
        c, h, w = ref.shape
        arr[i] = Image(_ptr(u0), _ptr(f), _ptr(o), h, w, ref.stride(1),
                       ref.stride(0) if c > 1 else h * ref.stride(1), c, lam_index[i])
    return arr


def solve_batched(fs, lam, iters: int, dt: float = 0.0, u0s=None, tuning=None):
    """Solves many (C, H, W) images of different sizes with one launch per
    fused block of sweeps over the work items of all images, graph-replayed.  lam: one value per image (tensor or list)."""
    fs = [None if f is None else _planes(f).contiguous() for f in fs]
    u0s = [None] * len(fs) if u0s is None else [None if u is None else _planes(u).contiguous()
                                                 for u in u0s]
    if len(u0s) != len(fs):
        raise ValueError("u0s must hold one entry per image")
    refs = [f if f is not None else u for f, u in zip(fs, u0s)]
    for i, (f, u) in enumerate(zip(fs, u0s)):
        if f is not None:
            require_shape(u, f.shape, f"u0s[{i}]")
    dev = refs[0].device
    outs = [torch.empty_like(r) for r in refs]
    lt = _lam_tensor(lam, len(fs), dev) if fs[0] is not None else None
    arr = _images(fs, u0s, outs, list(range(len(fs))))
    L = lib()
    wsb = L.wmc_batched_workspace(arr, len(fs))
    ws = torch.empty(max(1, wsb // 4), dtype=torch.float32, device=dev)
    tn = _tuning(tuning)
    check(L.wmc_solve_batched(arr, len(fs), _ptr(lt), int(iters), float(dt),
                              ctypes.byref(tn) if tn else None, _ptr(ws), ws.numel() * 4,
                              _stream()))
    return outs


class SolveBatchedPlan:
    """Pre-marshalled batched solve for repeated calls on the same buffers
    (keeps the descriptor array and workspace alive; the library replays its
    cached graph)."""

    def __init__(self, fs, lam, iters: int, dt: float = 0.0, outs=None, tuning=None):
        self.fs = [_planes(f).contiguous() for f in fs]
        dev = self.fs[0].device
        self.outs = outs if outs is not None else [torch.empty_like(f) for f in self.fs]
        self.lam = _lam_tensor(lam, len(self.fs), dev)
        self.arr = _images(self.fs, [None] * len(self.fs), self.outs, list(range(len(self.fs))))
        L = lib()
        self.ws = torch.empty(max(1, L.wmc_batched_workspace(self.arr, len(self.fs)) // 4),
                              dtype=torch.float32, device=dev)
        self.iters, self.dt = int(iters), float(dt)
        self.tuning = _tuning(tuning)

    def __call__(self):
        check(lib().wmc_solve_batched(self.arr, len(self.fs), _ptr(self.lam), self.iters, self.dt,
                                      ctypes.byref(self.tuning) if self.tuning else None,
                                      _ptr(self.ws), self.ws.numel() * 4, _stream()))
        return self.outs


def autotune(fs, iters: int = 100):
    """Runs the library's autotuner on a batch; returns the chosen tuning dict."""
    fs = [_planes(f).contiguous() for f in fs]
    outs = [torch.empty_like(f) for f in fs]
    arr = _images(fs, [None] * len(fs), outs, [0] * len(fs))
    L = lib()
    ws = torch.empty(max(1, L.wmc_batched_workspace(arr, len(fs)) // 4), dtype=torch.float32,
                     device=fs[0].device)
    t = Tuning()
    check(L.wmc_autotune(arr, len(fs), int(iters), ctypes.byref(t), _ptr(ws), ws.numel() * 4,
                         _stream()))
    return {"cols": t.cols, "tsteps": t.tsteps, "seg_rows": t.seg_rows, "use_graph": t.use_graph}


def bw_probe(a: torch.Tensor, o: torch.Tensor, b: torch.Tensor | None = None,
             nontemporal: bool = False) -> None:
    """Streaming bandwidth probe (measurement aid): o = a, or o = a + b."""
    for t in (a, b, o):
        if t is not None and (t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous()
                              or t.numel() != a.numel()):
            raise ValueError("bw_probe takes contiguous float32 CUDA tensors of one size")
    check(lib().wmc_bw_probe(1 if b is not None else 0, _ptr(a), _ptr(b), _ptr(o), a.numel(),
                             1 if nontemporal else 0, _stream()))


def selftest():
    check(lib().wmc_selftest())


def release():
    lib().wmc_release()


# Keeping every state of the forward (checkpoint period 1) removes the
# backward's recomputation; the fused forward stores them as it goes.  It
# costs K plane sets of memory, so it is the default only up to this size.
KEEP_ALL_STATES_BYTES = 2 << 30


def default_ckpt_every(K: int, plane_set_bytes: int) -> int:
    """1 (keep every state) when K states fit KEEP_ALL_STATES_BYTES, else
    ceil(sqrt(K)) (about 2 sqrt(K) states in memory, one recomputation)."""
    K = max(int(K), 1)
    if K * int(plane_set_bytes) <= KEEP_ALL_STATES_BYTES:
        return 1
    return max(1, math.ceil(math.sqrt(K)))


class WMCSolve3(torch.autograd.Function):
    """U^K = solve3(f, lam, K) on (N, D, H, W) volumes as a differentiable
    layer: the forward stores a checkpoint every ckpt_every steps (default
    default_ckpt_every), the backward runs the hand-written 3-D adjoint.
    Gradients flow to f and to lam (N,)."""

    @staticmethod
    def forward(ctx, f, lam, K: int, dt: float = 0.0, ckpt_every: int | None = None):
        K = int(K)
        c = int(ckpt_every) if ckpt_every else default_ckpt_every(K, f.numel() * 4)
        fv = _volumes(f.detach())
        lam_t = _lam_tensor(lam, fv.shape[0], f.device)
        out, ck = solve3(fv, lam_t, K, dt=dt, ckpt_every=c)
        ctx.save_for_backward(fv, lam_t, ck)
        ctx.K, ctx.c, ctx.dt = K, c, float(dt)
        ctx.f_shape = tuple(f.shape)
        ctx.lam_is_tensor = isinstance(lam, torch.Tensor)
        ctx.lam_shape = tuple(lam.shape) if ctx.lam_is_tensor else None
        ctx.lam_numel = lam.numel() if ctx.lam_is_tensor else 0
        return out.reshape(f.shape)

    @staticmethod
    def backward(ctx, g):
        f, lam_t, ck = ctx.saved_tensors
        g_f, _, g_lam = backward3(g.reshape(f.shape).contiguous(), f, lam_t, ctx.K, ck, ctx.c,
                                  dt=ctx.dt)
        gl = None
        if ctx.lam_is_tensor:
            gl = g_lam.reshape(ctx.lam_shape) if ctx.lam_numel == g_lam.numel() else \
                g_lam.sum().reshape(ctx.lam_shape)
        return g_f.reshape(ctx.f_shape), gl, None, None, None


class WMCSolve(torch.autograd.Function):
    """U^K = solve(f, lam, K) as a differentiable layer: forward runs the fused
    solver storing a checkpoint every ckpt_every steps (default
    default_ckpt_every), backward runs the hand-written adjoint, recomputing
    each segment from its checkpoint.  Gradients flow to f (N, H, W) and to
    lam (N,)."""

    @staticmethod
    def forward(ctx, f, lam, K: int, dt: float = 0.0, ckpt_every: int | None = None, tuning=None):
        K = int(K)
        c = int(ckpt_every) if ckpt_every else default_ckpt_every(K, f.numel() * 4)
        lam_t = _lam_tensor(lam, _planes(f).shape[0], f.device)
        out, ck = solve(f.detach(), lam_t, K, dt=dt, ckpt_every=c, tuning=tuning)
        ctx.save_for_backward(f.detach(), lam_t, ck)
        ctx.K, ctx.c, ctx.dt = K, c, float(dt)
        ctx.lam_is_tensor = isinstance(lam, torch.Tensor)
        ctx.lam_shape = tuple(lam.shape) if ctx.lam_is_tensor else None
        ctx.lam_numel = lam.numel() if ctx.lam_is_tensor else 0
        return out

    @staticmethod
    def backward(ctx, g):
        f, lam_t, ck = ctx.saved_tensors
        g_f, _, g_lam = backward(g.contiguous(), f, lam_t, ctx.K, ck, ctx.c, dt=ctx.dt)
        g_f = g_f.reshape(f.shape)
        gl = None
        if ctx.lam_is_tensor:
            gl = g_lam.reshape(ctx.lam_shape) if ctx.lam_numel == g_lam.numel() else \
                g_lam.sum().reshape(ctx.lam_shape)
        return g_f, gl, None, None, None, None
