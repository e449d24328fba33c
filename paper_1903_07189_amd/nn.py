"""Neural-network form of the half-window operator (Sec. 4.3, Sec. 5.5).

:class:`HalfWindowLayer` is eq. (conv) with K learnable 3x3 kernels followed
by the minimum-magnitude activation of eq. (act); forward and backward run in
libwmc (wmc_layer_forward / wmc_layer_backward).  :class:`HalfWindowNet`
stacks T such layers into the unrolled solver of eq. (exp_model): layer t
updates U <- U + a_t (f - U) + b_t Hhat_t(U) with its own kernels and
learnable step scalars.  The per-layer scalars and the update are ordinary
tensor arithmetic; the operator is the HIP kernel.
"""
from __future__ import annotations

import torch

from .wmc import WMCKernelLayer

# The eight half-window kernels of Sec. 4.2 times 12, [i][row][col], row 0 is
# the image row above the pixel, col 0 the column to its left.
PRINTED_KERNELS_X12 = (
    ((2, 2, 0), (4, -12, 0), (2, 2, 0)),   # left half window
    ((2, 4, 2), (2, -12, 2), (0, 0, 0)),   # top
    ((0, 2, 2), (0, -12, 4), (0, 2, 2)),   # right
    ((0, 0, 0), (2, -12, 2), (2, 4, 2)),   # bottom
    ((2, 4, 1), (4, -12, 0), (1, 0, 0)),   # top-left
    ((1, 4, 2), (0, -12, 4), (0, 0, 1)),   # top-right
    ((0, 0, 1), (0, -12, 4), (1, 4, 2)),   # bottom-right
    ((1, 0, 0), (4, -12, 0), (2, 4, 1)),   # bottom-left
)


def printed_kernels(dtype=torch.float32, device=None) -> torch.Tensor:
    """The eight printed half-window kernels h_1..h_8 (centre weight -1)."""
    return torch.tensor(PRINTED_KERNELS_X12, dtype=dtype, device=device) / 12.0


class HalfWindowLayer(torch.nn.Module):
    """K learnable 3x3 kernels and the minimum-magnitude activation.

    init="half_laplace": the first min(K, 8) kernels are the printed ones
    (so K = 8 starts as the Half Laplace Operator), further kernels are
    printed ones plus small N(0, 0.05^2) noise; init="random":
    N(0, 0.3^2) weights with each kernel's centre set so the kernel sums to 0.
    """

    def __init__(self, K: int = 8, init: str = "half_laplace", generator=None, device=None):
        super().__init__()
        if not 1 <= K <= 16:
            raise ValueError("1 <= K <= 16")
        base = printed_kernels(device=device)
        if init == "half_laplace":
            w = base[torch.arange(K) % 8].clone()
            if K > 8:
                w[8:] += 0.05 * torch.randn((K - 8, 3, 3), generator=generator).to(w.device)
        elif init == "random":
            w = 0.3 * torch.randn((K, 3, 3), generator=generator).to(base.device)
            w[:, 1, 1] -= w.sum(dim=(1, 2))
        else:
            raise ValueError("init must be 'half_laplace' or 'random'")
        self.weight = torch.nn.Parameter(w)

    def forward(self, u: torch.Tensor) -> torch.Tensor:
        return WMCKernelLayer.apply(u, self.weight)


class HalfWindowNet(torch.nn.Module):
    """T unrolled updates U <- U + a_t (f - U) + b_t Hhat_t(U), U^0 = f, each
    with its own learnable kernels (the network of Sec. 5.5 for eq.
    (exp_model)).  a_t, b_t start at the plain iteration's 1/(1+lam) and
    lam/(1+lam)."""

    def __init__(self, layers: int = 2, K: int = 8, lam: float = 5.0, init: str = "half_laplace",
                 generator=None, device=None):
        super().__init__()
        self.ops = torch.nn.ModuleList(
            [HalfWindowLayer(K, init, generator, device) for _ in range(layers)])
        a0 = 1.0 / (1.0 + lam)
        self.a = torch.nn.Parameter(torch.full((layers,), a0, device=device))
        self.b = torch.nn.Parameter(torch.full((layers,), lam * a0, device=device))

    def forward(self, f: torch.Tensor) -> torch.Tensor:
        u = f
        for t, op in enumerate(self.ops):
            u = u + self.a[t] * (f - u) + self.b[t] * op(u)
        return u
