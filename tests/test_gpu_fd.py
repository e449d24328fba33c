"""The conventional finite-difference WMC of eq. (rhs) -- the comparator of
the curvature-flow study in Sec. 5.4 -- on the GPU against the oracle, and the
study itself on the GPU kernels.

Tolerances: both sides take the same FP32 inputs; the GPU evaluates the
stencil in FP32.  The first differences are single roundings of exact
differences (relative error 2^-24), so the direction of the gradient is
accurate; the second differences carry two roundings, and the normal term
num / (G + eps) is a Rayleigh quotient of the Hessian in the gradient
direction, bounded by its norm (<= 4 for values in [0, 1]).  A few FP32 ulps
of that bound give 2e-5 absolute per evaluation.  Over many flow steps the
iteration amplifies rounding where the gradient is small (measured on the
oracle: a 1e-7 input perturbation grows to 8e-6 max / 4e-8 mean after 20
steps of dt = 0.1), so the multi-step check bounds the max by 2e-4 and the
mean by 2e-6."""
import ctypes
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import wmc_synth

sys.path.insert(0, os.path.dirname(__file__))
from ssim_util import ssim  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 2e-5


@pytest.fixture(scope="module")
def wmc():
    import paper_1903_07189_amd as W
    W.lib()
    return W


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (6, 1), (5, 9), (3, 124), (4, 125), (70, 133),
                                   (130, 248), (257, 300), (1031, 40)])
def test_fd_compute_parity(wmc, shape):
    U = wmc_synth.random_unit(*shape, seed=sum(shape))
    g = wmc.fd_compute(to_gpu(U)).cpu().numpy()
    r = oracle.fd_compute(U)
    assert np.abs(g - r).max() <= TOL


def test_fd_compute_parity_natural_and_flat(wmc):
    noisy, clean = wmc_synth.c1()
    for U in (noisy[0], clean[0], np.full((33, 65), 0.3, np.float32)):
        g = wmc.fd_compute(to_gpu(U)).cpu().numpy()
        assert np.abs(g - oracle.fd_compute(U)).max() <= TOL
    # flat image: gradient 0, guard makes the normal term vanish exactly
    z = wmc.fd_compute(to_gpu(np.full((33, 65), 0.3, np.float32)))
    assert torch.count_nonzero(z).item() == 0


def test_fd_compute_strided_planes(wmc):
    """Three planes with padded rows and planes through the raw ABI; the
    padding is never written."""
    n, h, w, ld = 3, 41, 77, 96
    ps = h * ld + 32
    rng = np.random.default_rng(5)
    base = rng.uniform(0, 1, size=n * ps).astype(np.float32)
    src = to_gpu(base)
    out = torch.full((n * ps,), float("nan"), device="cuda:0")
    from paper_1903_07189_amd import wmc as M
    L = M.lib()
    M.check(L.wmc_fd_compute(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                             1e-12, M.Shape(n, h, w, ld, ps), None))
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    for p in range(n):
        plane = base[p * ps:p * ps + h * ld].reshape(h, ld)[:, :w]
        got = o[p * ps:p * ps + h * ld].reshape(h, ld)
        assert np.abs(got[:, :w] - oracle.fd_compute(plane)).max() <= TOL
        assert np.isnan(got[:, w:]).all()
        assert np.isnan(o[p * ps + h * ld:(p + 1) * ps]).all()


@pytest.mark.parametrize("eps", [0.0, 1e-12, 1e-4])
def test_fd_flow_one_step_parity(wmc, eps):
    noisy, _ = wmc_synth.c1()
    U = noisy[0]
    g = wmc.fd_flow(to_gpu(U), 1, dt=0.1, eps=eps).cpu().numpy()
    r = oracle.fd_flow(U, 0.1, 1, eps=eps)
    if eps == 0.0:  # 0/0 where the gradient vanishes: both sides give NaN there
        assert np.array_equal(np.isnan(g), np.isnan(r))
        m = ~np.isnan(r)
        assert np.abs(g[m] - r[m]).max() <= 0.1 * TOL
    else:
        assert np.abs(g - r).max() <= 0.1 * TOL


def test_fd_flow_chain_and_planes(wmc):
    """k steps in one call equal k single-step calls bitwise; colour planes
    are flowed independently."""
    noisy, _ = wmc_synth.c3_image(0, 67, 150, 0.1)
    u = to_gpu(noisy)
    ref = u
    for _ in range(7):
        ref = wmc.fd_flow(ref, 1, dt=0.2)
    assert torch.equal(wmc.fd_flow(u, 7, dt=0.2), ref)
    for c in range(3):
        assert torch.equal(wmc.fd_flow(u[c].contiguous(), 7, dt=0.2), ref[c])
    assert torch.equal(wmc.fd_flow(u, 0), u)


def test_fd_flow_multi_step_parity(wmc):
    noisy, _ = wmc_synth.c1()
    g = wmc.fd_flow(to_gpu(noisy[0]), 20, dt=0.1).cpu().numpy()
    r = oracle.fd_flow(noisy[0], 0.1, 20)
    d = np.abs(g - r)
    assert d.max() <= 2e-4 and d.mean() <= 2e-6


def test_mcf_study_on_gpu(wmc):
    """Sec. 5.4: on a piecewise-constant image the half-window flow keeps
    edges and corners much better than the conventional one (1 - SSIM
    against the input at t = 10, 50, 200), the GPU flows agree with the oracle's
    numbers on the same image, and both flows are monotone in t."""
    a = wmc_synth.shapes(512)
    u = to_gpu(a)
    prev = (1.0, 1.0)
    for t in (10, 50, 200):
        s_hl = ssim(a, wmc.solve(None, iters=t, u0=u).cpu().numpy())
        s_fd = ssim(a, wmc.fd_flow(u, t, dt=0.1).cpu().numpy())
        # the structure lost by the conventional flow is many times larger
        assert s_hl > 0.99 and (1 - s_fd) > 5 * (1 - s_hl), (t, s_hl, s_fd)
        assert s_hl <= prev[0] + 1e-9 and s_fd <= prev[1] + 1e-9
        prev = (s_hl, s_fd)
    small = wmc_synth.shapes(96)
    for t in (10, 50):
        g = ssim(small, wmc.fd_flow(to_gpu(small), t, dt=0.1).cpu().numpy())
        r = ssim(small, oracle.fd_flow(small, 0.1, t))
        assert abs(g - r) < 1e-4
