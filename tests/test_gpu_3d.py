"""The 3-D extension (18 half windows of the tensor-product Laplacian) on
the GPU against the oracle (O13).

Tolerances: each candidate is a sum of 26 weighted taps (weights 1..8,
values in [0, 1]) in FP32, so |S| <~ 64 with an error of a few ulps:
2e-6 on H = S/56.  Where two candidates of different value are within
TAU3 (x56 units, calibrated in parity_bounds.py) in magnitude FP32 and FP64
may select differently;
there the GPU value must be one of the near-minimal candidates."""
import os
import sys

import numpy as np
import pytest
import torch

import oracle

sys.path.insert(0, os.path.dirname(__file__))
from parity_bounds import TAU3  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 2e-6
TAU = TAU3


@pytest.fixture(scope="module")
def wmc():
    import paper_1903_07189_amd as W
    W.lib()
    return W


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def candidates(U):
    from scipy import ndimage
    return np.stack([ndimage.correlate(U, k.astype(np.float64), mode="nearest")
                     for k in oracle.kernels3()])


def check_h(U, h):
    U = U.astype(np.float64)
    ref = oracle.compute3(U)
    bad = np.abs(h - ref) > TOL
    if bad.any():
        S = candidates(U)
        mn = np.abs(S).min(axis=0)
        ok = np.any((np.abs(S) <= mn + TAU) & (np.abs(S / 56.0 - h[None]) <= TOL), axis=0)
        assert ok[bad].all()
        assert bad.mean() < 1e-3
    return bad.sum()


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 4), (5, 7, 9), (4, 1, 70), (17, 33, 70),
                                   (9, 65, 130)])
def test_compute3_parity(wmc, shape):
    U = np.random.default_rng(sum(shape)).uniform(0, 1, size=shape).astype(np.float32)
    h = wmc.compute3(to_gpu(U)).cpu().numpy()
    check_h(U, h)


def test_compute3_exact_cases(wmc):
    z, y, x = np.mgrid[0:9, 0:10, 0:11].astype(np.float32)
    assert torch.count_nonzero(wmc.compute3(to_gpu(np.full((5, 6, 7), 0.7, np.float32)))) == 0
    for U in (0.5 * x, -0.25 * y, 2.0 * z, x + y, x - z, y + z):
        h = wmc.compute3(to_gpu(U)).cpu().numpy()
        assert np.all(h[1:-1, 1:-1, 1:-1] == 0.0)
    c = 4
    U = (x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2
    h = wmc.compute3(to_gpu(U)).cpu().numpy()
    assert abs(h[c, c, c] - 12.0 / 7.0) <= 1e-6


def test_volumes_and_strides(wmc):
    rng = np.random.default_rng(3)
    U = rng.uniform(0, 1, size=(3, 6, 20, 90)).astype(np.float32)
    h = wmc.compute3(to_gpu(U)).cpu().numpy()
    for v in range(3):
        check_h(U[v], h[v])
    # a padded layout through the raw ABI
    from paper_1903_07189_amd import wmc as M
    n, d, hh, w, ld = 2, 5, 7, 33, 40
    ss, vs = hh * ld + 8, d * (hh * ld + 8) + 16
    base = rng.uniform(0, 1, size=n * vs).astype(np.float32)
    src = to_gpu(base)
    out = torch.full((n * vs,), float("nan"), device="cuda:0")
    import ctypes
    M.check(M.lib().wmc3_compute(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                 M.Shape3(n, d, hh, w, ld, ss, vs), None))
    o = out.cpu().numpy()
    for v in range(n):
        vol = np.stack([base[v * vs + z * ss: v * vs + z * ss + hh * ld].reshape(hh, ld)[:, :w]
                        for z in range(d)])
        got = np.stack([o[v * vs + z * ss: v * vs + z * ss + hh * ld].reshape(hh, ld) for z in range(d)])
        check_h(vol, got[:, :, :w])
        assert np.isnan(got[:, :, w:]).all()


def check_step3(u1, U, f, lam, delta):
    """One 3-D Jacobi update from U (FP32 values cast to FP64) against the
    oracle, voxel by voxel: a voxel off by more than 1e-5 passes only if it is
    the update through a candidate within TAU (x56 units) of the minimum
    magnitude.  Returns the number of such voxels."""
    U = U.astype(np.float64)
    f64 = None if f is None else f.astype(np.float64)
    ref = oracle.solve3(f64, lam, 1, delta=delta, u0=U)
    bad = np.abs(u1 - ref) > 1e-5
    if bad.any():
        S = candidates(U)
        mn = np.abs(S).min(axis=0)
        if f64 is None:
            upd = U[None] + delta * S / 56.0
        else:
            upd = U[None] + delta * ((f64 - U)[None] + lam * S / 56.0)
        ok = np.any((np.abs(S) <= mn + TAU) & (np.abs(upd - u1[None]) <= 1e-5), axis=0)
        assert ok[bad].all(), f"{int((bad & ~ok).sum())} voxels off by up to {np.abs(u1 - ref)[bad & ~ok].max()}"
    return int(bad.sum())


@pytest.mark.parametrize("mcf", [False, True])
def test_solve3_parity(wmc, mcf):
    """Ten steps, each checked voxel by voxel from the GPU's own previous
    state (the shadow protocol: every selection the GPU makes must be an
    allowed one), then k steps in one call against k single-step calls."""
    rng = np.random.default_rng(7)
    f = rng.uniform(0, 1, size=(12, 20, 70)).astype(np.float32)
    F = to_gpu(f)
    lam = 1.5
    delta = oracle.default_delta(lam, mcf)
    u = F
    flips = 0
    for _ in range(10):
        un = wmc.solve3(None, iters=1, u0=u) if mcf else wmc.solve3(F, lam, 1, u0=u)
        flips += check_step3(un.cpu().numpy().astype(np.float64), u.cpu().numpy(),
                             None if mcf else f, lam, delta)
        u = un
    assert flips <= 1e-3 * 10 * f.size
    # k steps in one call = k single-step calls, bitwise
    uk = wmc.solve3(None, iters=10, u0=F) if mcf else wmc.solve3(F, lam, 10)
    assert torch.equal(u, uk)
    if not mcf:
        # 10 free-running steps against FP64: near-tie flips decay in data mode
        g = uk.cpu().numpy()
        r = oracle.solve3(f, lam, 10)
        assert np.abs(g - r).mean() < 1e-5
        # maximum principle of the default step
        assert g.min() >= f.min() - 1e-6 and g.max() <= f.max() + 1e-6


def test_volume_beyond_2_pow_31_elements(wmc):
    """A 1300^3 volume (2.2e9 voxels): 64-bit plane offsets; sampled voxels
    against the oracle on local windows."""
    n = 1300
    g = torch.Generator(device="cuda:0").manual_seed(3)
    v = torch.rand((n, n, n), device="cuda:0", generator=g)
    h = wmc.compute3(v)
    rng = np.random.default_rng(4)
    pts = [(n - 1, n - 1, n - 1), (n - 1, 0, n - 1), (0, n - 1, 0)]
    pts += [tuple(int(c) for c in rng.integers(0, n, 3)) for _ in range(12)]
    for (z, y, x) in pts:
        z0, z1 = max(0, z - 1), min(n, z + 2)
        y0, y1 = max(0, y - 1), min(n, y + 2)
        x0, x1 = max(0, x - 1), min(n, x + 2)
        cu = v[z0:z1, y0:y1, x0:x1].cpu().numpy().astype(np.float64)
        got = float(h[z, y, x])
        ref = oracle.compute3(cu)[z - z0, y - y0, x - x0]
        if abs(got - ref) > TOL:
            S = candidates(cu)[:, z - z0, y - y0, x - x0]
            mn = np.abs(S).min()
            assert np.any((np.abs(S) <= mn + TAU) & (np.abs(S / 56.0 - got) <= TOL))
    del v, h
    torch.cuda.empty_cache()
