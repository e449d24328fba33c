"""Calibration of the near-tie width TAU (see parity_bounds.py): the largest
difference between the GPU's selected response and the oracle's response of
the same candidate, over pixels whose selection is not in doubt, must be at
most TAU / 8 (2-D, x12 units) and TAU3 / 8 (3-D, x56 units)."""
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import wmc_synth

sys.path.insert(0, os.path.dirname(__file__))
from parity_bounds import TAU, TAU3  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wmc():
    import paper_1903_07189_amd as W
    W.lib()
    return W


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def eps_2d(wmc, u32):
    """max |12 H_gpu - S_oracle[m]| over pixels where the GPU's selection (its
    selection map) equals the oracle's."""
    U = to_gpu(u32)
    h = wmc.compute(U).cpu().numpy().astype(np.float64)
    _, m = wmc.step(U, U, 1.0, return_argmin=True)
    m = m.cpu().numpy().astype(np.int64)
    U64 = u32.astype(np.float64)
    S = oracle.candidates(U64)
    _, mo = oracle.compute(U64, return_argmin=True)
    same = m == mo
    Sm = np.take_along_axis(S, mo[..., None].astype(np.int64), axis=2)[..., 0]
    return float(np.abs(12.0 * h - Sm)[same].max())


def test_tau_2d(wmc):
    noisy, _ = wmc_synth.c1()
    f = to_gpu(noisy[0])
    u = f
    eps = 0.0
    for _ in range(50):
        eps = max(eps, eps_2d(wmc, u.cpu().numpy()))
        u = wmc.step(u, f, 1.0)
    rng = np.random.default_rng(0)
    for _ in range(6):
        eps = max(eps, eps_2d(wmc, rng.uniform(0, 1, size=(300, 517)).astype(np.float32)))
    print(f"\n2-D: max |S_gpu - S_oracle| at settled pixels {eps:.3e}; 8x = {8 * eps:.3e}, "
          f"TAU = {TAU:.1e}")
    assert 0.0 < eps and 8.0 * eps <= TAU


def test_tau_3d(wmc):
    from scipy import ndimage
    rng = np.random.default_rng(1)
    eps = 0.0
    for shape in ((12, 20, 70), (9, 65, 130), (30, 30, 30)):
        U = rng.uniform(0, 1, size=shape).astype(np.float32)
        h = wmc.compute3(to_gpu(U)).cpu().numpy().astype(np.float64)
        U64 = U.astype(np.float64)
        S = np.stack([ndimage.correlate(U64, k.astype(np.float64), mode="nearest")
                      for k in oracle.kernels3()])
        mag = np.sort(np.abs(S), axis=0)
        # settled: the runner-up magnitude is clearly above the minimum
        settled = mag[1] - mag[0] > 1e-3
        ref, _ = oracle.compute3(U64, return_argmin=True)
        eps = max(eps, float(np.abs(56.0 * (h - ref))[settled].max()))
    print(f"\n3-D: max |S_gpu - S_oracle| at settled voxels {eps:.3e}; 8x = {8 * eps:.3e}, "
          f"TAU3 = {TAU3:.1e}")
    assert 0.0 < eps and 8.0 * eps <= TAU3
