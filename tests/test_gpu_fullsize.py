"""The benchmark workload at full size (4096 x 4096, 200 iterations) in the
launch configuration bench.py times: properties that hold at any size and
oracle checks on sampled pixels."""
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import wmc_synth

sys.path.insert(0, os.path.dirname(__file__))
from parity_bounds import TAU, TOL  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import paper_1903_07189_amd as W
    W.lib()
    noisy, _ = wmc_synth.c2()
    f = torch.from_numpy(noisy).to("cuda:0")
    lam = torch.tensor([1.0], device="cuda:0")
    tuning = W.solve_tuning(f, lam)
    return W, noisy, f, lam, tuning


def test_fused_equals_steps_at_full_size(setup):
    W, noisy, f, lam, tuning = setup
    out = W.SolvePlan(f, lam, 200, tuning=tuning)()
    ref = f.clone()
    for _ in range(200):
        ref = W.step(ref, f, lam)
    assert torch.equal(out, ref)
    # maximum principle over the whole solve
    assert out.min() >= f.min() and out.max() <= f.max()


def test_sampled_pixels_against_oracle(setup):
    W, noisy, f, lam, tuning = setup
    f64 = noisy[0].astype(np.float64)
    rng = np.random.default_rng(11)
    # first launch block: U^T from U^0 = f
    T = tuning["tsteps"]
    uT = W.solve(f, lam, T, tuning=tuning)[0].cpu().numpy()
    # last block: U^200 from U^(200-T)
    u_pre = W.solve(f, lam, 200 - T, tuning=tuning)[0].cpu().numpy().astype(np.float64)
    u200 = W.solve(f, lam, 200, tuning=tuning)[0].cpu().numpy()
    ys = list(rng.integers(0, 4096, size=150)) + [0, 4095, 0, 4095, 2047]
    xs = list(rng.integers(0, 4096, size=150)) + [0, 0, 4095, 4095, 3000]
    flips = 0
    for y, x in zip(ys, xs):
        for src, got in ((f64, uT), (u_pre, u200)):
            want = oracle.step_window(src, f64, int(y), int(x), T, lam=1.0)
            if abs(want - got[y, x]) > 1e-5:
                y0, y1 = max(0, y - T), min(4096, y + T + 1)
                x0, x1 = max(0, x - T), min(4096, x + T + 1)
                assert oracle.near_tie_mask(src[y0:y1, x0:x1], TAU).any(), (y, x)
                flips += 1
    assert flips <= 3


def test_full_plane_step_against_oracle(setup):
    """One Jacobi update of the whole 4096^2 plane from U = f, every pixel
    against the FP64 oracle: a pixel off by more than 1e-5 passes only as the
    update through a candidate within TAU (x12 units) of the minimum."""
    W, noisy, f, lam, tuning = setup
    f64 = noisy[0].astype(np.float64)
    u1 = W.step(f, f, lam)[0].cpu().numpy().astype(np.float64)
    ref = oracle.step(f64, f64, 1.0)
    bad = np.abs(u1 - ref) > TOL
    nb = int(bad.sum())
    if nb:
        S = oracle.candidates(f64)[bad]
        mag = np.abs(S)
        close = mag <= mag.min(axis=1, keepdims=True) + TAU
        upd = f64[bad][:, None] + 0.5 * S / 12.0   # U = f, delta = 1/2, lam = 1
        ok = np.any(close & (np.abs(upd - u1[bad][:, None]) <= TOL), axis=1)
        assert ok.all(), f"{int((~ok).sum())} pixels off outside near ties"
    assert nb <= 1e-4 * f64.size


def test_full_plane_fused_block_shadow(setup):
    """The first fused launch of the benchmark solve (T sweeps from U = f) over
    the whole plane, under the shadow protocol: at every sweep each selection
    the GPU made must be within TAU of the minimum magnitude of the oracle's
    candidates on the shadow state, and the oracle, replaying those
    selections, must end within 1e-5 of the fused output everywhere."""
    W, noisy, f, lam, tuning = setup
    T = tuning["tsteps"]
    f64 = noisy[0].astype(np.float64)
    uT = W.solve(f, lam, T, tuning=tuning)[0]
    u = f.clone()
    maps = []
    for _ in range(T):
        u, m = W.step(u, f, lam, return_argmin=True)
        maps.append(m[0].cpu().numpy().astype(np.int64))
    assert torch.equal(u[0], uT)   # the fused launch is its T single sweeps
    sh = f64.copy()
    for t in range(T):
        S = oracle.candidates(sh)
        mag = np.abs(S)
        chosen = np.take_along_axis(mag, maps[t][..., None], axis=2)[..., 0]
        assert (chosen <= mag.min(axis=2) + TAU).all(), f"disallowed selection at sweep {t}"
        del S, mag, chosen
        sh = oracle.step(sh, f64, 1.0, m_forced=maps[t])
    assert np.abs(uT.cpu().numpy().astype(np.float64) - sh).max() <= TOL


def test_denoising_quality(setup):
    """The solve moves the noisy input towards the clean image."""
    W, noisy, f, lam, tuning = setup
    _, clean = wmc_synth.c2()
    out = W.solve(f, lam, 200, tuning=tuning)[0].cpu().numpy()
    e_in = np.sqrt(((noisy[0] - clean[0]) ** 2).mean())
    e_out = np.sqrt(((out - clean[0]) ** 2).mean())
    assert e_out < 0.8 * e_in


def test_planes_beyond_2_pow_30_elements():
    """Two planes of 23000 x 47000 (each more than 2^30 elements, so plane
    offsets pass 2^31): one step, the operator and a 3-sweep fused solve,
    sampled against the oracle on local windows (exact: the window is cut
    only by the true image border or at least k pixels from the sample)."""
    import paper_1903_07189_amd as W
    H, Wd = 23000, 47000
    assert H * Wd > 2 ** 30
    g = torch.Generator(device="cuda:0").manual_seed(5)
    u = torch.rand((2, H, Wd), device="cuda:0", generator=g)
    f = torch.rand((2, H, Wd), device="cuda:0", generator=g)
    lam = torch.tensor([1.0, 2.0], device="cuda:0")
    u1 = W.step(u, f, lam)
    h = W.compute(u)
    u3 = W.solve(f, lam, 3, u0=u, tuning={"cols": 2, "tsteps": 3, "seg_rows": 64})
    rng = np.random.default_rng(9)
    pts = [(1, H - 1, Wd - 1), (1, H - 1, 0), (1, 0, Wd - 1), (0, 0, 0), (1, H // 2, Wd - 2)]
    pts += [(int(rng.integers(0, 2)), int(rng.integers(0, H)), int(rng.integers(0, Wd)))
            for _ in range(20)]
    for (p, y, x) in pts:
        for k, got in ((1, u1), (3, u3)):
            y0, y1 = max(0, y - k), min(H, y + k + 1)
            x0, x1 = max(0, x - k), min(Wd, x + k + 1)
            cu = u[p, y0:y1, x0:x1].cpu().numpy().astype(np.float64)
            cf = f[p, y0:y1, x0:x1].cpu().numpy().astype(np.float64)
            ref = oracle.step_window(cu, cf, y - y0, x - x0, k, lam=float(lam[p]))
            val = float(got[p, y, x])
            if abs(val - ref) > 1e-5:  # only through a near tie of the selection
                assert k == 1 and oracle.near_tie_mask(cu, TAU)[y - y0, x - x0], (p, y, x, k)
        y0, y1 = max(0, y - 1), min(H, y + 2)
        x0, x1 = max(0, x - 1), min(Wd, x + 2)
        cu = u[p, y0:y1, x0:x1].cpu().numpy().astype(np.float64)
        hr = oracle.compute(cu)[y - y0, x - x0]
        hv = float(h[p, y, x])
        if abs(hv - hr) > 1e-5:
            assert oracle.near_tie_mask(cu, TAU)[y - y0, x - x0], (p, y, x)
    del u, f, u1, h, u3
    torch.cuda.empty_cache()
