"""The benchmark workload at full size (4096 x 4096, 200 iterations) in the
launch configuration bench.py times: properties that hold at any size and
oracle checks on sampled pixels."""
import numpy as np
import pytest
import torch

import oracle
import wmc_synth

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
                assert oracle.near_tie_mask(src[y0:y1, x0:x1], 1e-4).any(), (y, x)
                flips += 1
    assert flips <= 3


def test_denoising_quality(setup):
    """The solve moves the noisy input towards the clean image."""
    W, noisy, f, lam, tuning = setup
    _, clean = wmc_synth.c2()
    out = W.solve(f, lam, 200, tuning=tuning)[0].cpu().numpy()
    e_in = np.sqrt(((noisy[0] - clean[0]) ** 2).mean())
    e_out = np.sqrt(((out - clean[0]) ** 2).mean())
    assert e_out < 0.8 * e_in
