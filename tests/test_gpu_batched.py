"""Uneven-size batched solve (one launch over all images, graph replay, autotuned
tiles) against per-image solves and, at full size, against the oracle on
sampled pixels."""
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import wmc_synth

sys.path.insert(0, os.path.dirname(__file__))
from parity_bounds import TAU  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wmc():
    import paper_1903_07189_amd as W
    W.lib()
    return W


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def small_batch(seed=0):
    rng = np.random.default_rng(seed)
    shapes = [(3, 1, 1), (1, 3, 200), (3, 57, 129), (2, 130, 64), (1, 200, 333), (3, 129, 517),
              (1, 64, 64), (3, 31, 1031)]
    return [to_gpu(rng.uniform(0, 1, size=s)) for s in shapes]


TUNE = [(1, 1, 8), (1, 4, 16), (2, 2, 8), (2, 3, 16), (2, 8, 64), (4, 3, 32), (4, 6, 8), (4, 1, 128)]


@pytest.mark.parametrize("c,t,r", TUNE)
def test_batched_equals_per_image(wmc, c, t, r):
    imgs = small_batch()
    lam = torch.linspace(0.5, 3.0, len(imgs), device="cuda:0")
    tun = {"cols": c, "tsteps": t, "seg_rows": r, "use_graph": 1}
    outs = wmc.solve_batched(imgs, lam, 13, tuning=tun)
    for i, x in enumerate(imgs):
        ref = x.clone()
        for _ in range(13):
            ref = wmc.step(ref, x, float(lam[i]))
        assert torch.equal(outs[i], ref), (i, c, t, r)


def test_batched_flow_mode_with_u0(wmc):
    rng = np.random.default_rng(1)
    u0s = [to_gpu(rng.uniform(0, 1, size=s)) for s in [(1, 40, 300), (3, 77, 91)]]
    outs = wmc.solve_batched([None, None], None, 7, dt=0.5, u0s=u0s,
                             tuning={"cols": 2, "tsteps": 4, "seg_rows": 16})
    for u0, o in zip(u0s, outs):
        ref = u0.clone()
        for _ in range(7):
            ref = wmc.step(ref, None, dt=0.5)
        assert torch.equal(o, ref)


def test_graph_replay_sees_new_data(wmc):
    """The cached graph is keyed by pointers: replays read the current contents."""
    imgs = small_batch(2)
    lam = torch.ones(len(imgs), device="cuda:0")
    plan = wmc.SolveBatchedPlan(imgs, lam, 9, tuning={"cols": 2, "tsteps": 3, "seg_rows": 16})
    first = [o.clone() for o in plan()]
    second = [o.clone() for o in plan()]
    for a, b in zip(first, second):
        assert torch.equal(a, b)
    imgs[3].mul_(0.5)
    third = plan()
    assert torch.equal(third[3], wmc.solve(imgs[3], 1.0, 9, tuning={"cols": 1, "tsteps": 1,
                                                                    "seg_rows": 8}))
    assert torch.equal(third[0], first[0])


def test_autotune_returns_valid_tuning(wmc, monkeypatch, tmp_path):
    monkeypatch.setenv("WMC_TUNE_CACHE", str(tmp_path / "t.json"))
    monkeypatch.setenv("WMC_TUNE", "force")
    imgs = small_batch(3)
    t = wmc.autotune(imgs, 20)
    assert t["cols"] in (1, 2, 4) and t["tsteps"] in (1, 2, 3, 4, 6, 8) and t["seg_rows"] >= 1
    # and the autotuned default path gives the same bits
    lam = torch.ones(len(imgs), device="cuda:0")
    monkeypatch.setenv("WMC_TUNE", "cached")
    a = wmc.solve_batched(imgs, lam, 10)
    b = wmc.solve_batched(imgs, lam, 10, tuning={"cols": 1, "tsteps": 1, "seg_rows": 8,
                                                 "use_graph": 0})
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_c3_full_batch(wmc):
    """The benchmark's uneven batch (64 images x 3 channels, sides 128..2048,
    100 iterations): batched == per-image plain launches bitwise, and sampled
    pixels == the FP64 oracle on their dependency cones."""
    sizes = wmc_synth.c3_sizes()
    imgs, nps = [], []
    for b, (h, w, sig) in enumerate(sizes):
        noisy, _ = wmc_synth.c3_image(b, h, w, sig)
        imgs.append(to_gpu(noisy))
        if b in (0, 5, 17, 63):
            nps.append((b, noisy))
    lam = torch.ones(len(imgs), device="cuda:0")
    outs = wmc.SolveBatchedPlan(imgs, lam, 100)()
    for i in (0, 9, 33, 63):
        ref = wmc.solve(imgs[i], 1.0, 100, tuning={"cols": 2, "tsteps": 1, "seg_rows": 32,
                                                   "use_graph": 0})
        assert torch.equal(outs[i], ref), i
    # oracle on sampled pixels: the last 3 iterations from the GPU state U^97
    rng = np.random.default_rng(7)
    for b, noisy in nps:
        u97 = wmc.solve(imgs[b], 1.0, 97, tuning={"cols": 2, "tsteps": 4, "seg_rows": 32})
        u97 = u97.cpu().numpy().astype(np.float64)
        got = outs[b].cpu().numpy()
        C, H, W = noisy.shape
        for _ in range(12):
            c, y, x = int(rng.integers(C)), int(rng.integers(H)), int(rng.integers(W))
            want = oracle.step_window(u97[c], noisy[c].astype(np.float64), y, x, 3, lam=1.0)
            if abs(want - got[c, y, x]) > 1e-5:
                # allowed only through a near tie in the dependency cone
                y0, y1, x0, x1 = max(0, y - 3), min(H, y + 4), max(0, x - 3), min(W, x + 4)
                assert oracle.near_tie_mask(u97[c, y0:y1, x0:x1], TAU).any(), (b, c, y, x)
