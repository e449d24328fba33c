"""GPU adjoint (wmc_backward / WMCSolve) against the FP64 oracle.

Bar: norm-wise relative error <= 1e-4 for dL/df and dL/dlam.  The GPU
gradient is the exact derivative of its own FP32 forward map; the oracle is
run with the GPU's selections replayed (shadow), because where two candidates
nearly tie FP32 and FP64 may select differently and the derivative of the
selected branch differs.  Finite differences are taken in FP64 by the oracle,
excluding perturbations that change any selection along the path.
"""
import numpy as np
import pytest
import torch

import oracle
import wmc_synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wmc():
    import paper_1903_07189_amd as W
    W.lib()
    return W


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def gpu_maps(wmc, f, lam, K, dt=0.0, mcf=False, u0=None):
    """Selection maps (N, K, H, W) of the GPU forward trajectory (bitwise the
    trajectory of solve) and the final state."""
    ref = u0 if u0 is not None else f
    if ref.dim() == 2:
        ref = ref.unsqueeze(0)
        f = None if f is None else f.unsqueeze(0)
    u = ref.clone()
    maps = []
    for _ in range(K):
        u, m = wmc.step(u, None if mcf else f, lam, dt=dt, return_argmin=True)
        maps.append(m.cpu().numpy().astype(np.int8))
    return np.stack(maps, axis=1), u


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("ckpt_every", [1, 3, 5, 20])
def test_backward_matches_oracle_shadow(wmc, ckpt_every):
    N, H, W, K = 2, 48, 70, 20
    noisy = np.stack([wmc_synth.image(H, W, 1, 0.1, seed=2000 + b)[0][0] for b in range(N)])
    clean = np.stack([wmc_synth.image(H, W, 1, 0.1, seed=2000 + b)[1][0] for b in range(N)])
    f = to_gpu(noisy)
    lam = torch.tensor([1.0, 2.5], device="cuda:0")
    uK, ck = wmc.solve(f, lam, K, ckpt_every=ckpt_every,
                       tuning={"cols": 2, "tsteps": 4, "seg_rows": 16})
    g_out = 2.0 * (uK - to_gpu(clean)) / uK.numel()
    g_f, g_u0, g_lam = wmc.backward(g_out, f, lam, K, ck, ckpt_every)
    maps, u_steps = gpu_maps(wmc, f, lam, K)
    assert torch.equal(u_steps, uK)
    for p in range(N):
        res = oracle.solve_adjoint(g_out[p].cpu().numpy().astype(np.float64),
                                   noisy[p].astype(np.float64), float(lam[p]), K,
                                   m_forced_all=maps[p])
        want_f = res["gf"] + res["gu0"]
        assert rel(g_f[p].cpu().numpy(), want_f) <= 1e-4
        assert rel(g_u0[p].cpu().numpy(), res["gu0"]) <= 1e-4
        assert abs(float(g_lam[p]) - res["glam"]) <= 1e-4 * max(abs(res["glam"]), 1e-12)


def test_backward_independent_of_checkpoint_period(wmc):
    rng = np.random.default_rng(1)
    f = to_gpu(rng.uniform(0, 1, size=(2, 40, 90)))
    lam = torch.tensor([0.7, 1.3], device="cuda:0")
    g_out = to_gpu(rng.standard_normal((2, 40, 90)))
    outs = []
    for c in (1, 2, 7, 13):
        _, ck = wmc.solve(f, lam, 13, ckpt_every=c, tuning={"cols": 1, "tsteps": 3, "seg_rows": 8})
        outs.append(wmc.backward(g_out, f, lam, 13, ck, c))
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert torch.equal(a, b)   # bitwise: deterministic, no atomics


def test_backward_fixed_step_and_flow_mode(wmc):
    rng = np.random.default_rng(2)
    H, W, K = 30, 41, 6
    u0 = rng.uniform(0, 1, size=(H, W))
    g = rng.standard_normal((H, W))
    # flow mode (no data term): gradient w.r.t. the initial state
    U0 = to_gpu(u0)
    uK, ck = wmc.solve(None, iters=K, dt=0.4, u0=U0, ckpt_every=2)
    _, g_u0, _ = wmc.backward(to_gpu(g), None, None, K, ck, 2, dt=0.4, u0=U0)
    maps, _ = gpu_maps(wmc, None, 1.0, K, dt=0.4, mcf=True, u0=U0)
    res = oracle.solve_adjoint(g, None, 1.0, K, delta=0.4, u0=u0, m_forced_all=maps[0])
    assert rel(g_u0[0].cpu().numpy(), res["gu0"]) <= 1e-4
    # data term with an explicit step: no d(delta)/d(lam) term
    f = to_gpu(u0)
    lam = torch.tensor([1.5], device="cuda:0")
    uK, ck = wmc.solve(f, lam, K, dt=0.3, ckpt_every=3)
    g_f, _, g_lam = wmc.backward(to_gpu(g), f, lam, K, ck, 3, dt=0.3)
    maps, _ = gpu_maps(wmc, f, lam, K, dt=0.3)
    res = oracle.solve_adjoint(g, u0, 1.5, K, delta=0.3, delta_from_lam=False,
                               m_forced_all=maps[0])
    assert rel(g_f[0].cpu().numpy(), res["gf"] + res["gu0"]) <= 1e-4
    assert abs(float(g_lam[0]) - res["glam"]) <= 1e-4 * abs(res["glam"])


def fd_crop_check(wmc, f64, c64, lam, K, rng, n_try=40):
    """dL/df at n_try random pixels and dL/dlam of one standalone crop: the
    GPU adjoint (checkpoints every ceil(sqrt(K))) against FP64 central
    differences of the oracle's solve, skipping perturbations that change a
    selection anywhere along the path."""
    c = int(np.ceil(np.sqrt(K)))
    f = to_gpu(f64)
    lt = torch.tensor([lam], device="cuda:0")
    uK, ck = wmc.solve(f, lt, K, ckpt_every=c)
    g_out = 2.0 * (uK - to_gpu(c64)) / uK.numel()
    g_f, _, g_lam = wmc.backward(g_out, f, lt, K, ck, c)
    g_f = g_f[0].cpu().numpy().astype(np.float64)

    def loss(ff, ll):
        u = oracle.solve(ff, lam=ll, iters=K)
        return float(((u - c64) ** 2).mean())

    def path_maps(ff):
        u = ff.copy()
        out = []
        for _ in range(K):
            u, m = oracle.step(u, ff, lam, return_argmin=True)
            out.append(m)
        return np.stack(out)

    h = 1e-6
    H, W = f64.shape
    checked, errs = 0, []
    for _ in range(n_try):
        y, x = int(rng.integers(H)), int(rng.integers(W))
        fp, fm = f64.copy(), f64.copy()
        fp[y, x] += h
        fm[y, x] -= h
        if not np.array_equal(path_maps(fp), path_maps(fm)):
            continue
        fd = (loss(fp, lam) - loss(fm, lam)) / (2 * h)
        errs.append(abs(fd - g_f[y, x]) / max(abs(fd), 1e-3 * np.abs(g_f).max()))
        checked += 1
    assert checked >= n_try // 2
    assert max(errs) <= 1e-4, max(errs)
    fdl = (loss(f64, lam + h) - loss(f64, lam - h)) / (2 * h)
    assert abs(fdl - float(g_lam[0])) <= 1e-4 * abs(fdl)


def c4_crops():
    """The four 32x32 crops of the differentiable-layer workload: (240, 240)
    of image 0 and three seeded ones on images 1..3."""
    rng = np.random.default_rng(2020)
    crops = [(0, 240, 240)]
    for b in (1, 2, 3):
        crops.append((b, int(rng.integers(0, 512 - 32)), int(rng.integers(0, 512 - 32))))
    return crops


@pytest.mark.parametrize("crop", range(4))
def test_backward_vs_fp64_finite_differences(wmc, crop):
    """32x32 crops of the differentiable-layer workload (lambda = 1, K = 20)
    as standalone images."""
    noisy, clean = wmc_synth.c4(batch=4, side=512)
    b, y0, x0 = c4_crops()[crop]
    f64 = noisy[b, 0, y0:y0 + 32, x0:x0 + 32].astype(np.float64)
    c64 = clean[b, 0, y0:y0 + 32, x0:x0 + 32].astype(np.float64)
    fd_crop_check(wmc, f64, c64, 1.0, 20, np.random.default_rng(3 + crop))


@pytest.mark.parametrize("lam", [0.3, 2.5])
def test_backward_vs_fp64_finite_differences_lambda(wmc, lam):
    """The same finite-difference check away from lambda = 1, where the
    default step 1/(1+lambda) differs from 1 - 1/(1+lambda), so a swapped
    data-term factor or a wrong d(delta)/d(lambda) term would show."""
    noisy, clean = wmc_synth.c4(batch=4, side=512)
    b, y0, x0 = c4_crops()[1 if lam < 1 else 2]
    f64 = noisy[b, 0, y0:y0 + 32, x0:x0 + 32].astype(np.float64)
    c64 = clean[b, 0, y0:y0 + 32, x0:x0 + 32].astype(np.float64)
    fd_crop_check(wmc, f64, c64, lam, 20, np.random.default_rng(int(lam * 10)))


def test_autograd_function(wmc):
    rng = np.random.default_rng(4)
    f = to_gpu(rng.uniform(0, 1, size=(3, 36, 50))).requires_grad_(True)
    target = to_gpu(rng.uniform(0, 1, size=(3, 36, 50)))
    lam = torch.tensor([0.5, 1.0, 2.0], device="cuda:0", requires_grad=True)
    c = 3  # ceil(sqrt(9)), passed explicitly (the default keeps every state)
    out = wmc.WMCSolve.apply(f, lam, 9, 0.0, c)
    loss = ((out - target) ** 2).mean()
    loss.backward()
    # same numbers through the explicit binding
    uK, ck = wmc.solve(f.detach(), lam.detach(), 9, ckpt_every=c)
    assert torch.equal(uK, out.detach())
    g_f, _, g_lam = wmc.backward(2 * (uK - target) / uK.numel(), f.detach(), lam.detach(), 9, ck, c)
    assert torch.allclose(f.grad, g_f, rtol=1e-6, atol=1e-12)
    assert torch.allclose(lam.grad, g_lam, rtol=1e-6, atol=1e-12)
    # scalar lambda tensor: gradient summed over planes
    ls = torch.tensor(1.0, device="cuda:0", requires_grad=True)
    out = wmc.WMCSolve.apply(f.detach(), ls, 4)
    out.sum().backward()
    assert ls.grad.shape == ()


def test_autograd_gradients_independent_of_forward_shape(wmc):
    """The differentiable solve's gradients are bitwise the same whatever
    launch shape the forward uses (its states are those of single steps) and
    whatever the checkpoint period (deterministic reductions)."""
    rng = np.random.default_rng(14)
    f0 = to_gpu(rng.uniform(0, 1, size=(2, 64, 136)))
    target = to_gpu(rng.uniform(0, 1, size=(2, 64, 136)))
    ref = None
    for tn in [None, {"cols": 2, "tsteps": 4, "seg_rows": 16}, {"cols": 2, "tsteps": 2, "seg_rows": 8},
               {"cols": 4, "tsteps": 3, "seg_rows": 12}, {"cols": 1, "tsteps": 1, "seg_rows": 5}]:
        for c in (1, 3):
            f = f0.clone().requires_grad_(True)
            lam = torch.tensor([0.6, 1.8], device="cuda:0", requires_grad=True)
            out = wmc.WMCSolve.apply(f, lam, 9, 0.0, c, tn)
            ((out - target) ** 2).mean().backward()
            got = (out.detach(), f.grad, lam.grad)
            if ref is None:
                ref = got
            for a, b in zip(got, ref):
                assert torch.equal(a, b), (tn, c)


def test_c4_batch_against_oracle(wmc):
    """The full differentiable-layer batch (16x1x512x512, K = 20, checkpoints
    every 5): every image checked against the shadowed FP64 adjoint."""
    noisy, clean = wmc_synth.c4()
    f = to_gpu(noisy[:, 0])
    lam = torch.ones(16, device="cuda:0")
    uK, ck = wmc.solve(f, lam, 20, ckpt_every=5)
    g_out = 2.0 * (uK - to_gpu(clean[:, 0])) / uK.numel()
    g_f, _, g_lam = wmc.backward(g_out, f, lam, 20, ck, 5)
    for b in range(16):
        fb = f[b:b + 1]
        maps, _ = gpu_maps(wmc, fb, lam[b:b + 1], 20)
        res = oracle.solve_adjoint(g_out[b].cpu().numpy().astype(np.float64),
                                   noisy[b, 0].astype(np.float64), 1.0, 20, m_forced_all=maps[0])
        assert rel(g_f[b].cpu().numpy(), res["gf"] + res["gu0"]) <= 1e-4
        assert abs(float(g_lam[b]) - res["glam"]) <= 1e-4 * abs(res["glam"])


@pytest.mark.parametrize("cols", ["1", "2", "4"])
@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (9, 1), (2, 3), (5, 60), (3, 61), (17, 62),
                                   (33, 120), (70, 121), (40, 250), (129, 257)])
def test_one_step_adjoint_shapes_and_lane_widths(wmc, monkeypatch, shape, cols):
    """One adjoint step on shapes around the strip and segment boundaries of
    every lane width (1, 2, 4 columns per lane), two planes, against the
    oracle with the GPU's selection replayed: dL/dU, dL/df and dL/dlam."""
    monkeypatch.setenv("WMC_ADJ_COLS", cols)
    H, W = shape
    rng = np.random.default_rng(H * 1000 + W)
    u0 = rng.uniform(0, 1, size=(2, H, W))
    fv = rng.uniform(0, 1, size=(2, H, W))
    g = rng.standard_normal((2, H, W))
    U0, F = to_gpu(u0), to_gpu(fv)
    lam = torch.tensor([0.8, 2.0], device="cuda:0")
    _, ck = wmc.solve(F, lam, 1, u0=U0, ckpt_every=1)
    g_f, g_u0, g_lam = wmc.backward(to_gpu(g), F, lam, 1, ck, 1, u0=U0)
    _, m = wmc.step(U0, F, lam, return_argmin=True)
    m = m.cpu().numpy().astype(np.int8)
    for p in range(2):
        res = oracle.solve_adjoint(g[p], fv[p].astype(np.float32), float(lam[p]), 1,
                                   u0=u0[p].astype(np.float32), m_forced_all=m[p][None])
        assert rel(g_u0[p].cpu().numpy(), res["gu0"]) <= 1e-5
        assert rel(g_f[p].cpu().numpy(), res["gf"]) <= 1e-5
        assert abs(float(g_lam[p]) - res["glam"]) <= 1e-4 * max(abs(res["glam"]), 1e-6)


@pytest.mark.parametrize("cols", ["1", "2", "4"])
def test_one_step_adjoint_on_tie_heavy_data(wmc, monkeypatch, cols):
    """Dyadic images of a few grey levels, where many of the eight responses
    tie exactly: the adjoint must take the forward's first-minimum choice at
    every tie (a different tied candidate has a different derivative).  One
    step, against the oracle with the forward's selection replayed."""
    monkeypatch.setenv("WMC_ADJ_COLS", cols)
    rng = np.random.default_rng(77)
    H, W = 37, 131
    u0 = rng.integers(0, 5, size=(2, H, W)) / 4.0
    u0[:, :, 60:] = np.round(np.linspace(0.0, 1.0, W - 60) * 8) / 8.0  # dyadic ramp
    fv = rng.integers(0, 3, size=(2, H, W)) / 2.0
    g = rng.standard_normal((2, H, W))
    U0, F = to_gpu(u0), to_gpu(fv)
    lam = torch.tensor([1.0, 3.0], device="cuda:0")
    _, ck = wmc.solve(F, lam, 1, u0=U0, ckpt_every=1)
    g_f, g_u0, g_lam = wmc.backward(to_gpu(g), F, lam, 1, ck, 1, u0=U0)
    _, m = wmc.step(U0, F, lam, return_argmin=True)
    m = m.cpu().numpy().astype(np.int8)
    for p in range(2):
        res = oracle.solve_adjoint(g[p], fv[p].astype(np.float32), float(lam[p]), 1,
                                   u0=u0[p].astype(np.float32), m_forced_all=m[p][None])
        assert rel(g_u0[p].cpu().numpy(), res["gu0"]) <= 1e-5
        assert rel(g_f[p].cpu().numpy(), res["gf"]) <= 1e-5
        assert abs(float(g_lam[p]) - res["glam"]) <= 1e-4 * max(abs(res["glam"]), 1e-6)


def test_rows_per_item_override(wmc, monkeypatch):
    """WMC_ADJ_ROWS (more rows per adjoint work item than the default) gives
    the same gradients: dL/df bitwise (per-pixel arithmetic is unchanged),
    dL/dlam to rounding (its partial sums group the pixels differently)."""
    rng = np.random.default_rng(5)
    f = to_gpu(rng.uniform(0, 1, size=(2, 90, 70)))
    lam = torch.tensor([1.0, 2.0], device="cuda:0")
    uK, ck = wmc.solve(f, lam, 6, ckpt_every=2)
    g = to_gpu(rng.standard_normal((2, 90, 70)))
    ref = wmc.backward(g, f, lam, 6, ck, 2)
    monkeypatch.setenv("WMC_ADJ_ROWS", "40")
    got = wmc.backward(g, f, lam, 6, ck, 2)
    assert torch.equal(got[0], ref[0])
    assert torch.allclose(got[2], ref[2], rtol=1e-5, atol=0.0)


def test_tall_image_checkpointed_solve_and_backward(wmc):
    """An image taller than 65535 rows (1 x 70000 x 64) through the paths that
    copy and accumulate whole plane sets: a zero-step solve (a copy), a
    checkpointed solve, and the backward from those checkpoints (dL/df,
    dL/dU^0 and dL/dlam), against the FP64 oracle with the GPU's selections
    replayed, over the whole image."""
    H, W, K, c = 70000, 64, 6, 3
    rng = np.random.default_rng(70000)
    f_np = rng.uniform(0, 1, size=(H, W))
    u0_np = rng.uniform(0, 1, size=(H, W))
    g_np = rng.standard_normal((H, W))
    f, u0, g = to_gpu(f_np), to_gpu(u0_np), to_gpu(g_np)
    lam = torch.tensor([2.5], device="cuda:0")
    assert torch.equal(wmc.solve(f, lam, 0, u0=u0), u0)
    uK, ck = wmc.solve(f, lam, K, u0=u0, ckpt_every=c)
    g_f, g_u0, g_lam = wmc.backward(g, f, lam, K, ck, c, u0=u0)
    maps, u_steps = gpu_maps(wmc, f, lam, K, u0=u0)
    assert torch.equal(uK, u_steps[0])
    # the checkpoints are the states U^0 and U^3 of the trajectory
    assert torch.equal(ck[0, 0], u0)
    res = oracle.solve_adjoint(g_np, f_np.astype(np.float32), 2.5, K,
                               u0=u0_np.astype(np.float32), m_forced_all=maps[0])
    assert rel(g_f[0].cpu().numpy(), res["gf"]) <= 1e-4
    assert rel(g_u0[0].cpu().numpy(), res["gu0"]) <= 1e-4
    assert abs(float(g_lam[0]) - res["glam"]) <= 1e-4 * abs(res["glam"])
    # U^0 = f: dL/df includes the path through U^0 (a plane-set accumulate)
    uK2, ck2 = wmc.solve(f, lam, K, ckpt_every=c)
    g_f2, _, _ = wmc.backward(g, f, lam, K, ck2, c)
    maps2, _ = gpu_maps(wmc, f, lam, K)
    res2 = oracle.solve_adjoint(g_np, f_np.astype(np.float32), 2.5, K, m_forced_all=maps2[0])
    assert rel(g_f2[0].cpu().numpy(), res2["gf"] + res2["gu0"]) <= 1e-4
