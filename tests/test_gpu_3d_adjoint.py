"""The 3-D adjoint (wmc3_backward) on the GPU against the oracle (O14).

The oracle replays the GPU's own selections (the byte map wmc3_step
returns), so the comparison is of the adjoint arithmetic alone; the GPU's
selections are checked separately against the oracle's, tie-aware.

Tolerances (FP32 against FP64):
- dL/dU: the gather sums 27 products of integer weights (sum |w| = 112) and
  cotangents, scaled by coef = delta lam / 56 <= 0.03 here: a few ulps of
  112 max|g| times coef, under 2e-5 max|g|;
- dL/df = delta g per step: 1e-6 relative;
- dL/dlam: sums of g dU'/dlam over the volume in FP32 partials: 1e-5 of
  sum |g dU'/dlam| (computed from the oracle's per-voxel terms)."""
import ctypes
import os
import sys

import numpy as np
import pytest
import torch

import oracle

sys.path.insert(0, os.path.dirname(__file__))
from parity_bounds import TAU3  # noqa: E402

pytestmark = pytest.mark.gpu


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


def gpu_selection(wmc, U, f, lam, dt=0.0):
    _, am = wmc.step3(to_gpu(U), None if f is None else to_gpu(f), lam, dt, return_argmin=True)
    return am.cpu().numpy().astype(np.int8)


def dudlam_scale(U, f, lam, delta, m, g):
    """sum |g dU'/dlam| over the volume with the selection m (default step)."""
    S = np.take_along_axis(candidates(U), m[None].astype(np.int64), axis=0)[0]
    h = S / 56.0
    du = delta * h - delta * delta * ((f - U) + lam * h)
    return float(np.sum(np.abs(g * du)))


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 2, 3), (2, 1, 1), (3, 3, 3), (4, 1, 70),
                                   (5, 7, 9), (3, 5, 130), (9, 17, 64)])
def test_selection_map(wmc, shape):
    """The GPU's selection equals the oracle's first minimum except where two
    candidates are within TAU3 of the least magnitude."""
    rng = np.random.default_rng(sum(shape))
    U = rng.uniform(0, 1, size=shape).astype(np.float32)
    m = gpu_selection(wmc, U, None, 1.0, 0.3)
    _, mo = oracle.step3(U.astype(np.float64), None, 1.0, 0.3, return_argmin=True)
    diff = m != mo
    if diff.any():
        S = np.abs(candidates(U.astype(np.float64)))
        mn = S.min(axis=0)
        picked = np.take_along_axis(S, m[None].astype(np.int64), axis=0)[0]
        assert np.all(picked[diff] <= mn[diff] + TAU3)
        assert diff.mean() < 1e-3


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 2, 3), (2, 1, 1), (3, 3, 3), (4, 1, 70),
                                   (5, 7, 9), (3, 5, 130), (6, 20, 64)])
@pytest.mark.parametrize("lam", [0.3, 2.5])
def test_one_step_against_oracle(wmc, shape, lam):
    rng = np.random.default_rng(100 + sum(shape) + int(lam * 10))
    U = rng.uniform(0, 1, size=shape).astype(np.float32)
    f = rng.uniform(0, 1, size=shape).astype(np.float32)
    g = (rng.uniform(-1, 1, size=shape) + 0.5).astype(np.float32)
    m = gpu_selection(wmc, U, f, lam)
    _, ck = wmc.solve3(to_gpu(f), lam, 1, u0=to_gpu(U), ckpt_every=1)
    g_f, g_u0, g_lam = wmc.backward3(to_gpu(g), to_gpu(f), lam, 1, ck, 1, u0=to_gpu(U))
    U64, f64, g64 = U.astype(np.float64), f.astype(np.float64), g.astype(np.float64)
    delta = 1.0 / (1.0 + lam)
    gU, gf, glam = oracle.step3_adjoint(U64, g64, f64, lam, m_forced=m)
    gmax = float(np.abs(g64).max())
    assert np.abs(g_u0[0].cpu().numpy() - gU).max() <= 2e-5 * gmax
    assert np.allclose(g_f[0].cpu().numpy(), gf, rtol=1e-6, atol=1e-7 * gmax)
    scale = dudlam_scale(U64, f64, lam, delta, m, g64)
    assert abs(float(g_lam[0]) - glam) <= 1e-5 * scale + 1e-7


@pytest.mark.parametrize("shape", [(1, 2, 3), (4, 1, 70), (5, 7, 9)])
def test_one_step_flow(wmc, shape):
    rng = np.random.default_rng(7 + sum(shape))
    U = rng.uniform(0, 1, size=shape).astype(np.float32)
    g = rng.normal(size=shape).astype(np.float32)
    dt = 0.3
    m = gpu_selection(wmc, U, None, 1.0, dt)
    _, ck = wmc.solve3(None, 1.0, 1, dt=dt, u0=to_gpu(U), ckpt_every=1)
    g_f, g_u0, g_lam = wmc.backward3(to_gpu(g), None, 1.0, 1, ck, 1, dt=dt, u0=to_gpu(U))
    assert g_f is None and g_lam is None
    gU, _, _ = oracle.step3_adjoint(U.astype(np.float64), g.astype(np.float64), None, 1.0, dt,
                                    m_forced=m)
    assert np.abs(g_u0[0].cpu().numpy() - gU).max() <= 2e-5 * float(np.abs(g).max())


def _gpu_trajectory_selections(wmc, f, lam, K):
    """The GPU's states and selections of K steps from U^0 = f."""
    u = to_gpu(f)
    F = to_gpu(f)
    ms = []
    for _ in range(K):
        un, am = wmc.step3(u, F, lam, return_argmin=True)
        ms.append(am.cpu().numpy().astype(np.int8))
        u = un
    return u, np.stack(ms)


@pytest.mark.parametrize("shape", [(5, 7, 9), (8, 12, 70)])
def test_k_steps_against_oracle_and_checkpoint_periods(wmc, shape):
    """K = 6 steps from U^0 = f: every checkpoint period gives the same bits;
    the gradients match the oracle replaying the GPU's selections."""
    rng = np.random.default_rng(sum(shape))
    f = rng.uniform(0, 1, size=shape).astype(np.float32)
    gK = (rng.uniform(-1, 1, size=shape) + 0.3).astype(np.float32)
    lam, K = 1.5, 6
    uK, ms = _gpu_trajectory_selections(wmc, f, lam, K)
    res = {}
    for c in (1, 2, 3, 4, 6, 7):
        out, ck = wmc.solve3(to_gpu(f), lam, K, ckpt_every=c)
        assert torch.equal(out, uK.reshape(out.shape))
        res[c] = wmc.backward3(to_gpu(gK), to_gpu(f), lam, K, ck, c)
    for c in (2, 3, 4, 6, 7):
        for a, b in zip(res[1], res[c]):
            assert torch.equal(a, b), c
    g_f, g_u0, g_lam = res[1]
    r = oracle.solve3_adjoint(gK.astype(np.float64), f.astype(np.float64), lam, K,
                              m_forced_all=ms)
    gmax = float(np.abs(gK).max())
    assert np.abs(g_u0[0].cpu().numpy() - r["gu0"]).max() <= 1e-4 * gmax
    assert np.abs(g_f[0].cpu().numpy() - (r["gf"] + r["gu0"])).max() <= 1e-4 * gmax
    assert abs(float(g_lam[0]) - r["glam"]) <= 1e-4 * (1.0 + abs(r["glam"]))


def test_k_steps_from_u0_split_and_flow(wmc):
    """From u0 != f the data-term dL/df and dL/dU^0 come apart; the flow has
    only dL/dU^0."""
    rng = np.random.default_rng(21)
    shape = (6, 9, 40)
    f = rng.uniform(0, 1, size=shape).astype(np.float32)
    u0 = rng.uniform(0, 1, size=shape).astype(np.float32)
    gK = rng.normal(size=shape).astype(np.float32)
    lam, K = 0.7, 4
    u = to_gpu(u0)
    ms = []
    for _ in range(K):
        u, am = wmc.step3(u, to_gpu(f), lam, return_argmin=True)
        ms.append(am.cpu().numpy().astype(np.int8))
    _, ck = wmc.solve3(to_gpu(f), lam, K, u0=to_gpu(u0), ckpt_every=2)
    g_f, g_u0, g_lam = wmc.backward3(to_gpu(gK), to_gpu(f), lam, K, ck, 2, u0=to_gpu(u0))
    r = oracle.solve3_adjoint(gK.astype(np.float64), f.astype(np.float64), lam, K,
                              u0=u0.astype(np.float64), m_forced_all=np.stack(ms))
    gmax = float(np.abs(gK).max())
    assert np.abs(g_u0[0].cpu().numpy() - r["gu0"]).max() <= 1e-4 * gmax
    assert np.abs(g_f[0].cpu().numpy() - r["gf"]).max() <= 1e-4 * gmax
    assert abs(float(g_lam[0]) - r["glam"]) <= 1e-4 * (1.0 + abs(r["glam"]))
    # flow from u0
    dt = 0.25
    u = to_gpu(u0)
    ms = []
    for _ in range(K):
        u, am = wmc.step3(u, None, 1.0, dt, return_argmin=True)
        ms.append(am.cpu().numpy().astype(np.int8))
    _, ck = wmc.solve3(None, 1.0, K, dt=dt, u0=to_gpu(u0), ckpt_every=3)
    _, g_u0, _ = wmc.backward3(to_gpu(gK), None, 1.0, K, ck, 3, dt=dt, u0=to_gpu(u0))
    r = oracle.solve3_adjoint(gK.astype(np.float64), None, 1.0, K, delta=dt,
                              u0=u0.astype(np.float64), m_forced_all=np.stack(ms))
    assert np.abs(g_u0[0].cpu().numpy() - r["gu0"]).max() <= 1e-4 * gmax


def test_padded_volumes_through_the_abi(wmc):
    """Two volumes with padded rows, slices and volumes: each volume's
    gradients equal those of the same volume solved alone (dL/dU and dL/df
    bitwise; dL/dlam to rounding, its work items group differently), and
    the padding of every output stays untouched."""
    from paper_1903_07189_amd import wmc as M
    L = M.lib()
    n, d, h, w = 2, 5, 9, 70
    ld, ss = 72, 9 * 72 + 8
    vs = d * ss + 40
    rng = np.random.default_rng(33)
    lam = np.array([0.6, 1.8], dtype=np.float32)
    vols = [rng.uniform(0, 1, size=(d, h, w)).astype(np.float32) for _ in range(n)]
    gs = [rng.normal(size=(d, h, w)).astype(np.float32) for _ in range(n)]

    def pack(arrs):
        flat = np.full(n * vs, np.nan, dtype=np.float32)
        for v, a in enumerate(arrs):
            for z in range(d):
                for y in range(h):
                    flat[v * vs + z * ss + y * ld: v * vs + z * ss + y * ld + w] = a[z, y]
        return flat

    def unpack(flat):
        return [np.stack([np.stack([flat[v * vs + z * ss + y * ld: v * vs + z * ss + y * ld + w]
                                    for y in range(h)]) for z in range(d)]) for v in range(n)]

    s = M.Shape3(n, d, h, w, ld, ss, vs)
    K, c = 3, 2
    F, G = to_gpu(pack(vols)), to_gpu(pack(gs))
    lt = to_gpu(lam)
    setst = L.wmc3_set_stride(s)
    nck = L.wmc_num_checkpoints(K, c)
    ck = torch.full((nck * setst,), float("nan"), device="cuda:0")
    out = torch.full((n * vs,), float("nan"), device="cuda:0")
    ws = torch.empty(L.wmc3_solve_workspace(s) // 4 + 64, device="cuda:0")
    M.check(L.wmc3_solve(M._ptr(F), None, M._ptr(out), M._ptr(lt), K, 0.0, M._ptr(ck), c,
                         M._ptr(ws), ws.numel() * 4, s, M._stream()))
    bws = torch.empty(L.wmc3_backward_workspace(s, K, c) // 4 + 64, device="cuda:0")
    gf = torch.full((n * vs,), float("nan"), device="cuda:0")
    gl = torch.empty(n, device="cuda:0")
    M.check(L.wmc3_backward(M._ptr(F), None, M._ptr(lt), K, 0.0, M._ptr(ck), c, M._ptr(G),
                            M._ptr(gf), None, M._ptr(gl), M._ptr(bws), bws.numel() * 4, s,
                            M._stream()))
    gff = gf.cpu().numpy()
    pad = np.isnan(pack([np.zeros((d, h, w), np.float32)] * n))
    assert np.isnan(gff[pad]).all()
    got = unpack(gff)
    for v in range(n):
        o1, ck1 = wmc.solve3(to_gpu(vols[v]), float(lam[v]), K, ckpt_every=c)
        g1, _, l1 = wmc.backward3(to_gpu(gs[v]), to_gpu(vols[v]), float(lam[v]), K, ck1, c)
        assert np.array_equal(got[v], g1.cpu().numpy()[0])
        assert abs(float(gl[v]) - float(l1[0])) <= 1e-5 * (1.0 + abs(float(l1[0])))
        assert np.array_equal(unpack(out.cpu().numpy())[v], o1.cpu().numpy())


def test_autograd_matches_backward3(wmc):
    rng = np.random.default_rng(4)
    f = to_gpu(rng.uniform(0, 1, size=(2, 6, 10, 33)))
    clean = to_gpu(rng.uniform(0, 1, size=(2, 6, 10, 33)))
    lam = torch.tensor([0.8, 1.6], device="cuda:0", requires_grad=True)
    fg = f.clone().requires_grad_(True)
    u = wmc.WMCSolve3.apply(fg, lam, 5, 0.0, 2)
    loss = ((u - clean) ** 2).sum()
    loss.backward()
    out, ck = wmc.solve3(f, lam.detach(), 5, ckpt_every=2)
    assert torch.equal(u.detach(), out)
    g_f, _, g_lam = wmc.backward3(2 * (out - clean), f, lam.detach(), 5, ck, 2)
    assert torch.equal(fg.grad, g_f)
    assert torch.equal(lam.grad, g_lam)


def test_full_volume_one_step_64cubed(wmc):
    """One step on a 64^3 volume (every voxel against the oracle replaying the
    GPU's selection)."""
    rng = np.random.default_rng(64)
    shape = (64, 64, 64)
    U = rng.uniform(0, 1, size=shape).astype(np.float32)
    f = rng.uniform(0, 1, size=shape).astype(np.float32)
    g = rng.normal(size=shape).astype(np.float32)
    lam = 1.0
    m = gpu_selection(wmc, U, f, lam)
    _, ck = wmc.solve3(to_gpu(f), lam, 1, u0=to_gpu(U), ckpt_every=1)
    g_f, g_u0, g_lam = wmc.backward3(to_gpu(g), to_gpu(f), lam, 1, ck, 1, u0=to_gpu(U))
    gU, gf, glam = oracle.step3_adjoint(U.astype(np.float64), g.astype(np.float64),
                                        f.astype(np.float64), lam, m_forced=m)
    gmax = float(np.abs(g).max())
    assert np.abs(g_u0[0].cpu().numpy() - gU).max() <= 2e-5 * gmax
    assert np.allclose(g_f[0].cpu().numpy(), gf, rtol=1e-6, atol=1e-7 * gmax)
    scale = dudlam_scale(U.astype(np.float64), f.astype(np.float64), lam, 0.5, m,
                         g.astype(np.float64))
    assert abs(float(g_lam[0]) - glam) <= 1e-5 * scale + 1e-6


def test_adjoint_volume_beyond_2_pow_31_elements(wmc):
    """A 1300^3 volume (2.2e9 voxels, 64-bit offsets in both adjoint
    kernels): one step's dL/dU^0 and dL/df at sampled voxels, corners
    included, against the oracle on 7^3 crops with the GPU's selections
    (a voxel's gradient depends only on the selections and cotangents of
    its 27 neighbours, all inside the crop; where the crop is cut by the
    volume's border, that border is the real one)."""
    n = 1300
    gen = torch.Generator(device="cuda:0").manual_seed(5)
    f = torch.rand((n, n, n), device="cuda:0", generator=gen)
    g = torch.rand((n, n, n), device="cuda:0", generator=gen) - 0.5
    out, ck = wmc.solve3(f, 1.0, 1, ckpt_every=1)
    del out
    g_f, g_u0, _ = wmc.backward3(g, f, 1.0, 1, ck, 1)
    del ck
    out, am = wmc.step3(f, f, 1.0, return_argmin=True)
    del out
    torch.cuda.empty_cache()
    rng = np.random.default_rng(6)
    pts = [(0, 0, 0), (n - 1, n - 1, n - 1), (n - 1, 0, n - 1), (0, n - 1, 0), (650, 0, 1299)]
    pts += [tuple(int(c) for c in rng.integers(0, n, 3)) for _ in range(12)]
    for (z, y, x) in pts:
        lo = [max(0, c - 3) for c in (z, y, x)]
        hi = [min(n, c + 4) for c in (z, y, x)]
        sl = tuple(slice(a, b) for a, b in zip(lo, hi))
        fc = f[sl].cpu().numpy().astype(np.float64)
        gc = g[sl].cpu().numpy().astype(np.float64)
        mc = am[sl].cpu().numpy().astype(np.int8)
        gU, gfd, _ = oracle.step3_adjoint(fc, gc, fc, 1.0, m_forced=mc)
        k = (z - lo[0], y - lo[1], x - lo[2])
        assert abs(float(g_u0[0, z, y, x]) - gU[k]) <= 2e-5, (z, y, x)
        assert abs(float(g_f[0, z, y, x]) - (gfd[k] + gU[k])) <= 2e-5, (z, y, x)
    del f, g, g_f, g_u0, am
    torch.cuda.empty_cache()


def test_binding_rejects_mismatched_shapes(wmc):
    """The 3-D binding checks shapes before any kernel is enqueued: a
    checkpoint buffer of another period, a cotangent or data term of
    another shape."""
    f = to_gpu(np.zeros((3, 4, 5)))
    _, ck = wmc.solve3(f, 1.0, 6, ckpt_every=3)  # 2 checkpoint sets
    with pytest.raises(ValueError, match="ckpt"):
        wmc.backward3(f, f, 1.0, 6, ck, 2)       # period 2 needs 3 sets
    with pytest.raises(ValueError, match="g_out"):
        wmc.backward3(to_gpu(np.zeros((3, 4, 6))), f, 1.0, 6, ck, 3)
    with pytest.raises(ValueError, match="f has shape"):
        wmc.step3(f, to_gpu(np.zeros((2, 4, 5))))
    with pytest.raises(ValueError, match="has shape"):
        wmc.solve3(to_gpu(np.zeros((3, 4, 6))), 1.0, 2, u0=f)


@pytest.mark.parametrize("shape", [(2, 3, 4), (5, 7, 70)])
def test_one_step_explicit_step_size(wmc, shape):
    """Data term with an explicit dt > 0: dU'/dlam = dt H has no delta'(lam)
    term (the default-step branch of the selection pass is off)."""
    rng = np.random.default_rng(300 + sum(shape))
    U = rng.uniform(0, 1, size=shape).astype(np.float32)
    f = rng.uniform(0, 1, size=shape).astype(np.float32)
    g = (rng.uniform(-1, 1, size=shape) + 0.5).astype(np.float32)
    lam, dt = 2.5, 0.2
    m = gpu_selection(wmc, U, f, lam, dt)
    _, ck = wmc.solve3(to_gpu(f), lam, 1, dt=dt, u0=to_gpu(U), ckpt_every=1)
    g_f, g_u0, g_lam = wmc.backward3(to_gpu(g), to_gpu(f), lam, 1, ck, 1, dt=dt, u0=to_gpu(U))
    U64, f64, g64 = U.astype(np.float64), f.astype(np.float64), g.astype(np.float64)
    gU, gf, glam = oracle.step3_adjoint(U64, g64, f64, lam, dt, delta_from_lam=False, m_forced=m)
    gmax = float(np.abs(g64).max())
    assert np.abs(g_u0[0].cpu().numpy() - gU).max() <= 2e-5 * gmax
    assert np.allclose(g_f[0].cpu().numpy(), gf, rtol=1e-6, atol=1e-7 * gmax)
    S = np.take_along_axis(candidates(U64), m[None].astype(np.int64), axis=0)[0]
    scale = float(np.sum(np.abs(g64 * dt * S / 56.0)))
    assert abs(float(g_lam[0]) - glam) <= 1e-5 * scale + 1e-7


def test_zero_steps(wmc):
    """A solve of 0 steps returns U^0: its backward gives dL/dU^0 = g_out,
    dL/df = g_out when U^0 = f (zero when u0 is given), dL/dlam = 0."""
    rng = np.random.default_rng(8)
    f = to_gpu(rng.uniform(0, 1, size=(3, 5, 70)))
    u0 = to_gpu(rng.uniform(0, 1, size=(3, 5, 70)))
    g = to_gpu(rng.normal(size=(3, 5, 70)))
    out, ck = wmc.solve3(f, 1.3, 0, ckpt_every=2)
    assert torch.equal(out, f)
    g_f, g_u0, g_lam = wmc.backward3(g, f, 1.3, 0, ck, 2)
    assert torch.equal(g_u0[0], g) and torch.equal(g_f[0], g)
    assert float(g_lam[0]) == 0.0
    _, ck = wmc.solve3(f, 1.3, 0, u0=u0, ckpt_every=2)
    g_f, g_u0, g_lam = wmc.backward3(g, f, 1.3, 0, ck, 2, u0=u0)
    assert torch.equal(g_u0[0], g)
    assert torch.count_nonzero(g_f) == 0 and float(g_lam[0]) == 0.0
