"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (FP32 kernel vs FP64 oracle on [0, 1] images):
  * single operator / step: max-abs <= 1e-5 outside the near-tie set;
  * 50 / 100 iterations: <= 1e-4 under the shadow protocol.
The selection of eq. (act) is discontinuous where two candidates of opposite
sign have (nearly) equal magnitude; there FP32 and FP64 may legitimately pick
differently.  A pixel whose value differs from the oracle's by more than the
tolerance passes only if the GPU value is the update of a candidate within
TAU (x12 units) of the minimum magnitude, and such pixels are counted.
"""
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
def wmc():
    import paper_1903_07189_amd as W
    W.lib()
    W.selftest()
    return W


def dev():
    return torch.device("cuda:0")


def to_gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev())


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def tie_aware_compute(gpu, U64):
    """Returns the number of near-tie pixels; asserts all others match."""
    ref = oracle.compute(U64)
    diff = np.abs(gpu - ref)
    bad = diff > TOL
    if not bad.any():
        return 0
    allowed = oracle.allowed_values(U64, TAU)
    near = np.nanmin(np.abs(allowed - gpu[..., None]), axis=2) <= TOL
    assert near[bad].all(), f"{(~near & bad).sum()} pixels off by up to {diff[bad & ~near].max()}"
    return int(bad.sum())


def tie_aware_step(gpu, U64, f64, lam, delta):
    ref = oracle.step(U64, f64, lam, delta)
    diff = np.abs(gpu - ref)
    bad = diff > TOL
    if not bad.any():
        return 0
    allowed = oracle.allowed_values(U64, TAU)  # H_d values of allowed candidates
    if f64 is None:
        upd = U64[..., None] + delta * allowed
    else:
        upd = U64[..., None] + delta * ((f64 - U64)[..., None] + lam * allowed)
    near = np.nanmin(np.abs(upd - gpu[..., None]), axis=2) <= TOL
    assert near[bad].all(), f"{(~near & bad).sum()} pixels off by up to {diff[bad & ~near].max()}"
    return int(bad.sum())


SHAPES = [(1, 1), (1, 7), (6, 1), (3, 5), (37, 300), (130, 517), (64, 64), (257, 129), (20, 1100)]


def test_selftest(wmc):
    wmc.selftest()


@pytest.mark.parametrize("shape", SHAPES)
def test_compute_random(wmc, shape):
    U = wmc_synth.random_unit(*shape, seed=sum(shape))
    got = to_np(wmc.compute(to_gpu(U)))
    n_tie = tie_aware_compute(got, U.astype(np.float64))
    assert n_tie <= max(2, U.size // 1000)


def test_compute_c1_image(wmc):
    noisy, _ = wmc_synth.c1()
    got = to_np(wmc.compute(to_gpu(noisy[0])))
    n_tie = tie_aware_compute(got, noisy[0].astype(np.float64))
    assert n_tie <= 20


def test_compute_exact_cases(wmc):
    """Dyadic inputs make every FP32 operation exact: the GPU must reproduce
    the oracle's canonical tie choices (opposite-sign exact ties included)."""
    H = W = 23
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    cases = [
        ((x - 11) ** 2 + (y - 11) ** 2) / 64.0,          # paraboloid with the (2,2) tie
        0.25 * x - 0.875 * y,                              # plane: cross tie of h1/h5
        0.375 * x + 0.125 * y,
        np.where((x >= 5) & (x < 15) & (y >= 4) & (y < 12), 0.75, 0.25),  # rectangle corners
        np.full((H, W), 0.3125),
        np.random.default_rng(3).integers(0, 16, size=(H, W)) / 16.0,
    ]
    for U in cases:
        got = to_np(wmc.compute(to_gpu(U)))
        ref = oracle.compute(U)
        # values S/12 are not all representable; the selection (incl. sign) is exact
        assert np.abs(got - ref).max() <= 1e-6
        g_step, g_m = wmc.step(to_gpu(U), None, dt=0.5, return_argmin=True)
        _, m = oracle.compute(U, return_argmin=True)
        assert np.array_equal(g_m.cpu().numpy().astype(np.int8), m)


@pytest.mark.parametrize("mcf", [False, True])
@pytest.mark.parametrize("shape", [(1, 1), (5, 9), (37, 300), (130, 517), (256, 256)])
def test_step_random(wmc, shape, mcf):
    U = wmc_synth.random_unit(*shape, seed=7 + sum(shape))
    f = None if mcf else wmc_synth.random_unit(*shape, seed=8 + sum(shape))
    lam = 1.7
    delta = 0.8 if mcf else 1 / (1 + lam)
    got, gm = wmc.step(to_gpu(U), None if mcf else to_gpu(f), lam, dt=delta if mcf else 0.0,
                       return_argmin=True)
    U64 = U.astype(np.float64)
    f64 = None if mcf else f.astype(np.float64)
    n = tie_aware_step(to_np(got), U64, f64, lam, delta)
    assert n <= max(2, U.size // 1000)
    # the selection map agrees except at near ties
    _, m = oracle.compute(U64, return_argmin=True)
    near = oracle.near_tie_mask(U64, TAU)
    assert np.array_equal(gm.cpu().numpy().astype(np.int8)[~near], m[~near])


def test_step_explicit_dt_and_multi_plane(wmc):
    rng = np.random.default_rng(2)
    N, H, W = 3, 33, 70
    U = rng.uniform(0, 1, size=(N, H, W)).astype(np.float32)
    f = rng.uniform(0, 1, size=(N, H, W)).astype(np.float32)
    lam = torch.tensor([0.5, 1.0, 3.0], device=dev())
    got = to_np(wmc.step(to_gpu(U), to_gpu(f), lam, dt=0.2))
    for p in range(N):
        n = tie_aware_step(got[p], U[p].astype(np.float64), f[p].astype(np.float64),
                           float(lam[p]), 0.2)
        assert n <= 3


def test_strided_layout(wmc):
    """Row stride > width and plane stride > h*ld (views into larger buffers)."""
    rng = np.random.default_rng(4)
    big = to_gpu(rng.uniform(0, 1, size=(2, 50, 97)))
    view = big[:, 3:43, 5:90]   # ld = 97, ps = 50*97, starts unaligned
    fview = to_gpu(rng.uniform(0, 1, size=(2, 50, 97)))[:, 3:43, 5:90]
    got = to_np(wmc.step(view, fview, 1.0))
    dense = to_np(wmc.step(view.contiguous(), fview.contiguous(), 1.0))
    assert np.array_equal(got, dense)
    for p in range(2):
        tie_aware_step(got[p], to_np(view[p]), to_np(fview[p]), 1.0, 0.5)


def test_vector_only_build_matches_general(wmc):
    """The vector-only kernel builds (taken when every strip moves its rows
    with vector accesses) give bitwise the results of the general builds
    (taken here through a padded layout whose odd row stride leaves rows
    unaligned), for the operator, a step, fused solves and trajectories."""
    rng = np.random.default_rng(40)
    f = to_gpu(rng.uniform(0, 1, size=(2, 70, 300)))       # 300 columns: every C qualifies
    pad_f = torch.zeros((2, 70, 301), device="cuda:0")
    pad_f[:, :, :300] = f
    fv = pad_f[:, :, :300]                                   # ld = 301: unaligned rows
    assert fv.stride(1) == 301
    lam = torch.tensor([0.8, 2.0], device="cuda:0")
    assert torch.equal(wmc.compute(f), wmc.compute(fv))
    assert torch.equal(wmc.step(f, f, lam), wmc.step(fv, fv, lam))
    for c, t, r in [(2, 1, 8), (4, 1, 3), (2, 3, 16), (4, 4, 35), (2, 2, 5), (4, 2, 64)]:
        tn = {"cols": c, "tsteps": t, "seg_rows": r}
        a = wmc.solve(f, lam, 9, tuning=tn)
        b = wmc.solve(fv, lam, 9, tuning=tn)
        assert torch.equal(a, b), (c, t, r)
    # checkpoints stored from inside fused launches (vector-only trajectory
    # builds here) are the states of single steps (general builds)
    a, ck = wmc.solve(f, lam, 9, ckpt_every=2, tuning={"cols": 2, "tsteps": 4, "seg_rows": 16})
    u = fv
    for t in range(9):
        if t % 2 == 0:
            assert torch.equal(ck[t // 2], u.contiguous()), t
        u = wmc.step(u, fv, lam)
    assert torch.equal(a, u.contiguous())


TUNINGS = [(c, t, r) for c in (1, 2, 4) for t in (1, 2, 3, 4, 6, 8) for r in (1, 5, 16, 64)]


@pytest.mark.parametrize("shape", [(1, 1), (2, 3), (9, 70), (67, 300), (130, 517)])
def test_fused_solve_bitwise_equals_steps(wmc, shape):
    """Temporal blocking, strip/segment tiling and graph replay are bitwise
    invisible: every launch shape gives exactly the result of repeated steps."""
    rng = np.random.default_rng(11)
    f = to_gpu(rng.uniform(0, 1, size=shape))
    iters = 11
    ref = f.clone()
    for _ in range(iters):
        ref = wmc.step(ref, f, 1.3)
    for c, t, r in TUNINGS:
        for g in (0, 1):
            out = wmc.solve(f, 1.3, iters, tuning={"cols": c, "tsteps": t, "seg_rows": r,
                                                   "use_graph": g})
            assert torch.equal(out, ref), (c, t, r, g)


def test_fused_solve_flow_mode_and_u0(wmc):
    rng = np.random.default_rng(12)
    u0 = to_gpu(rng.uniform(0, 1, size=(45, 260)))
    f = to_gpu(rng.uniform(0, 1, size=(45, 260)))
    ref = u0.clone()
    for _ in range(9):
        ref = wmc.step(ref, None, dt=0.7)
    for c, t, r in [(1, 4, 8), (2, 3, 16), (4, 8, 64), (2, 6, 5)]:
        out = wmc.solve(None, iters=9, dt=0.7, u0=u0,
                        tuning={"cols": c, "tsteps": t, "seg_rows": r, "use_graph": 1})
        assert torch.equal(out, ref)
    ref = u0.clone()
    for _ in range(7):
        ref = wmc.step(ref, f, 2.0)
    out = wmc.solve(f, 2.0, 7, u0=u0, tuning={"cols": 2, "tsteps": 4, "seg_rows": 16})
    assert torch.equal(out, ref)


def test_resume_is_bitwise(wmc):
    rng = np.random.default_rng(13)
    f = to_gpu(rng.uniform(0, 1, size=(64, 200)))
    tun = {"cols": 2, "tsteps": 4, "seg_rows": 32}
    full = wmc.solve(f, 1.0, 100, tuning=tun)
    part = wmc.solve(f, 1.0, 60, u0=wmc.solve(f, 1.0, 40, tuning=tun), tuning=tun)
    assert torch.equal(full, part)


def test_checkpoints_are_the_states(wmc):
    rng = np.random.default_rng(14)
    f = to_gpu(rng.uniform(0, 1, size=(2, 30, 90)))
    tun = {"cols": 1, "tsteps": 4, "seg_rows": 8}
    out, ck = wmc.solve(f, 0.8, 13, ckpt_every=5, tuning=tun)
    assert ck.shape[0] == 3
    for j, t in enumerate([0, 5, 10]):
        want = f.clone() if t == 0 else wmc.solve(f, 0.8, t, tuning=tun)
        assert torch.equal(ck[j], want)
    assert torch.equal(out, wmc.solve(f, 0.8, 13, tuning=tun))


@pytest.mark.parametrize("cols,tsteps,every", [(1, 2, 1), (2, 3, 1), (2, 4, 1), (4, 3, 2),
                                                (1, 4, 3), (2, 3, 5), (2, 4, 7), (2, 6, 4),
                                                (1, 8, 1), (2, 6, 7)])
@pytest.mark.parametrize("flow", [False, True])
def test_checkpoints_inside_fused_launches(wmc, cols, tsteps, every, flow):
    """Checkpoints that fall inside a fused launch (stored by the trajectory
    variant, T <= 4; a deeper T with denser checkpoints runs T = 4 launches,
    a deeper T with sparser ones ends its launches at the checkpoints) are
    bitwise the states of single steps, on a ragged multi-strip shape."""
    rng = np.random.default_rng(100 + 10 * cols + tsteps + every)
    f = to_gpu(rng.uniform(0, 1, size=(2, 37, 150)))
    tun = {"cols": cols, "tsteps": tsteps, "seg_rows": 9}
    K = 17
    if flow:
        out, ck = wmc.solve(None, iters=K, dt=0.3, u0=f, ckpt_every=every, tuning=tun)
    else:
        out, ck = wmc.solve(f, 0.7, K, ckpt_every=every, tuning=tun)
    assert ck.shape[0] == -(-K // every)
    u = f.clone()
    step1 = {"cols": cols, "tsteps": 1, "seg_rows": 9}
    for t in range(K + 1):
        if t % every == 0 and t < K:
            assert torch.equal(ck[t // every], u), t
        if t < K:
            u = (wmc.solve(None, iters=1, dt=0.3, u0=u, tuning=step1) if flow
                 else wmc.solve(f, 0.7, 1, u0=u, tuning=step1))
    assert torch.equal(out, u)


@pytest.mark.parametrize("tsteps,every,ld", [(1, 3, 160), (2, 3, 160), (3, 3, 160), (4, 3, 160),
                                              (4, 5, 160), (6, 6, 160), (4, 3, 161)])
def test_checkpoint0_on_padded_rows(wmc, tsteps, every, ld):
    """Checkpoint 0 (= f) is stored by the first trajectory launch as it
    reads its input rows (T = 2..4 with rows moved by vector accesses), or by
    a plane copy (T = 1, a deeper T whose launches end at the checkpoints, or
    an odd row stride): either way it is f bitwise, on a padded row layout
    whose padding stays untouched, and the solve's result is that of the same
    solve on the unpadded image."""
    import ctypes
    from paper_1903_07189_amd import wmc as M
    L = M.lib()
    n, h, w, K = 2, 41, 150, 13
    ps = h * ld + 32
    rng = np.random.default_rng(40 + tsteps + every)
    base = rng.uniform(0, 1, size=n * ps).astype(np.float32)
    f = to_gpu(base)
    s = M.Shape(n, h, w, ld, ps)
    setst = L.wmc_set_stride(s)
    nck = L.wmc_num_checkpoints(K, every)
    ck = torch.full((nck * setst,), float("nan"), device=dev())
    out = torch.full((n * ps,), float("nan"), device=dev())
    ws = torch.empty(L.wmc_solve_workspace(s) // 4 + 64, device=dev())
    lt = torch.full((n,), 0.7, device=dev())
    tn = M.Tuning(2, tsteps, 9, 1)
    M.check(L.wmc_solve(M._ptr(f), None, M._ptr(out), M._ptr(lt), K, 0.0, M._ptr(ck), every,
                        ctypes.byref(tn), M._ptr(ws), ws.numel() * 4, s, M._stream()))
    c0 = ck[:setst].cpu().numpy()
    o = out.cpu().numpy()
    img = np.stack([base[v * ps: v * ps + h * ld].reshape(h, ld)[:, :w] for v in range(n)])
    ref = wmc.solve(to_gpu(img), 0.7, K, tuning={"cols": 2, "tsteps": tsteps, "seg_rows": 9}).cpu().numpy()
    for v in range(n):
        rows = c0[v * ps: v * ps + h * ld].reshape(h, ld)
        assert np.array_equal(rows[:, :w], img[v])
        assert np.isnan(rows[:, w:]).all()
        got = o[v * ps: v * ps + h * ld].reshape(h, ld)
        assert np.array_equal(got[:, :w], ref[v])
        assert np.isnan(got[:, w:]).all()


def test_default_tuning_path(wmc, monkeypatch, tmp_path):
    """The autotuned default (no tuning given) is bitwise the same result."""
    monkeypatch.setenv("WMC_TUNE_CACHE", str(tmp_path / "tune.json"))
    rng = np.random.default_rng(15)
    f = to_gpu(rng.uniform(0, 1, size=(100, 300)))
    ref = wmc.solve(f, 1.0, 12, tuning={"cols": 1, "tsteps": 1, "seg_rows": 64, "use_graph": 0})
    out = wmc.solve(f, 1.0, 12)
    assert torch.equal(out, ref)
    assert (tmp_path / "tune.json").exists()


@pytest.mark.parametrize("two_sets", [False, True])
def test_tuning_search_workspaces(wmc, monkeypatch, tmp_path, two_sets):
    """A forced search through wmc_solve_tuning, with a workspace of one
    plane set (candidates read U from u0) or of two (candidates ping-pong in
    the workspace), writes nothing but the workspace and returns a shape
    whose solve is bitwise the fixed-shape one."""
    import ctypes
    from paper_1903_07189_amd import wmc as M
    monkeypatch.setenv("WMC_TUNE", "force")
    monkeypatch.setenv("WMC_TUNE_CACHE", str(tmp_path / "tune.json"))
    rng = np.random.default_rng(16)
    f = to_gpu(rng.uniform(0, 1, size=(2, 100, 300)))
    u0 = to_gpu(rng.uniform(0, 1, size=(2, 100, 300)))
    f_keep, u0_keep = f.clone(), u0.clone()
    lam = torch.tensor([0.7, 1.5], device="cuda:0")
    s = M.shape_of(f)
    L = M.lib()
    set_bytes = L.wmc_solve_workspace(s)
    nbytes = 2 * set_bytes + 256 if two_sets else set_bytes
    ws = torch.empty((nbytes + 3) // 4, dtype=torch.float32, device="cuda:0")
    t = M.Tuning()
    M.check(L.wmc_solve_tuning(M._ptr(f), M._ptr(u0), M._ptr(lam), 0.0, M._ptr(ws), nbytes,
                               s, ctypes.byref(t), M._stream()))
    torch.cuda.synchronize()
    assert torch.equal(f, f_keep) and torch.equal(u0, u0_keep)
    assert t.cols in (1, 2, 4) and t.tsteps in (1, 2, 3, 4, 6, 8) and t.seg_rows >= 1
    got = wmc.solve(f, lam, 11, u0=u0, tuning={"cols": t.cols, "tsteps": t.tsteps,
                                                 "seg_rows": t.seg_rows, "use_graph": 1})
    ref = wmc.solve(f, lam, 11, u0=u0, tuning={"cols": 1, "tsteps": 1, "seg_rows": 64,
                                                 "use_graph": 0})
    assert torch.equal(got, ref)


def _shadow(wmc, f32, lam, iters, mcf=False, delta=None):
    """Shadow protocol: the GPU runs `iters` steps recording its selection maps;
    the oracle follows in FP64, adopting the GPU's choice wherever it is one of
    the candidates within TAU of the minimum (and failing if it is not)."""
    f = to_gpu(f32)
    u = f.clone()
    maps = []
    for _ in range(iters):
        u, m = wmc.step(u, None if mcf else f, lam, dt=delta or 0.0, return_argmin=True)
        maps.append(m.cpu().numpy().astype(np.int8))
    f64 = f32.astype(np.float64)
    d = delta if delta else (1.0 if mcf else 1 / (1 + lam))
    U = f64.copy()
    adopted = 0
    for t in range(iters):
        S = oracle.candidates(U)
        mag = np.abs(S)
        mn = mag.min(axis=2)
        m_or = np.argmin(mag, axis=2)
        mg = maps[t].astype(np.int64)
        gmag = np.take_along_axis(mag, mg[..., None], axis=2)[..., 0]
        assert (gmag <= mn + TAU).all(), f"step {t}: GPU selected a non-minimal half window"
        adopted += int((mg != m_or).sum())
        U = oracle.step(U, None if mcf else f64, lam, d, m_forced=maps[t])
    return u, U, adopted


def test_shadow_c1_50_iterations(wmc):
    noisy, _ = wmc_synth.c1()
    u_gpu, U_or, adopted = _shadow(wmc, noisy[0], 1.0, 50)
    err = np.abs(to_np(u_gpu) - U_or).max()
    assert err <= 1e-4, err
    # the fused solver gives the same bits as the recorded steps
    fused = wmc.solve(to_gpu(noisy[0]), 1.0, 50, tuning={"cols": 2, "tsteps": 4, "seg_rows": 32})
    assert torch.equal(fused, u_gpu)
    # free-running FP64 for information: flips decay by lam/(1+lam) per step
    free = oracle.solve(noisy[0].astype(np.float64), lam=1.0, iters=50)
    assert np.abs(to_np(fused) - free).max() <= 1e-3
    print(f"shadow: max err {err:.2e}, adopted GPU choices {adopted}")


def test_shadow_100_iterations_random(wmc):
    f = wmc_synth.random_unit(96, 160, seed=21)
    u_gpu, U_or, _ = _shadow(wmc, f, 1.0, 100)
    assert np.abs(to_np(u_gpu) - U_or).max() <= 1e-4


def test_shadow_flow_mode(wmc):
    noisy, _ = wmc_synth.image(64, 96, 1, 0.05, seed=31)
    u_gpu, U_or, _ = _shadow(wmc, noisy[0], 1.0, 30, mcf=True, delta=0.5)
    assert np.abs(to_np(u_gpu) - U_or).max() <= 1e-4


def test_invariants_on_gpu(wmc):
    """Properties the paper fixes, checked on the GPU result directly."""
    H = W = 40
    y, x = np.mgrid[0:H, 0:W]
    # constant -> fixed point, exactly
    c = to_gpu(np.full((H, W), 0.37))
    assert torch.equal(wmc.solve(c, 1.0, 10, tuning={"cols": 2, "tsteps": 4, "seg_rows": 8}), c)
    # axis-aligned step edge -> fixed point (edge preservation).  Exact when the
    # FP32 arithmetic is exact (dyadic levels); otherwise the column-sum form
    # cancels A against E1 only to rounding, so the edge holds to ~1e-7.
    e = to_gpu(np.where(x >= 17, 0.75, 0.25))
    assert torch.equal(wmc.solve(e, 3.0, 20, tuning={"cols": 1, "tsteps": 8, "seg_rows": 16}), e)
    e = to_gpu(np.where(x >= 17, 0.9, 0.1))
    out = wmc.solve(e, 3.0, 20, tuning={"cols": 1, "tsteps": 8, "seg_rows": 16})
    assert (out - e).abs().max().item() <= 1e-6
    # contrast equivariance, exact for powers of two
    rng = np.random.default_rng(5)
    U = rng.uniform(0, 1, size=(H, W)).astype(np.float32)
    h1 = wmc.compute(to_gpu(U))
    for a in (2.0, -1.0, 0.5):
        assert torch.equal(wmc.compute(to_gpu(a * U)), a * h1)
    # maximum principle with the default step
    f = to_gpu(U)
    out = wmc.solve(f, 4.0, 30, tuning={"cols": 4, "tsteps": 6, "seg_rows": 16})
    assert out.min() >= f.min() and out.max() <= f.max()
    # rectangle: only the four corners move in the first step, to J - delta lam J/6
    R = np.where((x >= 8) & (x < 20) & (y >= 5) & (y < 30), 1.0, 0.0)
    r1 = to_np(wmc.step(to_gpu(R), to_gpu(R), 2.0))
    moved = np.argwhere(r1 != R)
    assert len(moved) == 4
    for yy, xx in moved:
        assert r1[yy, xx] == pytest.approx(1 - (1 / 3) * 2 / 6, abs=1e-6)


@pytest.mark.parametrize("kind", ["random", "integers", "dyadic", "tiny_a", "flat_patches"])
def test_selection_map_variant_is_bitwise_equal(wmc, kind):
    """The selection-map variant (select with index) and the plain kernels
    (select value only) must produce bitwise the same update on inputs rich
    in exact ties, absorbed A and signed zeros (data and flow mode)."""
    rng = np.random.default_rng(["random", "integers", "dyadic", "tiny_a", "flat_patches"].index(kind))
    H, W = 97, 203
    if kind == "random":
        U = rng.uniform(0, 1, size=(2, H, W))
    elif kind == "integers":
        U = rng.integers(0, 4, size=(2, H, W)).astype(np.float64)
    elif kind == "dyadic":
        U = rng.integers(0, 64, size=(2, H, W)) / 16.0
    elif kind == "tiny_a":
        # a smooth quadratic bowl plus 1e-9 jitter: A ~ 0 against large odd parts
        yy, xx = np.mgrid[0:H, 0:W]
        U = np.stack([0.3 * xx + 0.2 * yy + 1e-9 * rng.standard_normal((H, W))] * 2)
    else:
        U = np.repeat(np.repeat(rng.uniform(0, 1, size=(2, H // 8 + 1, W // 8 + 1)), 8, 1), 8, 2)
        U = U[:, :H, :W]
    u = to_gpu(U)
    f = to_gpu(rng.uniform(0, 1, size=(2, H, W)))
    lam = torch.tensor([1.0, 3.0], device="cuda:0")
    for ff in (f, None):
        a = wmc.step(u, ff, lam, dt=0.3)
        b, _ = wmc.step(u, ff, lam, dt=0.3, return_argmin=True)
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))
    h = wmc.compute(u)
    assert torch.isfinite(h).all()
