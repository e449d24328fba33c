"""Pins of the oracle's 3-D adjoint (O14) against facts outside its own
formula:

- the forward step with the selection held fixed is affine in U, so
  <J dU, g> computed through the forward step must equal <dU, J^T g>
  computed by the adjoint (the dot-product identity); this fixes every tap's
  orientation, the replicate-border fold and the keep / coef factors, on
  tiny volumes where every voxel touches a border;
- central finite differences in f, lam, u0 of the forward solve (selections
  do not move for small perturbations of random inputs) fix the data-term
  factor, the delta'(lam) term of the default step and the split between
  dL/df and dL/dU^0 at lam != 1, where delta != 1 - delta.

The adjoint itself is this build's derivation (the paper leaves the
gradient of the regulariser open, end of Sec. 3); the operator is the 3-D
extension of the conclusion (Sec. 6), built as Sec. 4.1 builds the 2-D one."""
import numpy as np
import pytest

import oracle

SHAPES = [(1, 1, 1), (1, 2, 3), (2, 1, 1), (2, 3, 4), (3, 3, 3), (4, 1, 5), (5, 6, 7)]


def _affine_jvp(U, dU, f, lam, delta, m):
    """J dU of the step with the selection m held: the step is affine in U,
    so the difference of two forward steps is exactly linear in dU."""
    a = oracle.step3(U + dU, f, lam, delta, m_forced=m)
    b = oracle.step3(U, f, lam, delta, m_forced=m)
    return a - b


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("mode", ["data", "flow"])
def test_adjoint_dot_product_identity(shape, mode):
    rng = np.random.default_rng(sum(shape) + (7 if mode == "flow" else 0))
    U = rng.uniform(0, 1, shape)
    f = rng.uniform(0, 1, shape) if mode == "data" else None
    lam, delta = (2.5, 1.0 / 3.5) if mode == "data" else (1.0, 0.3)
    _, m = oracle.step3(U, f, lam, delta, return_argmin=True)
    dU = rng.normal(size=shape)
    g = rng.normal(size=shape)
    jv = _affine_jvp(U, dU, f, lam, delta, m)
    gU, _, _ = oracle.step3_adjoint(U, g, f, lam, delta, delta_from_lam=False, m_forced=m)
    lhs = float(np.sum(jv * g))
    rhs = float(np.sum(dU * gU))
    assert abs(lhs - rhs) <= 1e-11 * (1.0 + abs(lhs)), (lhs, rhs)


def test_adjoint_columns_against_unit_vectors():
    """Every column of J^T: J^T e_v equals the forward response row, so the
    adjoint of a unit cotangent at v is dU'(v)/dU read off the forward step
    (all 60 voxels of a 3x4x5 volume, data mode, lam = 0.3)."""
    rng = np.random.default_rng(11)
    shape = (3, 4, 5)
    U = rng.uniform(0, 1, shape)
    f = rng.uniform(0, 1, shape)
    lam = 0.3
    delta = 1.0 / (1.0 + lam)
    _, m = oracle.step3(U, f, lam, delta, return_argmin=True)
    n = U.size
    J = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        J[:, j] = _affine_jvp(U, e.reshape(shape), f, lam, delta, m).ravel()
    for v in range(n):
        g = np.zeros(n)
        g[v] = 1.0
        gU, _, _ = oracle.step3_adjoint(U, g.reshape(shape), f, lam, delta, delta_from_lam=False,
                                        m_forced=m)
        assert np.allclose(gU.ravel(), J[v], atol=1e-13)


@pytest.mark.parametrize("lam", [0.3, 2.5])
@pytest.mark.parametrize("default_step", [True, False])
def test_one_step_f_and_lam_by_finite_differences(lam, default_step):
    rng = np.random.default_rng(int(lam * 10) + default_step)
    shape = (3, 4, 5)
    U = rng.uniform(0, 1, shape)
    f = rng.uniform(0, 1, shape)
    g = rng.normal(size=shape)
    dt = None if default_step else 0.37

    def loss(fv, lv):
        d = 1.0 / (1.0 + lv) if dt is None else dt
        return float(np.sum(g * oracle.step3(U, fv, lv, d)))

    d0 = 1.0 / (1.0 + lam) if dt is None else dt
    _, gf, glam = oracle.step3_adjoint(U, g, f, lam, d0, delta_from_lam=dt is None)
    eps = 1e-6
    for idx in [(0, 0, 0), (2, 3, 4), (1, 2, 2), (0, 3, 1)]:
        fp, fm = f.copy(), f.copy()
        fp[idx] += eps
        fm[idx] -= eps
        fd = (loss(fp, lam) - loss(fm, lam)) / (2 * eps)
        assert abs(fd - gf[idx]) <= 1e-8, (idx, fd, gf[idx])
        assert abs(gf[idx] - d0 * g[idx]) <= 1e-15
    fd = (loss(f, lam + eps) - loss(f, lam - eps)) / (2 * eps)
    assert abs(fd - glam) <= 1e-7 * (1.0 + abs(glam)), (fd, glam)


def _fd_solve(fun, x, idx, eps=1e-6):
    xp, xm = x.copy(), x.copy()
    xp[idx] += eps
    xm[idx] -= eps
    return (fun(xp) - fun(xm)) / (2 * eps)


@pytest.mark.parametrize("lam", [0.3, 2.5])
def test_k_step_gradients_split_by_finite_differences(lam):
    """K = 3 steps from u0 != f: dL/df (data term only) and dL/dU^0 each
    against FD with the other input fixed, dL/dlam with the default step."""
    rng = np.random.default_rng(int(lam * 100))
    shape = (3, 4, 5)
    f = rng.uniform(0, 1, shape)
    u0 = rng.uniform(0, 1, shape)
    gK = rng.normal(size=shape)
    K = 3
    r = oracle.solve3_adjoint(gK, f, lam, K, u0=u0)
    assert np.allclose(r["UK"], oracle.solve3(f, lam, K, u0=u0), atol=1e-14)

    def L(fv=f, uv=u0, lv=lam):
        return float(np.sum(gK * oracle.solve3(fv, lv, K, u0=uv)))

    for idx in [(0, 0, 0), (2, 3, 4), (1, 1, 2), (2, 0, 3), (0, 2, 4)]:
        assert abs(_fd_solve(lambda x: L(fv=x), f, idx) - r["gf"][idx]) <= 1e-7
        assert abs(_fd_solve(lambda x: L(uv=x), u0, idx) - r["gu0"][idx]) <= 1e-7
    eps = 1e-6
    fd = (L(lv=lam + eps) - L(lv=lam - eps)) / (2 * eps)
    assert abs(fd - r["glam"]) <= 1e-6 * (1.0 + abs(r["glam"])), (fd, r["glam"])


def test_k_step_from_f_total_gradient():
    """From U^0 = f the total dL/df is gf + gu0 (both paths)."""
    rng = np.random.default_rng(5)
    shape = (2, 3, 6)
    f = rng.uniform(0, 1, shape)
    gK = rng.normal(size=shape)
    lam, K = 2.5, 4
    r = oracle.solve3_adjoint(gK, f, lam, K)
    tot = r["gf"] + r["gu0"]
    for idx in [(0, 0, 0), (1, 2, 5), (0, 1, 3), (1, 0, 1)]:
        fd = _fd_solve(lambda x: float(np.sum(gK * oracle.solve3(x, lam, K))), f, idx)
        assert abs(fd - tot[idx]) <= 1e-7


def test_flow_mode_by_finite_differences():
    rng = np.random.default_rng(9)
    shape = (3, 3, 4)
    u0 = rng.uniform(0, 1, shape)
    gK = rng.normal(size=shape)
    K, d = 3, 0.2
    r = oracle.solve3_adjoint(gK, None, 1.0, K, delta=d, u0=u0)
    assert r["gf"] is None and r["glam"] == 0.0
    for idx in [(0, 0, 0), (2, 2, 3), (1, 1, 1), (2, 0, 2)]:
        fd = _fd_solve(lambda x: float(np.sum(gK * oracle.solve3(None, 1.0, K, delta=d, u0=x))),
                       u0, idx)
        assert abs(fd - r["gu0"][idx]) <= 1e-7


def test_constant_volume_gradient_is_plain_relaxation():
    """On a constant U every candidate is 0 and the first kernel is selected;
    the operator still acts on the cotangent: with lam = 0 the adjoint is
    keep * g exactly (no regulariser term), and with the data term at any
    lam the f-gradient is delta * g."""
    shape = (2, 3, 4)
    U = np.full(shape, 0.4)
    g = np.random.default_rng(1).normal(size=shape)
    gU, gf, glam = oracle.step3_adjoint(U, g, U, 0.0, 0.5, delta_from_lam=False)
    assert np.array_equal(gU, 0.5 * g)
    assert np.array_equal(gf, 0.5 * g)
    assert glam == 0.0


def test_step3_with_forced_selection_against_library_candidates():
    """The step with a forced selection is the update through that
    candidate: U + delta((f - U) + lam S_m / 56) with S_m from an independent
    evaluation (scipy's correlation with replicate borders); without forcing
    it is the one-step solve, and its recorded selection is the first
    minimum of those candidates."""
    from scipy import ndimage
    rng = np.random.default_rng(17)
    shape = (4, 5, 6)
    U = rng.uniform(0, 1, shape)
    f = rng.uniform(0, 1, shape)
    lam, delta = 0.8, 0.45
    S = np.stack([ndimage.correlate(U, k.astype(np.float64), mode="nearest")
                  for k in oracle.kernels3()])
    out, m = oracle.step3(U, f, lam, delta, return_argmin=True)
    assert np.allclose(out, oracle.solve3(f, lam, 1, delta=delta, u0=U), atol=1e-15)
    assert np.array_equal(m, np.argmin(np.abs(S), axis=0))
    forced = rng.integers(0, 18, size=shape).astype(np.int8)
    got, used = oracle.step3(U, f, lam, delta, m_forced=forced, return_argmin=True)
    Sm = np.take_along_axis(S, forced[None].astype(np.int64), axis=0)[0]
    assert np.array_equal(used, forced)
    assert np.allclose(got, U + delta * ((f - U) + lam * Sm / 56.0), atol=1e-13)
    # flow mode
    got = oracle.step3(U, None, 1.0, 0.3, m_forced=forced)
    assert np.allclose(got, U + 0.3 * Sm / 56.0, atol=1e-13)
