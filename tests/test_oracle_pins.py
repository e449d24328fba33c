"""Pins for the FP64 oracle: each test checks the oracle against something other
than itself -- values the paper prints, closed forms derived from the printed
kernels, invariants the paper states, or brute force -- so that a dropped
term, a wrong sign, a transposed kernel or a wrong tie rule fails here.

Notation: S_i = 12 d_i (the "x12 domain", integer weights), H_d = S_m / 12,
x = column, y = row (downwards), the printed top kernel row sits on row y-1.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import wmc_synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_kernels(name):
    """Parse a golden kernel file into {label: 3x3 Fraction array}."""
    out, label, rows = {}, None, []
    with open(os.path.join(GOLD, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            toks = line.split()
            if len(toks) == 1 and not any(ch.isdigit() for ch in toks[0][:1]) and toks[0][0] != "-":
                label, rows = toks[0], []
                out[label] = rows
            else:
                rows.append([Fraction(t) for t in toks])
    return out


# ---------------------------------------------------------------------------------------
# P1 -- the kernel table
# ---------------------------------------------------------------------------------------

def test_table_matches_printed_kernels():
    """The oracle's x12 table equals the kernels printed in Sec. 4.2."""
    printed = _read_kernels("half_window_kernels.txt")
    table = oracle.kernel_table()
    for i in range(8):
        k = printed[f"h{i + 1}"]
        for r in range(3):
            for c in range(3):
                assert Fraction(int(table[i, r, c]), 12) == k[r][c], (i, r, c)


def _half_window_from_k4(direction):
    """Build a half-window kernel from k4 alone (Neumann/reflection condition of
    Sec. 4.1.2).  direction: normal (dy, dx) pointing *out of* the half window, one of
    the 8 compass directions.  Taps with a positive component along the normal
    are outside; their reflection across the line through the centre that is
    perpendicular to the normal carries their weight inside."""
    k4 = _read_kernels("laplace_kernels.txt")["k4"]
    ny, nx = direction
    out = [[Fraction(0)] * 3 for _ in range(3)]
    for r in range(3):
        for c in range(3):
            oy, ox = r - 1, c - 1
            dot = oy * ny + ox * nx
            if dot <= 0:
                out[r][c] += k4[r][c]
            else:
                # reflect o across the line perpendicular to n: o - 2 (o.n / n.n) n
                nn = ny * ny + nx * nx
                ry = oy - Fraction(2 * dot, nn) * ny
                rx = ox - Fraction(2 * dot, nn) * nx
                assert ry.denominator == 1 and rx.denominator == 1
                out[int(ry) + 1][int(rx) + 1] += k4[r][c]
    return out


# outward normals: h1 left half window -> the cut removes the right column, etc.
_OUTWARD = {
    1: (0, 1),    # left window, right side cut away
    2: (1, 0),    # top window, bottom cut away
    3: (0, -1),   # right window
    4: (-1, 0),   # bottom window
    5: (1, 1),    # top-left window, bottom-right cut away
    6: (1, -1),   # top-right window
    7: (-1, -1),  # bottom-right window
    8: (-1, 1),   # bottom-left window
}


@pytest.mark.parametrize("i", range(1, 9))
def test_kernels_are_k4_with_reflection(i):
    """Independent derivation: folding the most isotropic Laplacian k4 of
    eq. (kernel3) onto each half window reproduces the table exactly."""
    derived = _half_window_from_k4(_OUTWARD[i])
    table = oracle.kernel_table()
    for r in range(3):
        for c in range(3):
            assert Fraction(int(table[i - 1, r, c]), 12) == derived[r][c], (i, r, c)


def test_table_structure():
    t = oracle.kernel_table()
    assert (t.sum(axis=(1, 2)) == 0).all()
    assert (t[:, 1, 1] == -12).all()
    assert ((t != 0).sum(axis=(1, 2)) == 6).all()           # six taps per half window
    k4x12 = np.array([[1, 2, 1], [2, -12, 2], [1, 2, 1]])
    for a, b in [(0, 2), (1, 3), (4, 6), (5, 7)]:           # opposite windows
        s = t[a] + t[b]
        off = np.ones((3, 3), bool)
        off[1, 1] = False
        assert (s[off] == 2 * k4x12[off]).all()
        assert (t[a] == np.rot90(t[b], 2)).all()           # closed under 180 degrees


def test_appendix_kernels_give_same_set():
    """The Appendix A kernels (true convolution = correlation with the 180-degree
    rotated kernel) are the printed set, in the order h3 h1 h4 h2 h7 h8 h6 h5."""
    base = _read_kernels("appendix_base_kernels.txt")
    lk = oracle.listing_kernels()
    b1 = np.array([[float(v) for v in row] for row in base["base1"][:3]]) / 6.0
    b2 = np.array([[float(v) for v in row] for row in base["base2"][:3]]) / 12.0
    assert np.array_equal(lk[0], b1) and np.array_equal(lk[4], b2)
    t = oracle.kernel_table() / 12.0
    order = [3, 1, 4, 2, 7, 8, 6, 5]
    for s in range(8):
        assert np.allclose(np.rot90(lk[s], 2), t[order[s] - 1], atol=0, rtol=0), s


# ---------------------------------------------------------------------------------------
# P2 -- constants
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (6, 1), (2, 2), (5, 9), (17, 13)])
def test_constant_gives_zero_everywhere(shape):
    rng = np.random.default_rng(1)
    for c in rng.uniform(-3, 3, size=4):
        U = np.full(shape, c)
        Hd = oracle.compute(U)
        assert np.all(Hd == 0.0)
        assert np.all(oracle.candidates(U) == 0.0)


# ---------------------------------------------------------------------------------------
# P3/P4 -- planes and quadratics: closed forms from the identities
#   A  = 12 k4*U       = 4 Lap U = 8(a + c)
#   E1 = (h1-k4)*U x12 = -8 U_x,  E2 = -8 U_y,
#   E5 = -6 (U_x + U_y),          E6 = 6 (U_x - U_y)
#   S = [A+E1, A+E2, A-E1, A-E2, A+E5, A+E6, A-E5, A-E6]
# ---------------------------------------------------------------------------------------

def _closed_form_candidates(a, b, c, d, e, y, x):
    ux = 2 * a * x + b * y + d
    uy = b * x + 2 * c * y + e
    A = 8 * (a + c)
    E1, E2, E5, E6 = -8 * ux, -8 * uy, -6 * (ux + uy), 6 * (ux - uy)
    return [A + E1, A + E2, A - E1, A - E2, A + E5, A + E6, A - E5, A - E6]


def _first_min(vals):
    m = 0
    for i in range(1, len(vals)):
        if abs(vals[i]) < abs(vals[m]):
            m = i
    return m


def _quadratic(a, b, c, d, e, g, H, W):
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    return a * x * x + b * x * y + c * y * y + d * x + e * y + g


def test_quadratic_closed_form_all_candidates():
    rng = np.random.default_rng(7)
    H, W = 11, 13
    for _ in range(40):
        a, b, c, d, e, g = (int(v) for v in rng.integers(-3, 4, size=6))
        U = _quadratic(a, b, c, d, e, g, H, W)
        S = oracle.candidates(U)
        Hd, m = oracle.compute(U, return_argmin=True)
        for y in range(1, H - 1):
            for x in range(1, W - 1):
                want = _closed_form_candidates(a, b, c, d, e, y, x)
                assert list(S[y, x]) == [float(v) for v in want], (a, b, c, d, e, y, x)
                k = _first_min(want)
                assert m[y, x] == k
                assert Hd[y, x] == want[k] / 12.0


def test_plane_closed_form_and_tie_sign():
    """General plane beta x + gamma y: |H_d| = min(2/3|b|, 2/3|g|, 1/2|b+g|, 1/2|b-g|)
    in the interior; the sign is the lowest-index member of the tied set."""
    H, W = 7, 8
    vals = [Fraction(k, 4) for k in range(-12, 13)]
    for beta in vals[::3]:
        for gamma in vals[::2]:
            U = _quadratic(0, 0, 0, float(beta), float(gamma), 0.25, H, W)
            Hd = oracle.compute(U)
            mag = min(Fraction(2, 3) * abs(beta), Fraction(2, 3) * abs(gamma),
                      abs(beta + gamma) / 2, abs(beta - gamma) / 2)
            cand = _closed_form_candidates(0, 0, 0, float(beta), float(gamma), 3, 3)
            want = cand[_first_min(cand)] / 12.0
            assert abs(want) == pytest.approx(float(mag), abs=1e-15)
            inner = Hd[1:-1, 1:-1]
            assert np.all(inner == want), (beta, gamma)


def test_aligned_planes_are_zero():
    H, W = 9, 9
    for beta, gamma in [(0.5, 0), (0, -1.25), (0.75, 0.75), (-2, 2), (3, 0)]:
        U = _quadratic(0, 0, 0, beta, gamma, 0.0, H, W)
        assert np.all(oracle.compute(U)[1:-1, 1:-1] == 0.0)


def test_paraboloid_worked_values():
    """U = (x-cx)^2 + (y-cy)^2 around a pixel centre; hand-derived values at
    offsets (dx, dy), including the exact opposite-sign tie at (2, 2) whose
    canonical (first index) winner is h1 -> -4/3."""
    H = W = 11
    c = 5
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    U = (x - c) ** 2 + (y - c) ** 2
    Hd, m = oracle.compute(U, return_argmin=True)
    expect = {(0, 0): 4 / 3, (1, 0): 0.0, (2, 0): -2 / 3, (3, 0): 4 / 3, (1, 1): 0.0,
              (2, 1): 0.0, (2, 2): -4 / 3}
    for (dx, dy), v in expect.items():
        assert Hd[c + dy, c + dx] == pytest.approx(v, abs=1e-15), (dx, dy)
    assert m[c + 2, c + 2] == 0  # h1 wins the tie


# ---------------------------------------------------------------------------------------
# P5 -- spherical cap apex (all eight responses equal by symmetry)
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("R", [3.0, 10.0, 40.0])
def test_spherical_cap_apex(R):
    n = 5 if R < 4 else 7
    c = n // 2
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    U = np.sqrt(R * R - (x - c) ** 2 - (y - c) ** 2)
    S = oracle.candidates(U)[c, c]
    want = (2 / 3) * (np.sqrt(R * R - 1) - R) + (1 / 3) * (np.sqrt(R * R - 2) - R)
    assert np.allclose(S / 12.0, want, rtol=1e-12, atol=1e-14)
    assert oracle.compute(U)[c, c] == pytest.approx(want, rel=1e-12)
    if R == 10.0:
        assert want == pytest.approx(-0.066919, abs=5e-7)
    # "becomes the Laplace operator" at the extremum (Sec. 3.3): k4 applied there
    k4 = np.array([[1, 2, 1], [2, -12, 2], [1, 2, 1]]) / 12.0
    assert oracle.compute(U)[c, c] == pytest.approx(float((k4 * U[c - 1:c + 2, c - 1:c + 2]).sum()),
                                                     rel=1e-12)


# ---------------------------------------------------------------------------------------
# P6 -- rectilinear shapes: the exact discrete form of sampling/scale invariance
# ---------------------------------------------------------------------------------------

def _rect(H, W, y0, y1, x0, x1, J, bg=0.0):
    U = np.full((H, W), bg)
    U[y0:y1, x0:x1] = bg + J
    return U


def test_rectangle_corners_only():
    rng = np.random.default_rng(3)
    for _ in range(25):
        h, w = (int(v) for v in rng.integers(2, 9, size=2))
        H, W = h + int(rng.integers(4, 8)), w + int(rng.integers(4, 8))
        y0, x0 = int(rng.integers(2, H - h - 1)), int(rng.integers(2, W - w - 1))
        J = float(rng.choice([0.5, -0.75, 1.0, 0.125, -2.0]))
        U = _rect(H, W, y0, y0 + h, x0, x0 + w, J, bg=0.25)
        Hd = oracle.compute(U)
        corners = {(y0, x0), (y0, x0 + w - 1), (y0 + h - 1, x0), (y0 + h - 1, x0 + w - 1)}
        for yy in range(H):
            for xx in range(W):
                want = -J / 6 if (yy, xx) in corners else 0.0
                assert Hd[yy, xx] == pytest.approx(want, abs=1e-15), (yy, xx)
        assert Hd.sum() == pytest.approx(-2 * J / 3, abs=1e-13)
        assert np.abs(Hd).sum() == pytest.approx(2 * abs(J) / 3, abs=1e-13)


@pytest.mark.parametrize("scale", [1, 2, 3, 5])
def test_rectangle_total_invariant_under_upsampling(scale):
    """Nearest-neighbour integer upsampling (a change of sampling rate and
    scale of the same geometry) leaves sum |H_d| unchanged."""
    U = _rect(12, 14, 3, 8, 4, 10, 1.0)
    Uk = np.kron(U, np.ones((scale, scale)))
    assert np.abs(oracle.compute(Uk)).sum() == pytest.approx(2 / 3, abs=1e-13)


def test_diagonal_staircase_edge_zero():
    H = W = 12
    y, x = np.mgrid[0:H, 0:W]
    for k in [6, 9, 13]:
        # interior only: the replicate border bends a diagonal edge where it
        # meets the image boundary
        U = np.where(x + y >= k, 1.0, 0.0)
        assert np.all(oracle.compute(U)[1:-1, 1:-1] == 0.0)
        U2 = np.where(x - y >= k - 10, 0.5, -0.5)
        assert np.all(oracle.compute(U2)[1:-1, 1:-1] == 0.0)


@pytest.mark.parametrize("mcf", [False, True])
def test_step_edges_are_fixed_points(mcf):
    H, W = 10, 12
    y, x = np.mgrid[0:H, 0:W]
    # axis-aligned step edges stay straight under the replicate border
    for U in [np.where(x >= 5, 1.0, 0.0), np.where(y >= 3, 0.75, 0.25)]:
        out = oracle.solve(None if mcf else U, lam=2.0, iters=7, u0=U)
        assert np.array_equal(out, U)
    # a 45-degree edge meets the border at a bend; one step leaves every pixel
    # at distance >= 2 from the border unchanged
    U = np.where(x - y >= 2, 1.0, 0.0)
    out = oracle.step(U, None if mcf else U, lam=2.0)
    assert np.array_equal(out[2:-2, 2:-2], U[2:-2, 2:-2])


# ---------------------------------------------------------------------------------------
# P7 -- contrast equivariance (eq. (scale))
# ---------------------------------------------------------------------------------------

def test_contrast_equivariance_exact_for_powers_of_two():
    rng = np.random.default_rng(5)
    U = rng.uniform(0, 1, size=(15, 17))
    Hd = oracle.compute(U)
    for alpha in [2.0, 0.5, -1.0, -4.0, 0.125]:
        assert np.array_equal(oracle.compute(alpha * U), alpha * Hd)


def test_contrast_equivariance_general():
    rng = np.random.default_rng(6)
    U = rng.uniform(0, 1, size=(15, 17))
    Hd = oracle.compute(U)
    for alpha, c in [(3.7, 0.2), (-0.3, 5.0), (1e3, -7.0)]:
        got = oracle.compute(alpha * U + c)
        assert np.allclose(got, alpha * Hd, rtol=1e-9, atol=1e-12 * max(1, abs(alpha) + abs(c)))


def test_solver_contrast_equivariance():
    rng = np.random.default_rng(8)
    f = rng.uniform(0, 1, size=(12, 10))
    base = oracle.solve(f, lam=1.5, iters=9)
    for alpha in [2.0, -0.5]:
        assert np.array_equal(oracle.solve(alpha * f, lam=1.5, iters=9), alpha * base)
    got = oracle.solve(3.0 * f + 0.7, lam=1.5, iters=9)
    assert np.allclose(got, 3.0 * base + 0.7, atol=1e-12)


# ---------------------------------------------------------------------------------------
# P8 -- the column/row-sum form agrees with the direct eight-kernel sum
# ---------------------------------------------------------------------------------------

def _ae_form(U):
    """Appendix-B-style identities, written independently of the oracle:
    column sums colW/colC/colE, row sums rowN/rowS, A = binomial - 16C,
    E1 = colW-colE, E2 = rowN-rowS, E5 = (E1+E2)/2 + (N-S) + (W-E),
    E6 = (E2-E1)/2 + (N-S) + (E-W)."""
    P = np.pad(U, 1, mode="edge")
    NW, N, NE = P[:-2, :-2], P[:-2, 1:-1], P[:-2, 2:]
    Wv, C, E = P[1:-1, :-2], P[1:-1, 1:-1], P[1:-1, 2:]
    SW, S, SE = P[2:, :-2], P[2:, 1:-1], P[2:, 2:]
    colW, colC, colE = NW + 2 * Wv + SW, N + 2 * C + S, NE + 2 * E + SE
    rowN, rowS = NW + 2 * N + NE, SW + 2 * S + SE
    A = colW + 2 * colC + colE - 16 * C
    E1, E2 = colW - colE, rowN - rowS
    E5 = (E1 + E2) / 2 + (N - S) + (Wv - E)
    E6 = (E2 - E1) / 2 + (N - S) + (E - Wv)
    return np.stack([A + E1, A + E2, A - E1, A - E2, A + E5, A + E6, A - E5, A - E6], axis=-1)


def test_ae_form_matches_direct_random():
    rng = np.random.default_rng(9)
    for shape in [(1, 1), (1, 5), (4, 1), (9, 14), (32, 31)]:
        U = rng.uniform(0, 1, size=shape)
        assert np.allclose(_ae_form(U), oracle.candidates(U), atol=1e-13, rtol=0)


def test_ae_form_matches_direct_dyadic_exact():
    rng = np.random.default_rng(10)
    U = rng.integers(-64, 64, size=(20, 23)) / 16.0
    assert np.array_equal(_ae_form(U), oracle.candidates(U))


# ---------------------------------------------------------------------------------------
# border rule and listing mode (reading of the Neumann condition vs. Appendix A)
# ---------------------------------------------------------------------------------------

def test_listing_mode_constant_corners():
    """Zero padding (Appendix A) gives -c/6 at the four image corners of a
    constant image and 0 elsewhere; the replicate border gives 0 everywhere."""
    c = 0.75
    U = np.full((6, 7), c)
    Hd = oracle.listing(U)
    want = np.zeros_like(U)
    for yy, xx in [(0, 0), (0, 6), (5, 0), (5, 6)]:
        want[yy, xx] = -c / 6
    assert np.allclose(Hd, want, atol=1e-15)


def test_listing_mode_interior_same_values():
    """Away from the border both modes see the same eight responses, so the
    selected magnitude agrees everywhere and the value wherever no opposite-
    sign exact tie exists."""
    rng = np.random.default_rng(11)
    U = rng.uniform(0, 1, size=(16, 16))
    a = oracle.compute(U)[1:-1, 1:-1]
    b = oracle.listing(U)[1:-1, 1:-1]
    assert np.allclose(np.abs(a), np.abs(b), atol=1e-15)
    assert np.allclose(a, b, atol=1e-15)


# ---------------------------------------------------------------------------------------
# P9 -- solver invariants
# ---------------------------------------------------------------------------------------

def test_maximum_principle():
    rng = np.random.default_rng(12)
    f = rng.uniform(0, 1, size=(24, 20))
    u0 = rng.uniform(0.2, 0.9, size=f.shape)
    for lam in [0.5, 1.0, 4.0]:
        for delta in [1 / (1 + lam), 0.5 / (1 + lam)]:
            U = u0.copy()
            lo, hi = min(f.min(), u0.min()), max(f.max(), u0.max())
            for _ in range(15):
                U = oracle.step(U, f, lam, delta)
                assert U.min() >= lo - 1e-15 and U.max() <= hi + 1e-15


def test_lambda_zero_closed_form():
    rng = np.random.default_rng(13)
    f = rng.uniform(0, 1, size=(9, 9))
    u0 = rng.uniform(0, 1, size=(9, 9))
    for delta in [1.0, 0.5, 0.3]:
        t = 6
        got = oracle.solve(f, lam=0.0, iters=t, delta=delta, u0=u0)
        assert np.allclose(got, f + (1 - delta) ** t * (u0 - f), atol=1e-14)


def test_first_step_on_rectangle():
    lam, J = 2.0, 1.0
    U = _rect(14, 15, 4, 9, 3, 11, J)
    delta = 1 / (1 + lam)
    U1 = oracle.step(U, U, lam, delta)
    diff = U1 != U
    corners = [(4, 3), (4, 10), (8, 3), (8, 10)]
    assert diff.sum() == 4
    for c in corners:
        assert U1[c] == pytest.approx(J - delta * lam * J / 6, abs=1e-15)


def test_resume_is_exact():
    rng = np.random.default_rng(14)
    f = rng.uniform(0, 1, size=(18, 21))
    full = oracle.solve(f, lam=1.0, iters=25)
    part = oracle.solve(f, lam=1.0, iters=15, u0=oracle.solve(f, lam=1.0, iters=10))
    assert np.array_equal(full, part)


def test_mcf_shrinks_total_curvature_of_rectangle():
    """MCF (eq. (MCF)) with small delta rounds rectangle corners: only the
    corners move, towards the background, and no new extrema appear."""
    U = _rect(12, 12, 3, 9, 3, 9, 1.0)
    U1 = oracle.step(U, None, delta=0.5)
    assert U1.max() <= 1.0 and U1.min() >= 0.0
    assert (U1 != U).sum() == 4


# ---------------------------------------------------------------------------------------
# P10 -- the adjoint: dot-product test with frozen selection, finite differences
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("mcf", [False, True])
def test_adjoint_dot_product(mcf):
    rng = np.random.default_rng(15)
    for shape in [(1, 1), (1, 6), (5, 1), (7, 9), (12, 11)]:
        U = rng.uniform(0, 1, size=shape)
        f = None if mcf else rng.uniform(0, 1, size=shape)
        lam, delta = 1.3, 0.37
        _, m = oracle.step(U, f, lam, delta, return_argmin=True)
        v = rng.standard_normal(shape)
        w = rng.standard_normal(shape)
        # the map is affine in U with m frozen: J v = step(U+v) - step(U)
        Jv = oracle.step(U + v, f, lam, delta, m_forced=m) - oracle.step(U, f, lam, delta, m_forced=m)
        gU, _, _ = oracle.step_adjoint(U, w, f, lam, delta, delta_from_lam=False, m_forced=m)
        lhs, rhs = float((Jv * w).sum()), float((v * gU).sum())
        assert lhs == pytest.approx(rhs, rel=1e-12, abs=1e-12)


def _loss(UK, target):
    return 0.5 * float(((UK - target) ** 2).sum())


def test_adjoint_vs_finite_differences():
    rng = np.random.default_rng(16)
    H, W, K, lam = 8, 9, 6, 1.0
    f = rng.uniform(0, 1, size=(H, W))
    target = rng.uniform(0, 1, size=(H, W))
    res = oracle.solve_adjoint(np.zeros((H, W)), f, lam, K)  # for UK
    UK = res["UK"]
    res = oracle.solve_adjoint(UK - target, f, lam, K)
    gf_total = res["gf"] + res["gu0"]

    def run(ff, ll):
        return oracle.solve(ff, lam=ll, iters=K)

    h = 1e-6
    checked = 0
    for _ in range(20):
        y, x = int(rng.integers(H)), int(rng.integers(W))
        fp, fm = f.copy(), f.copy()
        fp[y, x] += h
        fm[y, x] -= h
        # skip perturbations that change a selection anywhere along the path
        same = True
        up, um = fp.copy(), fm.copy()
        for _t in range(K):
            _, mp = oracle.step(up, fp, lam, return_argmin=True)
            _, mm = oracle.step(um, fm, lam, return_argmin=True)
            if not np.array_equal(mp, mm):
                same = False
                break
            up, um = oracle.step(up, fp, lam), oracle.step(um, fm, lam)
        if not same:
            continue
        fd = (_loss(run(fp, lam), target) - _loss(run(fm, lam), target)) / (2 * h)
        assert fd == pytest.approx(gf_total[y, x], rel=1e-5, abs=1e-8)
        checked += 1
    assert checked >= 10
    fdl = (_loss(run(f, lam + h), target) - _loss(run(f, lam - h), target)) / (2 * h)
    assert fdl == pytest.approx(res["glam"], rel=1e-5, abs=1e-8)


def test_adjoint_fixed_delta_lambda_gradient():
    """With an explicit step size (not 1/(1+lam)) only delta*H_d enters dL/dlam."""
    rng = np.random.default_rng(17)
    H, W, K = 7, 7, 4
    f = rng.uniform(0, 1, size=(H, W))
    target = rng.uniform(0, 1, size=(H, W))
    lam, delta, h = 0.8, 0.3, 1e-6
    UK = oracle.solve(f, lam=lam, iters=K, delta=delta)
    res = oracle.solve_adjoint(UK - target, f, lam, K, delta=delta, delta_from_lam=False)
    fd = (_loss(oracle.solve(f, lam=lam + h, iters=K, delta=delta), target)
          - _loss(oracle.solve(f, lam=lam - h, iters=K, delta=delta), target)) / (2 * h)
    assert fd == pytest.approx(res["glam"], rel=1e-5, abs=1e-9)


# Away from lam = 1 the data-term factors differ: delta = 1/(1+lam) != 1 - delta and
# delta^2 != delta(1 - delta), so a swapped keep factor, a (1 - delta) in place of
# delta in dL/df or a wrong derivative of the default step fails here.  Starting
# from u0 != f separates dL/df (the data term, Sec. 5.2 update) from dL/dU^0.

def _path_maps(f, u0, lam, delta, K):
    """Selection maps along a K-step solve from u0 (f None: flow)."""
    maps, u = [], u0.copy()
    for _ in range(K):
        u, m = oracle.step(u, f, lam, delta, return_argmin=True)
        maps.append(m)
    return maps


def _fd_pins(f, u0, target, lam, delta, K, delta_follows_lam, rng, n_pix=14):
    """Central differences (h = 1e-6, FP64) of L = 1/2 ||U^K - target||^2 with
    respect to single entries of f and of u0 separately, and to lam, against
    the oracle adjoint.  Perturbations that change a selection anywhere along
    the path are skipped (the map is piecewise affine)."""
    H, W = u0.shape
    h = 1e-6

    def dlt(ll):
        return 1.0 / (1.0 + ll) if delta_follows_lam else delta

    def run(ff, uu, ll):
        return oracle.solve(ff, lam=ll, iters=K, delta=dlt(ll), u0=uu)

    UK = run(f, u0, lam)
    res = oracle.solve_adjoint(UK - target, f, lam, K, delta=dlt(lam), u0=u0,
                               delta_from_lam=delta_follows_lam)
    base = _path_maps(f, u0, lam, dlt(lam), K)
    checked = {"f": 0, "u0": 0}
    for which in ("f", "u0"):
        if which == "f" and f is None:
            continue
        for _ in range(n_pix):
            y, x = int(rng.integers(H)), int(rng.integers(W))
            runs = []
            for sgn in (1.0, -1.0):
                ff = None if f is None else f.copy()
                uu = u0.copy()
                (ff if which == "f" else uu)[y, x] += sgn * h
                runs.append((ff, uu))
            if any(not all(np.array_equal(a, b) for a, b in
                           zip(_path_maps(ff, uu, lam, dlt(lam), K), base)) for ff, uu in runs):
                continue
            fd = (_loss(run(*runs[0], lam), target) - _loss(run(*runs[1], lam), target)) / (2 * h)
            want = res["gf"][y, x] if which == "f" else res["gu0"][y, x]
            assert fd == pytest.approx(want, rel=1e-5, abs=1e-9), (which, y, x)
            checked[which] += 1
    if f is not None:
        assert checked["f"] >= n_pix // 2
        fdl = (_loss(run(f, u0, lam + h), target) - _loss(run(f, u0, lam - h), target)) / (2 * h)
        assert fdl == pytest.approx(res["glam"], rel=1e-5, abs=1e-9)
    assert checked["u0"] >= n_pix // 2
    return res


@pytest.mark.parametrize("lam", [0.3, 2.5])
def test_adjoint_fd_default_step_away_from_lambda_one(lam):
    rng = np.random.default_rng(int(lam * 10) + 30)
    H, W, K = 8, 9, 5
    f = rng.uniform(0, 1, size=(H, W))
    u0 = rng.uniform(0, 1, size=(H, W))
    target = rng.uniform(0, 1, size=(H, W))
    res = _fd_pins(f, u0, target, lam, None, K, True, rng)
    # the two parts really differ: dL/df is not dL/dU^0 (u0 != f)
    assert np.abs(res["gf"] - res["gu0"]).max() > 1e-3


def test_adjoint_fd_default_step_u0_is_f_lambda_2_5():
    """Starting from U^0 = f, dL/df is the data-term part plus dL/dU^0."""
    rng = np.random.default_rng(33)
    H, W, K, lam = 7, 10, 6, 2.5
    f = rng.uniform(0, 1, size=(H, W))
    target = rng.uniform(0, 1, size=(H, W))
    UK = oracle.solve(f, lam=lam, iters=K)
    res = oracle.solve_adjoint(UK - target, f, lam, K)
    total = res["gf"] + res["gu0"]
    base = _path_maps(f, f, lam, 1 / (1 + lam), K)
    h, checked = 1e-6, 0
    for _ in range(16):
        y, x = int(rng.integers(H)), int(rng.integers(W))
        fp, fm = f.copy(), f.copy()
        fp[y, x] += h
        fm[y, x] -= h
        if not all(all(np.array_equal(a, b) for a, b in zip(_path_maps(ff, ff, lam, 1 / (1 + lam), K),
                                                            base)) for ff in (fp, fm)):
            continue
        fd = (_loss(oracle.solve(fp, lam=lam, iters=K), target)
              - _loss(oracle.solve(fm, lam=lam, iters=K), target)) / (2 * h)
        assert fd == pytest.approx(total[y, x], rel=1e-5, abs=1e-9)
        checked += 1
    assert checked >= 8


def test_adjoint_fd_explicit_step():
    """An explicit step delta (here 0.2 at lam = 2.5, delta (1 + lam) = 0.7):
    the keep factor is 1 - delta, the data factor delta, and only delta H_d
    enters dL/dlam."""
    rng = np.random.default_rng(34)
    H, W, K = 9, 8, 5
    f = rng.uniform(0, 1, size=(H, W))
    u0 = rng.uniform(0, 1, size=(H, W))
    target = rng.uniform(0, 1, size=(H, W))
    _fd_pins(f, u0, target, 2.5, 0.2, K, False, rng)


def test_adjoint_fd_flow_mode():
    """Curvature flow (no data term), delta = 0.6: dL/dU^0 by central differences."""
    rng = np.random.default_rng(35)
    H, W, K = 8, 8, 4
    u0 = rng.uniform(0, 1, size=(H, W))
    target = rng.uniform(0, 1, size=(H, W))
    _fd_pins(None, u0, target, 1.0, 0.6, K, False, rng)


# ---------------------------------------------------------------------------------------
# brute force on tiny inputs: the selection is the first minimum in printed order
# ---------------------------------------------------------------------------------------

def test_selection_brute_force_small_integers():
    """Every 3x3 neighbourhood with entries in {0, 1, 2} centred in a 3x3
    image (borders replicate, so the centre's neighbourhood is the image):
    H_d equals the first-minimum response computed straight from the
    printed fractions."""
    printed = _read_kernels("half_window_kernels.txt")
    ks = [np.array([[float(v) for v in printed[f"h{i}"][r]] for r in range(3)]) for i in range(1, 9)]
    rng = np.random.default_rng(18)
    vals = rng.integers(0, 3, size=(4000, 3, 3)).astype(np.float64)
    for U in vals:
        d = [float((k * U).sum()) for k in ks]
        want = d[_first_min([round(v * 12) for v in d])]
        assert oracle.compute(U)[1, 1] == pytest.approx(want, abs=1e-14)


# ---------------------------------------------------------------------------------------
# energies along the iteration (reported, not assumed: the paper never claims a
# monotone decrease).  On the piecewise-smooth noisy workloads both the WMC energy
# (eq. (wmcr), q = 1, plus the data term) and the area energy (eq. (areaReg)) decrease
# at every step up to FP64 rounding once the iteration has converged.
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("dscale", [1.0, 0.5])
def test_energy_decreases_on_c1(dscale):
    import wmc_synth
    noisy, clean = wmc_synth.c1()
    f = noisy[0].astype(np.float64)
    lam = 1.0
    delta = dscale / (1 + lam)
    U = f.copy()
    ew, ea = [oracle.energy_wmc(U, f, lam)], [oracle.energy_area(U, f, lam)]
    for _ in range(50):
        U = oracle.step(U, f, lam, delta)
        ew.append(oracle.energy_wmc(U, f, lam))
        ea.append(oracle.energy_area(U, f, lam))
    ew, ea = np.array(ew), np.array(ea)
    assert np.all(ew[1:] <= ew[:-1] * (1 + 1e-12))
    assert np.all(ea[1:] <= ea[:-1] * (1 + 1e-12))
    assert ew[-1] < 0.6 * ew[0]
    # the denoised result is closer to the clean image than the input
    c = clean[0].astype(np.float64)
    assert np.sqrt(((U - c) ** 2).mean()) < 0.75 * np.sqrt(((f - c) ** 2).mean())


# ---------------------------------------------------------------------------------------
# energies and test helpers: closed forms
# ---------------------------------------------------------------------------------------

def test_energy_closed_forms():
    # eq. (wmcr), q = 1: a contrast-J rectangle has sum |H_d| = 2J/3 (four corners)
    J, lam = 0.5, 3.0
    U = _rect(12, 13, 3, 9, 4, 10, J)
    f = U + 0.25
    data = 0.5 * U.size * 0.25 ** 2
    assert oracle.energy_wmc(U, f, lam) == pytest.approx(data + lam * 2 * J / 3, rel=1e-14)
    assert oracle.energy_wmc(U, None, lam) == pytest.approx(lam * 2 * J / 3, rel=1e-14)
    # eq. (areaReg): constant -> lam * H * W; ramp of slope a along x -> each pixel but
    # the last column has |grad| = a
    H, W, a = 5, 8, 0.75
    assert oracle.energy_area(np.full((H, W), 0.3), None, lam) == pytest.approx(lam * H * W)
    ramp = np.tile(a * np.arange(W, dtype=np.float64), (H, 1))
    want = lam * (H * (W - 1) * np.sqrt(1 + a * a) + H)
    assert oracle.energy_area(ramp, None, lam) == pytest.approx(want, rel=1e-14)
    # the same ramp along y, and a plane a x + b y: interior pixels have
    # |grad|^2 = a^2 + b^2, the last column b^2 only, the last row a^2 only
    ramp_y = ramp.T.copy()
    want_y = lam * (H * (W - 1) * np.sqrt(1 + a * a) + H)
    assert oracle.energy_area(ramp_y, None, lam) == pytest.approx(want_y, rel=1e-14)
    b = -0.4
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    plane = a * xx + b * yy
    want_p = lam * ((H - 1) * (W - 1) * np.sqrt(1 + a * a + b * b)
                    + (H - 1) * np.sqrt(1 + b * b) + (W - 1) * np.sqrt(1 + a * a) + 1)
    assert oracle.energy_area(plane, None, lam) == pytest.approx(want_p, rel=1e-14)


def test_energy_area_matches_an_independent_evaluation():
    """eq. (areaReg) with forward differences (zero at the last row and column)
    plus the quadratic data term, evaluated with numpy array slicing."""
    rng = np.random.default_rng(3)
    u = rng.uniform(0, 1, size=(13, 17))
    f = rng.uniform(0, 1, size=(13, 17))
    lam = 5.0
    ux = np.zeros_like(u)
    uy = np.zeros_like(u)
    ux[:, :-1] = u[:, 1:] - u[:, :-1]
    uy[:-1, :] = u[1:, :] - u[:-1, :]
    e = (0.5 * (u - f) ** 2 + lam * np.sqrt(1.0 + ux * ux + uy * uy)).sum()
    assert oracle.energy_area(u, f, lam) == pytest.approx(e, rel=1e-13)


def test_near_tie_helpers():
    """The (2,2) paraboloid pixel is an exact opposite-sign tie; a generic
    random pixel is not."""
    H = W = 11
    c = 5
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    U = (x - c) ** 2 + (y - c) ** 2
    mask = oracle.near_tie_mask(U, 0.0)
    assert mask[c + 2, c + 2]
    assert not mask[c, c] and not mask[c + 1, c]
    allowed = oracle.allowed_values(U, 0.0)
    vals = allowed[c + 2, c + 2][~np.isnan(allowed[c + 2, c + 2])]
    assert set(np.round(vals * 3).astype(int)) == {-4, 4}


def test_step_window_equals_full_step():
    rng = np.random.default_rng(19)
    U = rng.uniform(0, 1, size=(20, 23))
    f = rng.uniform(0, 1, size=(20, 23))
    full = U.copy()
    for _ in range(3):
        full = oracle.step(full, f, 1.2)
    for (y, x) in [(0, 0), (10, 11), (19, 22), (0, 15), (7, 0), (3, 3)]:
        assert oracle.step_window(U, f, y, x, 3, lam=1.2) == pytest.approx(full[y, x], abs=1e-15)


# ---------------------------------------------------------------------------------------
# the l1-fidelity primal-dual iteration (Sec. 5.3)
# ---------------------------------------------------------------------------------------

def _shrink(r, a):
    """Soft threshold: the closed-form b of Sec. 5.3."""
    return np.where(r > a, r - a, np.where(r < -a, r + a, 0.0))


def test_l1_dual_update_matches_shrink_identity():
    """The dual update d' = clip(r) is the paper's d' = d + U - f - b with
    b = shrink(r, alpha), r = U - f + d."""
    rng = np.random.default_rng(30)
    U = rng.uniform(0, 1, size=(15, 17))
    f = rng.uniform(0, 1, size=U.shape)
    d = rng.uniform(-0.1, 0.1, size=U.shape)
    alpha = 0.07
    _, dn = oracle.l1_step(U, d, f, 1.0, alpha)
    r = U - f + d
    assert np.allclose(dn, d + U - f - _shrink(r, alpha), atol=1e-15)
    assert np.abs(dn).max() <= alpha


def test_l1_fixed_point_and_bounds():
    U = np.full((9, 11), 0.4)
    uo, do = oracle.l1_solve(U, lam=2.0, alpha=0.05, iters=20)
    assert np.array_equal(uo, U) and np.all(do == 0.0)
    rng = np.random.default_rng(31)
    f = rng.uniform(0, 1, size=(20, 20))
    uo, do = oracle.l1_solve(f, lam=1.0, alpha=0.03, iters=30)
    assert np.abs(do).max() <= 0.03 + 1e-15


def test_l1_spike_two_steps_closed_form():
    """Constant c with one spike c + J, U^0 = f, d^0 = 0.
    Step 1: r = 0 so d^1 = 0; only the spike moves, by delta lam H_d = -delta lam J
    (all eight responses equal -12J at the spike, zero at its neighbours).
    Step 2: at the spike r = -delta lam J, d^2 = clip(r); the spike's own response
    is -J(1 - delta lam) and its neighbours still see one half window without it."""
    c, J, lam, alpha = 0.3, 0.5, 1.0, 0.05
    delta = 1.0 / (lam + 2.0 / alpha)
    f = np.full((9, 9), c)
    f[4, 4] += J
    u1, d1 = oracle.l1_step(f, np.zeros_like(f), f, lam, alpha, delta)
    assert np.all(d1 == 0.0)
    want1 = f.copy()
    want1[4, 4] = c + J - delta * lam * J
    assert np.allclose(u1, want1, atol=1e-15)
    u2, d2 = oracle.l1_step(u1, d1, f, lam, alpha, delta)
    r = -delta * lam * J
    dn = min(max(r, -alpha), alpha)
    spike = u1[4, 4] + delta * (lam * (-J * (1 - delta * lam)) - 2 * dn / alpha)
    assert u2[4, 4] == pytest.approx(spike, abs=1e-15)
    assert d2[4, 4] == pytest.approx(dn, abs=1e-15)
    mask = np.ones_like(f, bool)
    mask[4, 4] = False
    assert np.allclose(u2[mask], f[mask], atol=1e-15) and np.all(d2[mask] == 0.0)


def test_l1_large_alpha_reduces_to_the_flow():
    """With alpha far above every residual the dual terms vanish and the
    iteration is the curvature flow of eq. (MCF) with step delta lam."""
    rng = np.random.default_rng(32)
    f = rng.uniform(0, 1, size=(14, 16))
    lam, alpha, delta = 2.0, 1e12, 0.2
    uo, _ = oracle.l1_solve(f, lam=lam, alpha=alpha, iters=12, delta=delta)
    flow = oracle.solve(None, iters=12, delta=delta * lam, u0=f)
    assert np.allclose(uo, flow, atol=1e-9)


# ---------------------------------------------------------------------------------------
# the conventional finite-difference WMC of eq. (rhs) (comparator of Sec. 5.4)
# ---------------------------------------------------------------------------------------

def test_fd_quadratic_closed_form():
    """Central differences are exact on quadratics, so in the interior
    H^w = 2a + 2c - (Uy^2 2c + 2 Ux Uy b + Ux^2 2a)/(Ux^2 + Uy^2)."""
    rng = np.random.default_rng(40)
    H, W = 9, 10
    for _ in range(20):
        a, b, c, d, e = (float(v) for v in rng.integers(-3, 4, size=5))
        U = _quadratic(a, b, c, d, e, 0.5, H, W)
        got = oracle.fd_compute(U, eps=0.0 + 1e-300)
        for y in range(1, H - 1):
            for x in range(1, W - 1):
                ux, uy = 2 * a * x + b * y + d, b * x + 2 * c * y + e
                g = ux * ux + uy * uy
                if g == 0:
                    want = 2 * a + 2 * c
                else:
                    want = 2 * a + 2 * c - (uy * uy * 2 * c + 2 * ux * uy * b + ux * ux * 2 * a) / g
                assert got[y, x] == pytest.approx(want, rel=1e-12, abs=1e-12)


def test_fd_paraboloid_and_plane():
    """U = r^2: the normal diffusion term equals U_rr = 2, so H^w = 4 - 2 = 2
    away from the centre, and the Laplacian 4 at the centre where the gradient
    vanishes (the guard).  Planes give 0 in the interior."""
    n, c = 13, 6
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    U = (x - c) ** 2 + (y - c) ** 2
    got = oracle.fd_compute(U)
    inner = got[1:-1, 1:-1].copy()
    assert inner[c - 1, c - 1] == pytest.approx(4.0)
    inner[c - 1, c - 1] = 2.0
    assert np.allclose(inner, 2.0, atol=1e-12)
    P = 0.3 * x - 0.7 * y
    assert np.allclose(oracle.fd_compute(P)[1:-1, 1:-1], 0.0, atol=1e-14)


def test_fd_flow_is_the_explicit_iteration():
    rng = np.random.default_rng(41)
    U = rng.uniform(0, 1, size=(12, 14))
    a = U.copy()
    for _ in range(5):
        a = a + 0.1 * oracle.fd_compute(a)
    assert np.allclose(oracle.fd_flow(U, 0.1, 5), a, atol=1e-14)


# ---- curvature-flow study of Sec. 5.4 (Fig. exp_flow) on the oracle -----------------
# The paper reports that the flow driven by the half-window operator keeps
# edges and sharp corners while the conventional discretisation blurs them.
# On a piecewise-constant image this shows as: the half-window flow leaves
# straight edges (axis-aligned and 45 degrees) bitwise unchanged and changes
# only corners and curved boundaries; the finite-difference flow moves the
# 45-degree edges and loses more structure (SSIM against the input) at every t.

def _edge_pixels(side):
    """Middle thirds of the square's top edge and of the diamond's upper-left
    edge in wmc_synth.shapes(side)."""
    q = side // 4
    r = 0.6 * q
    sq_top = int(np.ceil(3 * q - r))
    x0, x1 = int(np.ceil(3 * q - r)), int(np.floor(3 * q + r))
    n = x1 - x0 + 1
    square = [(sq_top, x) for x in range(x0 + n // 3, x1 - n // 3 + 1)]
    # diamond |x-3q| + |y-q| <= r: its upper-left edge holds the inside pixels
    # with (3q - x) + (q - y) == floor(r)
    k = int(np.floor(r))
    diamond = [(q - k + j, 3 * q - j) for j in range(k // 3, k - k // 3 + 1)]
    return square, diamond


def test_mcf_study_half_window_flow_keeps_straight_edges():
    import sys
    sys.path.insert(0, os.path.dirname(__file__))
    from ssim_util import ssim
    a = wmc_synth.shapes(192).astype(np.float64)
    square, diamond = _edge_pixels(192)
    for (y, x) in square + diamond:  # the pixels lie on the shapes' edges
        assert a[y, x] != a[y - 1, x] or a[y, x] != a[y, x - 1]
    hl5 = oracle.solve(None, 1.0, 5, u0=a)
    fd5 = oracle.fd_flow(a, 0.1, 5)
    for (y, x) in square + diamond:
        assert hl5[y, x] == a[y, x]
    # the conventional flow keeps axis-aligned edges (its normal term cancels
    # the across-edge second difference) but moves the diagonal ones
    assert max(abs(fd5[y, x] - a[y, x]) for (y, x) in square) < 1e-9  # eps guard only
    assert np.mean([abs(fd5[y, x] - a[y, x]) for (y, x) in diamond]) > 1e-2
    a = wmc_synth.shapes(96).astype(np.float64)
    prev_hl, prev_fd = 1.0, 1.0
    for t in (10, 50, 200):
        s_hl = ssim(a, oracle.solve(None, 1.0, t, u0=a))
        s_fd = ssim(a, oracle.fd_flow(a, 0.1, t))
        assert s_hl > 0.99 and (1 - s_fd) > 5 * (1 - s_hl), (t, s_hl, s_fd)
        assert s_fd <= prev_fd + 1e-9 and s_hl <= prev_hl + 1e-9
        prev_hl, prev_fd = s_hl, s_fd


# ---- learnable half-window layer (Sec. 4.3), O12 ------------------------------------

def test_layer_with_printed_kernels_is_the_operator():
    """With the eight printed kernels (x12, integer weights) the layer is the
    Half Laplace Operator: on integer images every value is exact, so output
    and selection (ties included) must match 12 * H_d bitwise."""
    K12 = oracle.kernel_table().astype(np.float64)
    rng = np.random.default_rng(31)
    for shape in [(1, 1), (3, 1), (1, 4), (9, 13), (40, 33)]:
        U = rng.integers(-20, 21, size=shape).astype(np.float64)
        out, m = oracle.layer_forward(U, K12, return_argmin=True)
        hd, mh = oracle.compute(U, return_argmin=True)
        assert np.array_equal(out, 12 * hd)
        assert np.array_equal(m, mh)


def test_layer_single_kernel_is_a_correlation():
    """K = 1: no selection, the layer is a correlation with replicate border
    (scipy.ndimage.correlate, mode 'nearest')."""
    from scipy import ndimage
    rng = np.random.default_rng(32)
    U = rng.uniform(-1, 1, size=(17, 23))
    w = rng.uniform(-1, 1, size=(1, 3, 3))
    ref = ndimage.correlate(U, w[0], mode="nearest")
    assert np.allclose(oracle.layer_forward(U, w), ref, atol=1e-13)


def _fixed_m_forward(U, w, m):
    """The layer's map with the selection held at m, built from scipy
    correlations (independent of the oracle's code)."""
    from scipy import ndimage
    resp = np.stack([ndimage.correlate(U, w[k], mode="nearest") for k in range(w.shape[0])])
    return np.take_along_axis(resp, m[None].astype(np.int64), axis=0)[0]


def test_layer_forward_selection_and_permutation():
    rng = np.random.default_rng(33)
    U = rng.uniform(0, 1, size=(25, 31))
    w = rng.standard_normal((6, 3, 3))
    out, m = oracle.layer_forward(U, w, return_argmin=True)
    from scipy import ndimage
    resp = np.stack([ndimage.correlate(U, w[k], mode="nearest") for k in range(6)])
    assert np.array_equal(m, np.argmin(np.abs(resp), axis=0))   # first minimum
    assert np.allclose(out, _fixed_m_forward(U, w, m), atol=1e-13)
    perm = rng.permutation(6)
    out2, m2 = oracle.layer_forward(U, w[perm], return_argmin=True)
    assert np.allclose(out2, out, atol=1e-13)
    assert np.array_equal(perm[m2], m)


def test_layer_backward_dot_product_and_weight_fd():
    """gU is the transpose of the fixed-selection map (dot-product test
    against scipy correlations); gW matches central differences of
    L = <g, out> in every weight (selections do not change for the step)."""
    rng = np.random.default_rng(34)
    H, W, K = 14, 19, 5
    U = rng.uniform(0, 1, size=(H, W))
    w = rng.standard_normal((K, 3, 3))
    g = rng.standard_normal((H, W))
    out, m = oracle.layer_forward(U, w, return_argmin=True)
    gU, gW = oracle.layer_backward(U, w, m, g)
    v = rng.standard_normal((H, W))
    lhs = float(np.sum(_fixed_m_forward(v, w, m) * g))
    assert abs(lhs - float(np.sum(v * gU))) <= 1e-12 * max(1.0, abs(lhs))
    eps = 1e-6
    for k in range(K):
        for r in range(3):
            for c in range(3):
                wp, wm = w.copy(), w.copy()
                wp[k, r, c] += eps
                wm[k, r, c] -= eps
                op, mp = oracle.layer_forward(U, wp, return_argmin=True)
                om, mm = oracle.layer_forward(U, wm, return_argmin=True)
                assert np.array_equal(mp, m) and np.array_equal(mm, m)
                fd = (np.sum(g * op) - np.sum(g * om)) / (2 * eps)
                assert abs(fd - gW[k, r, c]) <= 1e-6 * max(1.0, abs(gW[k, r, c]))


def test_network_module_kernel_table_matches_the_oracle():
    """The package's initialiser table (nn.py) and the oracle's table are
    transcribed separately from Sec. 4.2; they must agree entry for entry."""
    from paper_1903_07189_amd.nn import PRINTED_KERNELS_X12
    assert np.array_equal(np.array(PRINTED_KERNELS_X12), oracle.kernel_table())


# ---- 3-D extension (O13) --------------------------------------------------------------

def _fold_kernels(base, normals):
    """Half windows by Neumann reflection of `base` (centre excluded) across
    each mirror plane through the centre: for normal n and each side, weights
    on the dropped side move to their mirror image.  Dimension-generic."""
    nd = base.ndim
    out = []
    for n in normals:
        n = np.array(n)
        for sg in (1, -1):  # keep sg * n.o <= 0
            k = np.zeros_like(base)
            for idx in np.ndindex(base.shape):
                o = np.array(idx) - 1
                if not o.any():
                    continue
                d = sg * int(n @ o)
                t = o - 2 * int(n @ o) * n // int(n @ n) if d > 0 else o
                k[tuple(t + 1)] += base[idx]
            k[(1,) * nd] = -k.sum()
            out.append(k)
    return np.array(out)


def test_fold_construction_reproduces_the_printed_2d_kernels():
    """The construction used for 3-D, applied in 2-D to k4 (x12) with the four
    mirror lines of the square, gives exactly the eight printed kernels of
    Sec. 4.2 (as a set): the 3-D kernels follow the paper's own recipe."""
    s = np.array([1, 2, 1])
    k4 = np.outer(s, s).astype(np.int64)   # off-centre weights of 12 k4
    k4[1, 1] = 0
    folded = _fold_kernels(k4, [(0, 1), (1, 0), (1, 1), (1, -1)])
    printed = oracle.kernel_table()
    key = lambda a: sorted(map(lambda k: tuple(k.ravel()), a))  # noqa: E731
    assert key(folded) == key(printed)


def test_3d_kernels_match_an_independent_construction():
    s = np.array([1, 2, 1])
    base = np.einsum("i,j,k->ijk", s, s, s).astype(np.int64)  # [z][y][x]
    base[1, 1, 1] = 0
    # normals in (z, y, x) order for the [z][y][x] layout: e_x, e_y, e_z, e_x+-e_y, e_x+-e_z, e_y+-e_z
    normals = [(0, 0, 1), (0, 1, 0), (1, 0, 0), (0, 1, 1), (0, -1, 1), (1, 0, 1), (-1, 0, 1),
               (1, 1, 0), (-1, 1, 0)]
    ref = _fold_kernels(base, normals)
    k3 = oracle.kernels3()
    assert np.array_equal(k3, ref)
    # structure: 18 kernels, centre -56, off-centre weights >= 0 summing to 56,
    # opposite sides of a plane add up to twice the base kernel
    assert k3.shape == (18, 3, 3, 3)
    assert np.all(k3.reshape(18, 27).sum(1) == 0) and np.all(k3[:, 1, 1, 1] == -56)
    full = base.copy()
    full[1, 1, 1] = -56
    for j in range(9):
        assert np.array_equal(k3[2 * j] + k3[2 * j + 1], 2 * full)


def test_3d_operator_against_library_correlation():
    """compute3 = first-argmin over the 18 kernels applied with
    scipy.ndimage.correlate (replicate border), divided by 56."""
    from scipy import ndimage
    rng = np.random.default_rng(50)
    for shape in [(1, 1, 1), (2, 3, 4), (5, 6, 7), (9, 4, 11)]:
        U = rng.uniform(0, 1, size=shape)
        resp = np.stack([ndimage.correlate(U, k.astype(np.float64), mode="nearest")
                         for k in oracle.kernels3()])
        m = np.argmin(np.abs(resp), axis=0)
        ref = np.take_along_axis(resp, m[None], 0)[0] / 56.0
        H, mo = oracle.compute3(U, return_argmin=True)
        assert np.allclose(H, ref, atol=1e-13)
        # the selection agrees wherever the minimum is not a rounding-level tie
        a = np.sort(np.abs(resp), axis=0)
        clear = (a[1] - a[0]) > 1e-9
        assert np.array_equal(mo[clear], m[clear])


def test_3d_closed_forms_and_symmetry():
    rng = np.random.default_rng(51)
    # constants -> 0 exactly
    assert np.all(oracle.compute3(np.full((4, 5, 6), 0.7)) == 0.0)
    # linear along an axis or a face diagonal -> 0 in the interior
    z, y, x = np.mgrid[0:7, 0:8, 0:9].astype(np.float64)
    for U in (0.5 * x, -0.25 * y, 2.0 * z, x + y, x - z, y + z):
        assert np.all(oracle.compute3(U)[1:-1, 1:-1, 1:-1] == 0.0)
    # paraboloid centred on a voxel: all 18 candidates tie at
    # (8*1*3 + 12*2*2 + 6*4*1)/56 = 96/56 = 12/7
    c = 3
    U = (x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2
    assert oracle.compute3(U)[c, c, c] == 96.0 / 56.0
    # the cube's symmetries permute the kernels: H commutes with them on
    # generic data
    U = rng.uniform(0, 1, size=(6, 7, 8))
    H = oracle.compute3(U)
    assert np.allclose(oracle.compute3(U[::-1]), H[::-1], atol=1e-14)
    assert np.allclose(oracle.compute3(U.transpose(0, 2, 1)), H.transpose(0, 2, 1), atol=1e-14)
    assert np.allclose(oracle.compute3(U.transpose(2, 1, 0)), H.transpose(2, 1, 0), atol=1e-14)
    # the solver is the explicit iteration
    f = rng.uniform(0, 1, size=(4, 5, 6))
    a = f.copy()
    for _ in range(3):
        a = a + 0.5 * ((f - a) + 1.0 * oracle.compute3(a))
    assert np.allclose(oracle.solve3(f, 1.0, 3), a, atol=1e-14)
