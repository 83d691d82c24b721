"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test checks the oracle (oracle/mls_oracle.c) against something the paper
or the mathematics fixes -- closed forms of Muelder et al. Sec. 3.3 (Eq. 5 the
weighted mean, Eq. 6-8 the affine centroid form), polynomial reproduction,
invariances, exact interpolation, an SVD least-squares solve of the weighted
problem, the global least-squares limit -- chosen so that a dropped term, a
wrong sign or index, or a transposed operand in the oracle fails at least one.
"""
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dyadic_points(rng, n, bits=8):
    """Points on a 2^-bits lattice: exact in float32, exact under x -> 1 - x."""
    s = float(1 << bits)
    return rng.integers(0, (1 << bits) + 1, size=(n, 2)) / s


def poly_eval(coef, x, y):
    terms = [np.ones_like(x), x, y, x * x, x * y, y * y]
    return sum(c * t for c, t in zip(coef, terms))


def positions(rng, k, lo=0.15, hi=0.85):
    return rng.uniform(lo, hi, size=(k, 2))


def basis_cols(dx, dy, degree):
    cols = [np.ones_like(dx)]
    if degree >= 1:
        cols += [dx, dy]
    if degree >= 2:
        cols += [dx * dx, dx * dy, dy * dy]
    return np.stack(cols, axis=1)


def brute_force_value(pts, vals, p, degree, w):
    """Weighted least squares by SVD (numpy lstsq) in an unscaled basis
    centred on p; returns the fitted value at p for every column of vals."""
    dx, dy = pts[:, 0] - p[0], pts[:, 1] - p[1]
    B = basis_cols(dx, dy, degree)
    sw = np.sqrt(w)
    coef, *_ = np.linalg.lstsq(sw[:, None] * B, sw[:, None] * vals, rcond=None)
    return coef[0]


def gauss_w(pts, p, h):
    r2 = ((pts - p) ** 2).sum(axis=1)
    return np.exp(-r2 / h ** 2)


# --------------------------------------------------------------------------
# P1 / P2: reproduction of polynomials in the basis span and of constants
# --------------------------------------------------------------------------

@pytest.mark.parametrize("basis,deg", [("linear", 1), ("quadratic", 2)])
@pytest.mark.parametrize("weight,h", [("gaussian", 0.12), ("wendland", 0.35),
                                      ("invpow", 0.1)])
def test_polynomial_reproduction(oracle, basis, deg, weight, h):
    rng = np.random.default_rng(11 + deg)
    pts = dyadic_points(rng, 300)
    coef = rng.integers(-7, 8, size=6) / 8.0
    if deg == 1:
        coef[3:] = 0.0
    f = poly_eval(coef, pts[:, 0], pts[:, 1])
    assert np.all(f.astype(np.float32) == f)          # inputs are exact
    pos = positions(rng, 200)
    fields, degree, dmin = oracle.fit_at(pts, f, pos, basis=basis, weight=weight,
                                         h=h)
    ok = (degree == deg) & (dmin >= 1e-3)
    assert ok.sum() > 150
    exact = poly_eval(coef, pos[:, 0], pos[:, 1])
    S = f.max() - f.min()
    err = np.abs(fields[0] - exact)[ok] / S
    assert err.max() <= 1e-12


def test_lower_degree_does_not_reproduce_quadratic(oracle):
    """The reproduction pin has teeth: a linear fit of a curved field misses."""
    rng = np.random.default_rng(3)
    pts = dyadic_points(rng, 300)
    f = pts[:, 0] ** 2 + pts[:, 1] ** 2
    pos = positions(rng, 50)
    fields, degree, _ = oracle.fit_at(pts, f, pos, basis="linear", h=0.12)
    exact = pos[:, 0] ** 2 + pos[:, 1] ** 2
    assert np.all(degree == 1)
    assert np.abs(fields[0] - exact).max() > 1e-4


@pytest.mark.parametrize("basis", ["constant", "linear", "quadratic"])
@pytest.mark.parametrize("weight,h", [("gaussian", 0.1), ("wendland", 0.3),
                                      ("invpow", 0.1)])
def test_constant_reproduction(oracle, basis, weight, h):
    rng = np.random.default_rng(5)
    pts = rng.random((120, 2)).astype(np.float32)
    c = np.float32(0.3)
    vals = np.full((120, 2), c, np.float32)
    vals[:, 1] = np.float32(-7.25)
    pos = positions(rng, 100)
    fields, degree, _ = oracle.fit_at(pts, vals, pos, basis=basis, weight=weight, h=h)
    det = degree != oracle.DEG_NAN
    assert det.sum() > 80
    assert np.abs(fields[0][det] - float(c)).max() <= 1e-13
    assert np.abs(fields[1][det] + 7.25).max() <= 1e-12


def test_identity_reproduction(oracle):
    """f_i = x_i reproduces the coordinates themselves (undistorted identity,
    Sec. 3.3 criterion 3)."""
    rng = np.random.default_rng(8)
    pts = dyadic_points(rng, 250)
    pos = positions(rng, 80)
    for basis in ("linear", "quadratic"):
        fields, degree, dmin = oracle.fit_at(pts, pts, pos, basis=basis, h=0.1)
        ok = dmin >= 1e-3
        assert np.abs(fields[:, ok].T - pos[ok]).max() <= 1e-12


# --------------------------------------------------------------------------
# P3 / P4: linearity and affine equivariance in the values
# --------------------------------------------------------------------------

def test_linearity_and_affine_equivariance(oracle):
    rng = np.random.default_rng(21)
    pts = dyadic_points(rng, 200)
    f = rng.integers(-64, 65, size=200) / 32.0
    g = rng.integers(-64, 65, size=200) / 32.0
    vals = np.stack([f, g, 2.0 * f - 0.5 * g, 4.0 * f + 1.5], axis=1)
    assert np.all(vals.astype(np.float32) == vals)
    pos = positions(rng, 120)
    for basis in ("constant", "linear", "quadratic"):
        F, deg, _ = oracle.fit_at(pts, vals, pos, basis=basis, h=0.08)
        det = deg != oracle.DEG_NAN
        np.testing.assert_allclose(F[2][det], 2.0 * F[0][det] - 0.5 * F[1][det],
                                   rtol=0, atol=1e-12)
        np.testing.assert_allclose(F[3][det], 4.0 * F[0][det] + 1.5, rtol=0,
                                   atol=1e-12)


# --------------------------------------------------------------------------
# P5: invariances
# --------------------------------------------------------------------------

def test_rigid_motion_invariance_exact(oracle):
    """Rotation by 90 degrees plus a dyadic translation of points and
    evaluation positions together leaves the fields unchanged."""
    rng = np.random.default_rng(31)
    pts = dyadic_points(rng, 150)
    vals = rng.standard_normal((150, 3)).astype(np.float32)
    pos = dyadic_points(rng, 60, bits=10)

    def move(a):
        return np.stack([-a[:, 1] + 1.25, a[:, 0] - 0.5], axis=1)

    for basis in ("linear", "quadratic"):
        A, da, _ = oracle.fit_at(pts, vals, pos, basis=basis, h=0.1)
        B, db, _ = oracle.fit_at(move(pts), vals, move(pos), basis=basis, h=0.1)
        assert np.array_equal(da, db)
        det = da != oracle.DEG_NAN
        np.testing.assert_allclose(B[:, det], A[:, det], rtol=0, atol=1e-12)


def test_rotation_invariance_general_angle(oracle):
    rng = np.random.default_rng(32)
    pts = rng.random((150, 2))
    vals = rng.standard_normal((150, 2))
    th = 0.7
    Rm = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    pts32 = pts.astype(np.float32).astype(np.float64)
    rot = (pts32 @ Rm.T).astype(np.float32)
    pos = positions(rng, 60)
    # Evaluate the rotated set at the rotated positions; its points carry the
    # rounding of the rotation (about 6e-8), so the tolerance is loose.
    A, da, dmA = oracle.fit_at(pts32, vals, pos, basis="quadratic", h=0.15)
    B, db, _ = oracle.fit_at(rot, vals, pos @ Rm.T, basis="quadratic", h=0.15)
    ok = (da == db) & (dmA >= 1e-2)
    assert ok.sum() > 40
    S = np.ptp(vals.astype(np.float32), axis=0)[:, None]
    assert (np.abs(A - B)[:, ok] / S).max() < 1e-5


def test_invpow_independent_of_h(oracle):
    """For the inverse-distance weight of Eq. 4 a change of h scales every
    weight by one factor and rescales the basis: the fit must not move."""
    rng = np.random.default_rng(41)
    pts = rng.random((100, 2))
    vals = rng.standard_normal((100, 3))
    pos = positions(rng, 50)
    for basis in ("constant", "linear", "quadratic"):
        A, da, _ = oracle.fit_at(pts, vals, pos, basis=basis, weight="invpow",
                                 h=0.1, alpha=1.2, weight_floor=0.0)
        B, db, _ = oracle.fit_at(pts, vals, pos, basis=basis, weight="invpow",
                                 h=3.0, alpha=1.2, weight_floor=0.0)
        assert np.array_equal(da, db)
        np.testing.assert_allclose(A, B, rtol=1e-10, atol=1e-10)


# --------------------------------------------------------------------------
# P6: brute-force weighted least squares by SVD
# --------------------------------------------------------------------------

@pytest.mark.parametrize("basis,deg", [("constant", 0), ("linear", 1),
                                       ("quadratic", 2)])
def test_bruteforce_weighted_lstsq(oracle, basis, deg):
    rng = np.random.default_rng(50 + deg)
    for trial in range(10):
        n = int(rng.integers(8, 13))
        pts = rng.random((n, 2)).astype(np.float32).astype(np.float64)
        vals = rng.standard_normal((n, 2)).astype(np.float32).astype(np.float64)
        pos = rng.uniform(0.3, 0.7, size=(4, 2))
        F, dg, dmin = oracle.fit_at(pts, vals, pos, basis=basis, h=0.6)
        for k in range(4):
            assert dg[k] == deg and dmin[k] > 1e-6
            ref = brute_force_value(pts, vals, pos[k], deg, gauss_w(pts, pos[k], 0.6))
            np.testing.assert_allclose(F[:, k], ref, rtol=1e-10, atol=1e-10)


def test_bruteforce_wendland(oracle):
    rng = np.random.default_rng(55)
    pts = rng.random((12, 2)) * 0.4 + 0.3
    vals = rng.standard_normal((12, 3))
    pos = rng.uniform(0.4, 0.6, size=(5, 2))
    h = 0.5
    F, dg, _ = oracle.fit_at(pts, vals, pos, basis="quadratic", weight="wendland", h=h)
    pts = pts.astype(np.float32).astype(np.float64)
    vals = vals.astype(np.float32).astype(np.float64)
    for k in range(5):
        r = np.sqrt(((pts - pos[k]) ** 2).sum(1)) / h
        w = np.where(r < 1, (1 - r) ** 4 * (4 * r + 1), 0.0)
        assert dg[k] == 2
        np.testing.assert_allclose(F[:, k], brute_force_value(pts, vals, pos[k], 2, w),
                                   rtol=1e-10, atol=1e-10)


# --------------------------------------------------------------------------
# P7: exact interpolation when N equals the number of basis terms
# --------------------------------------------------------------------------

@pytest.mark.parametrize("weight,h", [("gaussian", 0.2), ("wendland", 2.0)])
def test_exact_interpolation(oracle, weight, h):
    rng = np.random.default_rng(61)
    # three points: the plane through them
    pts = np.array([[0.2, 0.3], [0.7, 0.25], [0.45, 0.8]])
    vals = np.array([[1.0], [-2.0], [0.5]])
    pos = rng.uniform(0.3, 0.6, size=(20, 2))
    F, dg, _ = oracle.fit_at(pts, vals, pos, basis="linear", weight=weight, h=h)
    P32 = pts.astype(np.float32).astype(np.float64)
    c = np.linalg.solve(np.column_stack([np.ones(3), P32]), vals[:, 0])
    ok = dg == 1
    assert ok.sum() >= 15
    np.testing.assert_allclose(F[0][ok], c[0] + pos[ok] @ c[1:], rtol=0, atol=1e-9)
    # six unisolvent points: the quadratic interpolant
    pts6 = np.array([[0.2, 0.2], [0.8, 0.25], [0.5, 0.85], [0.3, 0.55],
                     [0.65, 0.6], [0.5, 0.35]])
    v6 = rng.standard_normal((6, 1))
    F6, dg6, _ = oracle.fit_at(pts6, v6, pos, basis="quadratic", weight=weight, h=h,
                               tau=1e-14)
    P6 = pts6.astype(np.float32).astype(np.float64)
    V = basis_cols(P6[:, 0], P6[:, 1], 2)
    c6 = np.linalg.solve(V, v6.astype(np.float32).astype(np.float64)[:, 0])
    ok6 = dg6 == 2
    assert ok6.sum() >= 15
    ref = basis_cols(pos[:, 0], pos[:, 1], 2) @ c6
    np.testing.assert_allclose(F6[0][ok6], ref[ok6], rtol=0, atol=1e-8)


# --------------------------------------------------------------------------
# P8: the paper's closed forms (Eq. 5 and Eq. 6-8)
# --------------------------------------------------------------------------

def test_closed_form_mean_mls_eq5(oracle):
    """Mean MLS: f_m(v) = v + sum w (q - p) / sum w.  The constant-basis fit of
    the displacement q_i - p_i, plus v, must equal it."""
    rng = np.random.default_rng(71)
    p = rng.random((80, 2)).astype(np.float32).astype(np.float64)
    q = (p + 0.05 * rng.standard_normal((80, 2))).astype(np.float32).astype(np.float64)
    disp = (q - p).astype(np.float32).astype(np.float64)
    v = positions(rng, 40)
    F, dg, _ = oracle.fit_at(p, disp, v, basis="constant", h=0.2)
    for k in range(40):
        w = gauss_w(p, v[k], 0.2)
        fm = v[k] + (w[:, None] * disp).sum(0) / w.sum()
        np.testing.assert_allclose(v[k] + F[:, k], fm, rtol=0, atol=1e-13)


def test_closed_form_affine_mls_eq6_8(oracle):
    """Affine MLS: f_a(v) = (v - p*) (sum w p^T p)^-1 sum w p^T q + q*, with
    centred p, q (row vectors) and weighted centroids p*, q* (Eq. 7, 8)."""
    rng = np.random.default_rng(72)
    p = rng.random((90, 2)).astype(np.float32).astype(np.float64)
    q = rng.standard_normal((90, 4)).astype(np.float32).astype(np.float64)
    v = positions(rng, 40)
    F, dg, _ = oracle.fit_at(p, q, v, basis="linear", h=0.15)
    assert np.all(dg == 1)
    for k in range(40):
        w = gauss_w(p, v[k], 0.15)
        ps = (w[:, None] * p).sum(0) / w.sum()
        qs = (w[:, None] * q).sum(0) / w.sum()
        ph, qh = p - ps, q - qs
        A = np.linalg.solve((w[:, None, None] * ph[:, :, None] * ph[:, None, :]).sum(0),
                            (w[:, None, None] * ph[:, :, None] * qh[:, None, :]).sum(0))
        fa = (v[k] - ps) @ A + qs
        np.testing.assert_allclose(F[:, k], fa, rtol=0, atol=1e-11)


# --------------------------------------------------------------------------
# P9: point identity for the inverse-distance weight (Eq. 4)
# --------------------------------------------------------------------------

def test_invpow_point_identity(oracle):
    rng = np.random.default_rng(81)
    pts = rng.random((60, 2)).astype(np.float32)
    vals = rng.standard_normal((60, 2)).astype(np.float32)
    pos = pts[:10].astype(np.float64)
    for basis in ("constant", "linear", "quadratic"):
        F, dg, _ = oracle.fit_at(pts, vals, pos, basis=basis, weight="invpow",
                                 h=0.1, alpha=1.0)
        assert np.all(dg == oracle.DEG_HIT)
        assert np.array_equal(F.T, vals[:10].astype(np.float64))
        near = pos + 1e-7
        Fn, dn, _ = oracle.fit_at(pts, vals, near, basis=basis, weight="invpow",
                                  h=0.1, alpha=1.0)
        assert np.all(dn != oracle.DEG_HIT)
        np.testing.assert_allclose(Fn.T, vals[:10], atol=1e-3)


# --------------------------------------------------------------------------
# P10 / P11: global least-squares limit and mirror symmetry
# --------------------------------------------------------------------------

@pytest.mark.parametrize("basis,deg", [("linear", 1), ("quadratic", 2)])
def test_global_least_squares_limit(oracle, basis, deg):
    rng = np.random.default_rng(90 + deg)
    pts = rng.random((60, 2)).astype(np.float32).astype(np.float64)
    vals = rng.standard_normal((60, 2)).astype(np.float32).astype(np.float64)
    pos = positions(rng, 10)
    F, dg, _ = oracle.fit_at(pts, vals, pos, basis=basis, h=1e5)
    B = basis_cols(pts[:, 0], pts[:, 1], deg)
    coef, *_ = np.linalg.lstsq(B, vals, rcond=None)
    ref = basis_cols(pos[:, 0], pos[:, 1], deg) @ coef
    assert np.all(dg == deg)
    np.testing.assert_allclose(F.T, ref, rtol=0, atol=1e-9)


def test_mirror_symmetry(oracle):
    rng = np.random.default_rng(95)
    pts = dyadic_points(rng, 200)
    vals = rng.standard_normal((200, 2)).astype(np.float32)
    grid = {"x0": 0.5 / 32, "y0": 0.5 / 32, "dx": 1 / 32, "dy": 1 / 32,
            "width": 32, "height": 32}
    mir = pts.copy()
    mir[:, 0] = 1.0 - mir[:, 0]
    for basis in ("linear", "quadratic"):
        A, da, _ = oracle.fit_grid(pts, vals, grid, basis=basis, h=0.07)
        B, db, _ = oracle.fit_grid(mir, vals, grid, basis=basis, h=0.07)
        assert np.array_equal(da, db[:, ::-1])
        det = da != oracle.DEG_NAN
        np.testing.assert_allclose(A[:, det], B[:, :, ::-1][:, det], rtol=0,
                                   atol=1e-12)


# --------------------------------------------------------------------------
# Degree ladder and the undetermined mask
# --------------------------------------------------------------------------

def test_ladder_collinear_falls_to_mean(oracle):
    """Points on a line make the linear normal matrix singular: the ladder
    drops to degree 0, which is Eq. 5's weighted mean."""
    rng = np.random.default_rng(101)
    t = rng.random(50)
    pts = np.stack([t, t], axis=1).astype(np.float32).astype(np.float64)
    vals = rng.standard_normal((50, 1)).astype(np.float32).astype(np.float64)
    pos = positions(rng, 20)
    F, dg, _ = oracle.fit_at(pts, vals, pos, basis="linear", h=0.3)
    assert np.all(dg == 0)
    for k in range(20):
        w = gauss_w(pts, pos[k], 0.3)
        np.testing.assert_allclose(F[0, k], (w * vals[:, 0]).sum() / w.sum(),
                                   rtol=0, atol=1e-13)


def test_ladder_points_on_circle_fall_to_linear(oracle):
    """On a circle x^2 + y^2 - r^2 vanishes at every point: the quadratic
    system is singular, the ladder accepts degree 1 with the linear fit."""
    rng = np.random.default_rng(102)
    a = rng.random(40) * 2 * math.pi
    pts = np.stack([0.5 + 0.25 * np.cos(a), 0.5 + 0.25 * np.sin(a)], 1)
    # exactly on the circle in float32 is impossible; use a dyadic square
    # lattice circle instead: points (x, y) with x^2 + y^2 = 25 scaled
    lat = np.array([[3, 4], [4, 3], [-3, 4], [-4, 3], [3, -4], [4, -3], [-3, -4],
                    [-4, -3], [5, 0], [0, 5], [-5, 0], [0, -5]], np.float64)
    pts = 0.5 + lat / 32.0
    vals = rng.standard_normal((12, 2))
    pos = rng.uniform(0.45, 0.55, size=(10, 2))
    Fq, dq, _ = oracle.fit_at(pts, vals, pos, basis="quadratic", h=0.3)
    Fl, dl, _ = oracle.fit_at(pts, vals, pos, basis="linear", h=0.3)
    assert np.all(dq == 1) and np.all(dl == 1)
    np.testing.assert_array_equal(Fq, Fl)


def test_weight_floor_gives_nan(oracle):
    pts = np.array([[0.1, 0.1], [0.12, 0.1], [0.1, 0.13]])
    vals = np.ones((3, 2))
    pos = np.array([[0.9, 0.9], [0.11, 0.11]])
    F, dg, _ = oracle.fit_at(pts, vals, pos, basis="linear", h=0.02)
    assert dg[0] == oracle.DEG_NAN and np.all(np.isnan(F[:, 0]))
    assert dg[1] != oracle.DEG_NAN and np.all(np.isfinite(F[:, 1]))
    # sum of weights about 1.6e-9: positive, but below the default floor 1e-6
    far = np.array([[0.21, 0.1]])
    F, dg, _ = oracle.fit_at(pts, vals, far, basis="constant", h=0.02)
    assert dg[0] == oracle.DEG_NAN and np.all(np.isnan(F[:, 0]))
    F, dg, _ = oracle.fit_at(pts, vals, far, basis="constant", h=0.02,
                             weight_floor=1e-12)
    assert dg[0] == 0 and np.allclose(F[:, 0], 1.0)


# --------------------------------------------------------------------------
# Weight profiles, read back through two-point weighted means
# --------------------------------------------------------------------------

def _weight_ratio(oracle, r, weight, h):
    """With a constant basis and two points -- one at the evaluation position
    with value 1, one at distance r with value 0 -- the fit is
    w(0) / (w(0) + w(r)); invert that for w(r) / w(0)."""
    pts = np.array([[0.5, 0.5], [0.5 + r, 0.5]])
    vals = np.array([[1.0], [0.0]])
    F, dg, _ = oracle.fit_at(pts, vals, np.array([[0.5, 0.5]]), basis="constant",
                             weight=weight, h=h, weight_floor=0.0)
    return 1.0 / F[0, 0] - 1.0


def test_gaussian_weight_profile(oracle):
    h = 0.125
    r = 0.125  # exactly h, exact in float32
    np.testing.assert_allclose(_weight_ratio(oracle, r, "gaussian", h), math.exp(-1),
                               rtol=1e-12)
    np.testing.assert_allclose(_weight_ratio(oracle, 2 * r, "gaussian", h),
                               math.exp(-4), rtol=1e-12)
    # separability w(sqrt(a^2 + b^2)) = w(a) w(b) through a diagonal point
    pts = np.array([[0.5, 0.5], [0.5 + 0.0625, 0.5 + 0.125]])
    F, _, _ = oracle.fit_at(pts, np.array([[1.0], [0.0]]), np.array([[0.5, 0.5]]),
                            basis="constant", h=h)
    wd = 1.0 / F[0, 0] - 1.0
    wa = _weight_ratio(oracle, 0.0625, "gaussian", h)
    wb = _weight_ratio(oracle, 0.125, "gaussian", h)
    np.testing.assert_allclose(wd, wa * wb, rtol=1e-12)


def test_wendland_weight_profile(oracle):
    h = 0.25
    np.testing.assert_allclose(_weight_ratio(oracle, 0.125, "wendland", h), 3.0 / 16.0,
                               rtol=1e-13)
    assert _weight_ratio(oracle, 0.25, "wendland", h) == 0.0
    assert _weight_ratio(oracle, 0.3, "wendland", h) == 0.0
    # C2 at the support edge: w(h (1 - e)) / e^3 -> 0
    e = 1e-3
    assert _weight_ratio(oracle, h * (1 - e), "wendland", h) / e ** 3 < 1e-2
    # monotone decreasing inside the support
    rs = np.linspace(0.0, 0.24, 25)[1:]
    ws = [_weight_ratio(oracle, float(np.float32(r)), "wendland", h) for r in rs]
    assert all(a > b for a, b in zip(ws, ws[1:]))


def test_wendland_compact_support(oracle):
    """Points beyond the support radius do not change the fit at all."""
    rng = np.random.default_rng(111)
    near = rng.uniform(0.4, 0.6, size=(40, 2))
    far = rng.uniform(0.0, 0.1, size=(40, 2))
    vn = rng.standard_normal((40, 2))
    vf = rng.standard_normal((40, 2))
    pos = rng.uniform(0.48, 0.52, size=(10, 2))
    A, da, _ = oracle.fit_at(near, vn, pos, basis="quadratic", weight="wendland", h=0.15)
    B, db, _ = oracle.fit_at(np.concatenate([far, near]), np.concatenate([vf, vn]),
                             pos, basis="quadratic", weight="wendland", h=0.15)
    assert np.array_equal(da, db)
    assert np.array_equal(A, B)


# --------------------------------------------------------------------------
# Hand-derived golden values
# --------------------------------------------------------------------------

def test_golden_fit_cases(oracle):
    with open(os.path.join(GOLDEN, "fit_cases.json")) as fh:
        cases = json.load(fh)["cases"]
    for c in cases:
        F, dg, _ = oracle.fit_at(np.array(c["points"]), np.array(c["values"]),
                                 np.array(c["positions"]), basis=c["basis"],
                                 weight=c["weight"], h=c["h"],
                                 alpha=c.get("alpha", 1.0))
        np.testing.assert_allclose(F.T, np.array(c["expected"]), rtol=0,
                                   atol=c["atol"], err_msg=c["name"])
        assert list(dg) == c["degree"], c["name"]


def test_grid_nodes_on_rectangular_grid(oracle):
    """Grid evaluation sits node (r, c) at (x0 + c dx, y0 + r dy), also when
    dx != dy, and a pixel list picks the same values as the full grid."""
    rng = np.random.default_rng(121)
    pts = rng.random((150, 2))
    vals = rng.standard_normal((150, 2))
    grid = {"x0": 0.05, "y0": 0.1, "dx": 0.04, "dy": 0.025, "width": 23,
            "height": 31}
    F, dg, _ = oracle.fit_grid(pts, vals, grid, basis="quadratic", h=0.12)
    cc, rr = np.meshgrid(np.arange(23), np.arange(31))
    pos = np.stack([0.05 + cc.ravel() * 0.04, 0.1 + rr.ravel() * 0.025], axis=1)
    A, da, _ = oracle.fit_at(pts, vals, pos, basis="quadratic", h=0.12)
    assert np.array_equal(dg.ravel(), da)
    np.testing.assert_array_equal(F.reshape(2, -1), A)
    pix = rng.choice(23 * 31, size=40, replace=False)
    B, db, _ = oracle.fit_grid(pts, vals, grid, basis="quadratic", h=0.12, pixels=pix)
    np.testing.assert_array_equal(B, F.reshape(2, -1)[:, pix])
    np.testing.assert_array_equal(db, dg.ravel()[pix])
