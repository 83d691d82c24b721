"""Pins of the oracle's gradient output (the slope of the local fit at the
node, (c_1, c_2) / h, which the adaptive contour-line mapping of Muelder et
al. Sec. 3.4 needs) against facts that do not come from the oracle: exact
slopes of reproduced polynomials, the slope coefficients of an SVD
least-squares solve in an unscaled basis, mirror symmetry, and the
constant-basis, undetermined and exact-hit cases."""
import numpy as np
import pytest

from tests.test_oracle_pins import (basis_cols, dyadic_points, gauss_w, poly_eval,
                                    positions)


@pytest.mark.parametrize("basis,deg", [("linear", 1), ("quadratic", 2)])
@pytest.mark.parametrize("weight,h", [("gaussian", 0.12), ("wendland", 0.35),
                                      ("invpow", 0.1)])
def test_gradient_of_reproduced_polynomial(oracle, basis, deg, weight, h):
    rng = np.random.default_rng(21 + deg)
    pts = dyadic_points(rng, 300)
    coef = rng.integers(-7, 8, size=6) / 8.0
    if deg == 1:
        coef[3:] = 0.0
    f = poly_eval(coef, pts[:, 0], pts[:, 1])
    pos = positions(rng, 200)
    _, degree, dmin, g = oracle.fit_at(pts, f, pos, basis=basis, weight=weight, h=h,
                                       grads=True)
    ok = (degree == deg) & (dmin >= 1e-3)
    assert ok.sum() > 150
    x, y = pos[:, 0], pos[:, 1]
    gx = coef[1] + 2 * coef[3] * x + coef[4] * y
    gy = coef[2] + coef[4] * x + 2 * coef[5] * y
    scale = np.abs(coef).sum()
    assert np.abs(g[0, 0] - gx)[ok].max() <= 1e-10 * scale
    assert np.abs(g[0, 1] - gy)[ok].max() <= 1e-10 * scale


@pytest.mark.parametrize("basis,deg", [("linear", 1), ("quadratic", 2)])
def test_gradient_bruteforce_lstsq(oracle, basis, deg):
    """The slope coefficients of the weighted least-squares fit in an unscaled
    basis centred on the position (so no 1/h appears) by SVD."""
    rng = np.random.default_rng(60 + deg)
    for trial in range(8):
        n = int(rng.integers(9, 13))
        pts = rng.random((n, 2)).astype(np.float32).astype(np.float64)
        vals = rng.standard_normal((n, 2)).astype(np.float32).astype(np.float64)
        pos = rng.uniform(0.3, 0.7, size=(3, 2))
        _, dg, dmin, g = oracle.fit_at(pts, vals, pos, basis=basis, h=0.6, grads=True)
        for k in range(3):
            assert dg[k] == deg and dmin[k] > 1e-6
            dx, dy = pts[:, 0] - pos[k, 0], pts[:, 1] - pos[k, 1]
            B = basis_cols(dx, dy, deg)
            sw = np.sqrt(gauss_w(pts, pos[k], 0.6))
            coef, *_ = np.linalg.lstsq(sw[:, None] * B, sw[:, None] * vals, rcond=None)
            np.testing.assert_allclose(g[:, 0, k], coef[1], rtol=1e-9, atol=1e-9)
            np.testing.assert_allclose(g[:, 1, k], coef[2], rtol=1e-9, atol=1e-9)


def test_gradient_mirror_symmetry(oracle):
    """x -> 1 - x flips the x slope and keeps the y slope."""
    rng = np.random.default_rng(97)
    pts = dyadic_points(rng, 200)
    vals = rng.standard_normal((200, 2)).astype(np.float32)
    grid = {"x0": 0.5 / 32, "y0": 0.5 / 32, "dx": 1 / 32, "dy": 1 / 32,
            "width": 32, "height": 32}
    mir = pts.copy()
    mir[:, 0] = 1.0 - mir[:, 0]
    for basis in ("linear", "quadratic"):
        _, da, _, ga = oracle.fit_grid(pts, vals, grid, basis=basis, h=0.07, grads=True)
        _, db, _, gb = oracle.fit_grid(mir, vals, grid, basis=basis, h=0.07, grads=True)
        det = (da != oracle.DEG_NAN) & (da >= 1)
        np.testing.assert_allclose(ga[:, 0][:, det], -gb[:, 0, :, ::-1][:, det], atol=1e-9)
        np.testing.assert_allclose(ga[:, 1][:, det], gb[:, 1, :, ::-1][:, det], atol=1e-9)


def test_gradient_special_cases(oracle):
    """Constant basis: zero slope.  Undetermined nodes: NaN.  Exact hits of
    the inverse-distance weight: NaN (the field jumps to the point's value)."""
    rng = np.random.default_rng(5)
    pts = rng.random((100, 2)) * 0.3
    vals = rng.standard_normal((100, 2))
    grid = {"x0": 0.5 / 16, "y0": 0.5 / 16, "dx": 1 / 16, "dy": 1 / 16,
            "width": 16, "height": 16}
    _, dg, _, g = oracle.fit_grid(pts, vals, grid, basis="constant", h=0.05, grads=True)
    det = dg != oracle.DEG_NAN
    assert det.any() and (~det).any()
    assert np.all(g[:, :, det] == 0.0)
    assert np.all(np.isnan(g[:, :, ~det]))
    hit = np.array([[grid["x0"] + 3 * grid["dx"], grid["y0"] + 2 * grid["dy"]]])
    pts2 = np.concatenate([hit, rng.random((50, 2))])
    vals2 = rng.standard_normal((51, 1))
    _, dh, _, gh = oracle.fit_grid(pts2, vals2, grid, basis="linear", weight="invpow",
                                   h=0.1, grads=True)
    assert dh[2, 3] == oracle.DEG_HIT
    assert np.all(np.isnan(gh[:, :, 2, 3]))
    others = dh != oracle.DEG_HIT
    assert np.all(np.isfinite(gh[:, :, others]))
