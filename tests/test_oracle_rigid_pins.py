"""Pins of the oracle's rigid MLS (Muelder et al. Eq. 9-10, the rigid
transformation of the image-deformation MLS it cites) against facts that do
not come from the oracle: exact reproduction of rigid motions and of the
identity (the paper's third legibility criterion), the closed-form
weighted Procrustes optimum found by a direct 1-D search over the rotation
angle, and point identity at exact hits of the inverse-distance weight."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar


def grid16():
    return {"x0": 0.5 / 16, "y0": 0.5 / 16, "dx": 1 / 16, "dy": 1 / 16, "width": 16, "height": 16}


def nodes(grid):
    W, H = grid["width"], grid["height"]
    xs = grid["x0"] + np.arange(W) * grid["dx"]
    ys = grid["y0"] + np.arange(H) * grid["dy"]
    return np.meshgrid(xs, ys)


def rot(theta, x, y):
    c, s = math.cos(theta), math.sin(theta)
    return c * x - s * y, s * x + c * y


@pytest.mark.parametrize("theta", [0.0, 0.7, -2.3, math.pi / 2])
@pytest.mark.parametrize("weight,h", [("invpow", 0.1), ("gaussian", 0.15)])
def test_rigid_reproduces_rigid_motion(oracle, theta, weight, h):
    rng = np.random.default_rng(3)
    pts = rng.random((80, 2)).astype(np.float32).astype(np.float64)
    qx, qy = rot(theta, pts[:, 0], pts[:, 1])
    q = np.stack([qx + 0.3, qy - 1.1], axis=1)
    q32 = q.astype(np.float32).astype(np.float64)
    grid = grid16()
    F, deg = oracle.rigid_grid(pts, q32, grid, weight=weight, h=h)
    X, Y = nodes(grid)
    ex, ey = rot(theta, X, Y)
    ok = deg == 1
    assert ok.sum() > 200
    # the values were rounded to float32: the reproduction holds to that rounding
    assert np.abs(F[0][ok] - (ex + 0.3)[ok]).max() < 2e-6
    assert np.abs(F[1][ok] - (ey - 1.1)[ok]).max() < 2e-6


def test_rigid_identity(oracle):
    """Undistorted points (q = p) give the identity map (criterion 3)."""
    rng = np.random.default_rng(4)
    pts = (rng.integers(0, 257, size=(60, 2)) / 256.0)
    grid = grid16()
    F, deg = oracle.rigid_grid(pts, pts, grid, weight="invpow", h=0.1)
    X, Y = nodes(grid)
    ok = deg == 1
    assert ok.all()
    assert np.abs(F[0] - X).max() < 1e-12 and np.abs(F[1] - Y).max() < 1e-12


def test_rigid_is_the_weighted_procrustes_optimum(oracle):
    """f(v) = R(theta*) (v - p*) + q*, theta* minimising
    sum_i w_i |R(theta) dp_i - dq_i|^2, found here by a direct search."""
    rng = np.random.default_rng(8)
    pts = rng.random((40, 2)).astype(np.float32).astype(np.float64)
    q = (rng.random((40, 2)) * 2 - 0.5).astype(np.float32).astype(np.float64)
    grid = grid16()
    pix = rng.choice(256, 25, replace=False)
    F, deg = oracle.rigid_grid(pts, q, grid, weight="gaussian", h=0.2, pixels=pix)
    for k, lin in enumerate(pix):
        r, c = divmod(int(lin), 16)
        v = np.array([grid["x0"] + c * grid["dx"], grid["y0"] + r * grid["dy"]])
        w = np.exp(-((pts - v) ** 2).sum(1) / 0.04)
        ps = (w[:, None] * pts).sum(0) / w.sum()
        qs = (w[:, None] * q).sum(0) / w.sum()
        dp, dq = pts - ps, q - qs

        def cost(t):
            rx, ry = rot(t, dp[:, 0], dp[:, 1])
            return float((w * ((rx - dq[:, 0]) ** 2 + (ry - dq[:, 1]) ** 2)).sum())

        grid_t = np.linspace(-math.pi, math.pi, 721)
        t0 = grid_t[int(np.argmin([cost(t) for t in grid_t]))]
        best = minimize_scalar(cost, bracket=(t0 - 0.01, t0, t0 + 0.01), tol=1e-14).x
        ex, ey = rot(best, v[0] - ps[0], v[1] - ps[1])
        assert deg[k] == 1
        np.testing.assert_allclose(F[:, k], [ex + qs[0], ey + qs[1]], atol=1e-7)


def test_rigid_point_identity(oracle):
    """Exact hits of the inverse-distance weight take the mean of the
    coincident values (criterion 2)."""
    rng = np.random.default_rng(6)
    grid = grid16()
    hit = [grid["x0"] + 5 * grid["dx"], grid["y0"] + 9 * grid["dy"]]
    pts = np.concatenate([np.array([hit, hit]), rng.random((30, 2))])
    q = rng.random((32, 2)).astype(np.float32).astype(np.float64)
    F, deg = oracle.rigid_grid(pts, q, grid, weight="invpow", h=0.1)
    assert deg[9, 5] == oracle.DEG_HIT
    np.testing.assert_allclose(F[:, 9, 5], q[:2].mean(0), atol=1e-15)
    assert (deg == oracle.DEG_HIT).sum() == 1
