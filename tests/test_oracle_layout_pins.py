"""Pins of the oracle's planarity-preserving layout iteration (Muelder et
al. Sec. 3.2, Eq. 1-3 and the limiting-line constraint) against facts that
do not come from the oracle: no triangle of the mesh ever flips (the
section's theorem), closed forms for two nodes, the temperature cap, the
limiting lines, and exact equivariance under translation by dyadic shifts
and quarter turns."""
import math

import numpy as np
import pytest

from paper_1408_0677_amd import workloads as wl


def signed_areas(x, tri):
    a, b, c = x[tri[:, 0]], x[tri[:, 1]], x[tri[:, 2]]
    return (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])


def empty_mesh(n):
    z = np.zeros(n + 1, np.int32)
    return {"adj_start": z, "adj": np.zeros(1, np.int32), "fan_start": z,
            "fan": np.zeros(2, np.int32)}


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_no_triangle_flips(oracle, seed):
    """Strong forces and a hot start: the constraint alone keeps every
    triangle's orientation through the whole run."""
    rng = np.random.default_rng(seed)
    pts = rng.random((150, 2))
    mesh = wl.mesh_arrays(pts)
    tri = mesh["triangles"]
    s0 = np.sign(signed_areas(pts, tri))
    x = pts
    for _ in range(10):
        x = oracle.layout(x, mesh, C=5e-3, D=0.02, eta=1e-6, t0=0.05, lam=0.99, iterations=20)
        s = np.sign(signed_areas(x, tri))
        assert np.all(s == s0)
    assert np.abs(x - pts).max() > 1e-3          # the layout did move


def test_two_nodes_repel_by_the_closed_form(oracle):
    C, eta = 0.3, 1e-4
    x = np.array([[0.0, 0.0], [0.5, 0.0]])
    out = oracle.layout(x, empty_mesh(2), C=C, D=1.0, eta=eta, t0=10.0, lam=1.0, iterations=1)
    f = C * 0.5 / (0.5 ** 3 + eta)
    np.testing.assert_allclose(out, [[-f, 0.0], [0.5 + f, 0.0]], rtol=1e-14, atol=1e-15)


def test_spring_closed_form(oracle):
    C, D, eta = 1e-3, 0.2, 1e-5
    x = np.array([[0.1, 0.2], [0.1, 0.8]])
    mesh = {"adj_start": np.array([0, 1, 2], np.int32), "adj": np.array([1, 0], np.int32),
            "fan_start": np.zeros(3, np.int32), "fan": np.zeros(2, np.int32)}
    out = oracle.layout(x, mesh, C=C, D=D, eta=eta, t0=10.0, lam=1.0, iterations=1)
    L = 0.6
    push = C * L / (L ** 3 + eta)          # repulsion, away from the other node
    pull = L * math.log((L + eta) / D) * L  # spring magnitude |V|^2 log(...), towards it
    dy = push - pull                       # node 1 moves by +dy, node 0 by -dy
    np.testing.assert_allclose(out[:, 0], [0.1, 0.1], atol=1e-15)
    np.testing.assert_allclose(out[:, 1], [0.2 - dy, 0.8 + dy], rtol=1e-13)


def test_temperature_caps_every_move(oracle):
    rng = np.random.default_rng(4)
    pts = rng.random((40, 2))
    out = oracle.layout(pts, empty_mesh(40), C=10.0, D=1.0, eta=1e-6, t0=1e-3, lam=1.0,
                        iterations=1)
    step = np.linalg.norm(out - pts, axis=1)
    np.testing.assert_allclose(step, 1e-3, rtol=1e-12)


def test_moves_stop_short_of_limiting_lines(oracle):
    """After one hot iteration every node is still on its own side of every
    limiting line of its triangles (the midline parallel to the opposite
    edge of the starting triangle), at least eta away."""
    rng = np.random.default_rng(5)
    pts = rng.random((80, 2))
    mesh = wl.mesh_arrays(pts)
    eta = 1e-4
    out = oracle.layout(pts, mesh, C=1e-2, D=0.05, eta=eta, t0=1.0, lam=1.0, iterations=1)
    fs, fan = mesh["fan_start"], mesh["fan"]
    worst = np.inf
    for v in range(80):
        for k in range(fs[v], fs[v + 1]):
            tri = [pts[v], pts[fan[2 * k]], pts[fan[2 * k + 1]]]
            for i in range(3):
                # the line through the midpoints of the two edges at corner i
                c, e0, e1 = tri[i], tri[(i + 1) % 3], tri[(i + 2) % 3]
                e = e1 - e0
                nrm = np.array([-e[1], e[0]]) / np.linalg.norm(e)
                line = 0.5 * np.dot(c - e0, nrm)     # its signed offset from edge e0e1
                side0 = np.dot(pts[v] - e0, nrm) - line
                side1 = np.dot(out[v] - e0, nrm) - line
                worst = min(worst, side1 * np.sign(side0))
    assert worst >= eta * (1 - 1e-9)


def test_translation_and_quarter_turn_equivariance(oracle):
    rng = np.random.default_rng(6)
    pts = np.round(rng.random((60, 2)) * 1024) / 1024
    mesh = wl.mesh_arrays(pts)
    kw = dict(C=2e-3, D=0.05, eta=1e-5, t0=0.01, lam=0.97, iterations=5)
    base = oracle.layout(pts, mesh, **kw)
    shifted = oracle.layout(pts + [0.25, -0.5], mesh, **kw)
    np.testing.assert_allclose(shifted - [0.25, -0.5], base, atol=1e-12)
    rot = np.stack([-pts[:, 1], pts[:, 0]], 1)
    out = oracle.layout(rot, mesh, **kw)
    np.testing.assert_array_equal(out, np.stack([-base[:, 1], base[:, 0]], 1))


def test_single_triangle_closed_form(oracle):
    """One triangle, no springs: each corner is pushed by the other two
    corners (Eq. 1) and away from its opposite edge (Eq. 3), -C R / (|R|^2 +
    eta) with R the vector to the foot of the perpendicular; the forces are
    small, so neither the temperature nor the limiting lines bind."""
    C, eta = 1e-4, 1e-6
    x = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    mesh = {"adj_start": np.zeros(4, np.int32), "adj": np.zeros(1, np.int32),
            "fan_start": np.array([0, 1, 2, 3], np.int32),
            "fan": np.array([1, 2, 2, 0, 0, 1], np.int32)}
    out = oracle.layout(x, mesh, C=C, D=1.0, eta=eta, t0=1.0, lam=1.0, iterations=1)
    exp = np.zeros((3, 2))
    for v in range(3):
        for u in range(3):
            if u != v:
                V = x[v] - x[u]
                exp[v] += C * V / (np.linalg.norm(V) ** 3 + eta)
        a, b = x[(v + 1) % 3], x[(v + 2) % 3]
        e = b - a
        foot = a + np.dot(x[v] - a, e) / np.dot(e, e) * e
        R = foot - x[v]
        exp[v] += -C * R / (np.dot(R, R) + eta)
    np.testing.assert_allclose(out - x, exp, rtol=1e-11, atol=1e-16)


def test_step_nodes_matches_full_iteration(oracle):
    """The sampled-node entry makes exactly the first iteration's move of
    the full layout, for any subset and order of nodes."""
    from paper_1408_0677_amd import workloads as wl
    rng = np.random.default_rng(41)
    pts = rng.random((150, 2))
    mesh = wl.mesh_arrays(pts)
    src = np.repeat(np.arange(150), np.diff(mesh["adj_start"]))
    D = float(np.linalg.norm(pts[src] - pts[mesh["adj"]], axis=1).mean())
    prm = dict(C=D ** 3, D=D, eta=1e-3 * D)
    full = oracle.layout(pts, mesh, t0=0.3 * D, lam=0.5, iterations=1, **prm)
    nodes = rng.permutation(150)[:60]
    part = oracle.layout_step_nodes(pts, mesh, t=0.3 * D, nodes=nodes, **prm)
    assert np.array_equal(part, full[nodes])
    with pytest.raises(ValueError):
        oracle.layout_step_nodes(pts, mesh, t=0.3 * D, nodes=[150], **prm)
