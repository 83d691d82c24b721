"""Pins of the oracle's marching squares (contour lines of the MLS output,
Muelder et al. Sec. 3.4) against geometry that does not come from the oracle:
the exhaustive 2x2 case table, orientation by a side-of-line test, exact
crossings on planar fields, closed loops around a radial field."""
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
UNIT = {"x0": 0.0, "y0": 0.0, "dx": 1.0, "dy": 1.0}

# corner positions of the unit cell: v0 (0,0), v1 (1,0), v2 (1,1), v3 (0,1)
CORNERS = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
# field[i][j] indices of the corners for a 2x2 grid (row = y)
CORNER_RC = [(0, 0), (0, 1), (1, 1), (1, 0)]


def cell_field(vals):
    f = np.zeros((2, 2))
    for k, (r, c) in enumerate(CORNER_RC):
        f[r, c] = vals[k]
    return f


def edge_of(pt):
    x, y = pt
    if y == 0.0 and 0.0 <= x <= 1.0:
        return 0
    if x == 1.0:
        return 1
    if y == 1.0:
        return 2
    if x == 0.0:
        return 3
    raise AssertionError(f"point {pt} is not on the cell boundary")


def side(seg, p):
    """> 0 if p is left of the directed segment."""
    (ax, ay, bx, by) = seg
    return (bx - ax) * (p[1] - ay) - (by - ay) * (p[0] - ax)


def test_golden_case_table(oracle):
    """All 16 corner patterns, both saddle resolutions, against the
    hand-derived table in tests/golden/marching_squares_cases.json."""
    with open(os.path.join(GOLDEN, "marching_squares_cases.json")) as fh:
        table = json.load(fh)["cases"]
    for entry in table:
        cs = entry["case"]
        for hi, lo, key in ((2.0, -1.0, "joined"), (1.0, -2.0, "separated")):
            vals = [hi if (cs >> k) & 1 else lo for k in range(4)]
            cases, segs, ids = oracle.contour(cell_field(vals)[None], UNIT,
                                              np.array([[0.0]]))
            assert cases[0, 0, 0, 0] == cs
            want = entry.get(key, entry.get("segments"))
            got = [[edge_of(s[:2]), edge_of(s[2:])] for s in segs]
            assert got == want, (cs, key, got, want)


@pytest.mark.parametrize("cs", range(16))
@pytest.mark.parametrize("f32", [False, True])
def test_orientation_and_crossings(oracle, cs, f32):
    """Every segment separates the corners it cuts off: a corner alone on one
    side of the segment's line is above iff it is on the left; for a 2-2
    split all left corners are above and all right corners below.  Crossing
    points interpolate the edge to the isovalue."""
    rng = np.random.default_rng(cs)
    for trial in range(20):
        vals = [rng.uniform(0.1, 2.0) if (cs >> k) & 1 else -rng.uniform(0.1, 2.0)
                for k in range(4)]
        iso = rng.uniform(-0.05, 0.05)
        vals = [v + iso for v in vals]
        f = cell_field(vals)
        cases, segs, _ = oracle.contour(f[None], UNIT, np.array([[iso]]), f32=f32)
        assert cases[0, 0, 0, 0] == cs
        for s in segs:
            sides = np.array([side(s, c) for c in CORNERS])
            left, right = np.nonzero(sides > 0)[0], np.nonzero(sides < 0)[0]
            above = [(cs >> k) & 1 == 1 for k in range(4)]
            if len(left) == 1:
                assert above[left[0]]
            if len(right) == 1:
                assert not above[right[0]]
            if len(left) == 2 and len(right) == 2:
                assert all(above[k] for k in left)
                assert not any(above[k] for k in right)
            for pt in (s[:2], s[2:]):
                e = edge_of(pt)
                a, b = [(0, 1), (1, 2), (3, 2), (0, 3)][e]
                t = np.linalg.norm(pt - CORNERS[a])
                lerp = vals[a] + t * (vals[b] - vals[a])
                assert abs(lerp - iso) <= (1e-6 if f32 else 1e-14) * 4


def test_saddle_resolution_by_centre(oracle):
    # case 5: v0, v2 above; centre ((v0+v1)+(v2+v3))/4
    f = cell_field([1.0, -1.0, 1.0, -1.0])       # centre 0 == iso -> joined
    _, segs, _ = oracle.contour(f[None], UNIT, np.array([[0.0]]))
    assert [[edge_of(s[:2]), edge_of(s[2:])] for s in segs] == [[0, 1], [2, 3]]
    f = cell_field([1.0, -1.0, 1.0, -1.5])       # centre < iso -> separated
    _, segs, _ = oracle.contour(f[None], UNIT, np.array([[0.0]]))
    assert [[edge_of(s[:2]), edge_of(s[2:])] for s in segs] == [[0, 3], [2, 1]]


def test_ties_and_nan(oracle):
    f = cell_field([0.5, 0.0, 0.0, 0.0])         # corner equal to iso is above
    cases, _, _ = oracle.contour(f[None], UNIT, np.array([[0.5]]))
    assert cases[0, 0, 0, 0] == 1
    f = cell_field([0.5, np.nan, 0.0, 0.0])
    cases, segs, _ = oracle.contour(f[None], UNIT, np.array([[0.25]]))
    assert cases[0, 0, 0, 0] == 255 and len(segs) == 0


def test_planar_field_endpoints_on_line(oracle):
    W, H = 37, 29
    grid = {"x0": 0.1, "y0": -0.3, "dx": 0.03125, "dy": 0.0625, "width": W,
            "height": H}
    xs = grid["x0"] + np.arange(W) * grid["dx"]
    ys = grid["y0"] + np.arange(H) * grid["dy"]
    a, b, c = 0.7, -1.3, 0.2
    f = a * xs[None, :] + b * ys[:, None] + c
    iso = np.array([[-0.5, 0.0, 0.3, 0.9]])
    cases, segs, ids = oracle.contour(f[None], grid, iso)
    assert len(segs) > 50
    lv = iso[0, ids[:, 1]]
    for col in (0, 2):
        g = a * segs[:, col] + b * segs[:, col + 1] + c
        assert np.abs(g - lv).max() <= 4 * np.finfo(np.float64).eps * 4
    # a planar field has no saddles and one segment per crossed cell
    assert not np.isin(cases, [5, 10]).any()


def test_radial_field_closed_loops(oracle):
    n = 64
    grid = {"x0": 0.5 / n, "y0": 0.5 / n, "dx": 1.0 / n, "dy": 1.0 / n,
            "width": n, "height": n}
    xs = grid["x0"] + np.arange(n) * grid["dx"]
    r = np.sqrt((xs[None, :] - 0.5) ** 2 + (xs[:, None] - 0.5) ** 2)
    iso = np.array([[0.1, 0.2, 0.33]])
    _, segs, ids = oracle.contour(r[None], grid, iso)
    for k, R in enumerate(iso[0]):
        s = segs[ids[:, 1] == k]
        starts = {tuple(p) for p in s[:, :2]}
        ends = {tuple(p) for p in s[:, 2:]}
        assert len(starts) == len(s) and len(ends) == len(s)
        assert starts == ends                     # every loop closes
        rad = np.hypot(s[:, 0] - 0.5, s[:, 1] - 0.5)
        assert np.abs(rad - R).max() < 2.0 * grid["dx"] ** 2 / R + 1e-12
        # r >= iso (outside) is the above region: it lies on the left, so the
        # loop runs clockwise (negative signed area)
        area = 0.5 * np.sum(s[:, 0] * s[:, 3] - s[:, 2] * s[:, 1])
        assert area < 0 and abs(abs(area) - math.pi * R * R) < 0.02 * R


def test_f32_variant_tracks_f64(oracle):
    rng = np.random.default_rng(7)
    f = rng.standard_normal((3, 20, 24)).astype(np.float32)
    iso = rng.standard_normal((3, 4)).astype(np.float32)
    c64, s64, i64 = oracle.contour(f.astype(np.float64), UNIT, iso.astype(np.float64))
    c32, s32, i32 = oracle.contour(f, UNIT, iso, f32=True)
    assert np.array_equal(i64, i32)
    # cases can differ only where the saddle centre rounds across the isovalue
    diff = c64 != c32
    assert diff.sum() == 0
    assert np.abs(s64 - s32).max() <= 2 * np.finfo(np.float32).eps * 24


def test_segment_order(oracle):
    """Segments come in (field, iso, cell, k) order."""
    rng = np.random.default_rng(9)
    f = rng.standard_normal((2, 12, 13))
    iso = rng.standard_normal((2, 3)) * 0.5
    _, _, ids = oracle.contour(f, UNIT, iso)
    key = ids[:, 0].astype(np.int64) * 10 ** 8 + ids[:, 1] * 10 ** 6 + ids[:, 2]
    assert np.all(np.diff(key) >= 0)
