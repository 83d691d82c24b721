"""Pins of the oracle's space mappings (Sec. 3.4, Fig. 5b-d), CPU only.

Discrete colour bands are checked against the oracle's marching-squares
cases (pinned on their own), which share the tie rule: for one isovalue a
corner's case bit is set exactly where its band is 1.  Adaptive lines are
checked on planar fields, where line positions are known in closed form
from the geometry (a line of value c of f = a x lies at x = c / a), and by
the fade's closed form at the finer lines, plus invariances.
"""
import numpy as np
import pytest


def pixel_grid(w, h=None):
    h = w if h is None else h
    return {"x0": 0.5 / w, "y0": 0.5 / h, "dx": 1.0 / w, "dy": 1.0 / h, "width": w,
            "height": h}


def smooth_field(rng, grid):
    W, H = grid["width"], grid["height"]
    x = grid["x0"] + grid["dx"] * np.arange(W)
    y = grid["y0"] + grid["dy"] * np.arange(H)
    X, Y = np.meshgrid(x, y)
    a, b, c = rng.uniform(1, 3, 3)
    return (np.sin(a * X) * np.cos(b * Y) + c * X * Y).astype(np.float32)


# ---------------------------------------------------------------- bands

def test_bands_match_contour_case_bits(oracle):
    """One isovalue: a cell's marching-squares case has bit k set exactly
    where corner k's band is 1 (and case 255 exactly where a corner is
    NaN), including values equal to the isovalue."""
    rng = np.random.default_rng(1)
    grid = pixel_grid(40, 31)
    f = smooth_field(rng, grid)
    iso = np.float32(np.median(f))
    f[5, 7] = iso                      # exact ties count as above
    f[12, 3:6] = iso
    f[20, 20] = np.nan
    bands = oracle.map_bands(f[None], np.array([[iso]]))[0]
    cases = oracle.contour(f[None], grid, np.array([[iso]]), f32=True)[0][0, 0]
    H, W = f.shape
    b = bands.astype(np.int64)
    for i in range(H - 1):
        for j in range(W - 1):
            corners = [b[i, j], b[i, j + 1], b[i + 1, j + 1], b[i + 1, j]]
            if any(c == 255 for c in corners):
                assert cases[i, j] == 255
            else:
                assert cases[i, j] == sum(c << k for k, c in enumerate(corners))


def test_bands_several_isovalues(oracle):
    """Bands over several isovalues: unsorted isovalues give the same bands,
    the band counts the isovalues at or below, monotone in the value, 0
    below every isovalue, n_iso above all, 255 for NaN; per field."""
    rng = np.random.default_rng(2)
    vals = rng.standard_normal((2, 500)).astype(np.float32)
    vals[0, :3] = [np.nan, -10.0, 10.0]
    iso = np.array([[-1.0, 0.5, 0.0, 1.5], [0.2, -0.3, 0.9, 2.0]], np.float32)
    vals[1, 3:7] = iso[1]               # ties
    b = oracle.map_bands(vals, iso)
    b_sorted = oracle.map_bands(vals, np.sort(iso, axis=1))
    assert np.array_equal(b, b_sorted)
    assert b[0, 0] == 255 and b[0, 1] == 0 and b[0, 2] == 4
    assert list(b[1, 3:7]) == [2, 1, 3, 4]   # 0.2, -0.3, 0.9, 2.0 count themselves
    for d in range(2):
        ok = ~np.isnan(vals[d])
        order = np.argsort(vals[d][ok], kind="stable")
        assert np.all(np.diff(b[d][ok][order].astype(int)) >= 0)
        assert b[d][ok].min() >= 0 and b[d][ok].max() <= 4


# ------------------------------------------------------- adaptive lines

def planar(grid, a, c=0.0):
    """f = a x + c on the grid's nodes, gradient (a, 0)."""
    W, H = grid["width"], grid["height"]
    x = grid["x0"] + grid["dx"] * np.arange(W)
    f = np.broadcast_to((a * x + c).astype(np.float32), (H, W)).copy()
    g = np.zeros((2, H, W), np.float32)
    g[0] = a
    return f, g


def test_adaptive_level0_lines_on_a_plane(oracle):
    """Steep plane (finer levels faded out): the bright columns sit where
    the lines x = (origin + k spacing) / a fall, one column per line, the
    nearest node column to each line."""
    grid = pixel_grid(200, 4)
    a = 3.7
    f, g = planar(grid, a)
    spacing, origin = 0.25, 0.03
    # level-0 lines 0.25 / (3.7 / 200) = 13.5 px apart; level 1 at 6.8 px
    # is below fade_lo = 8 and contributes nothing
    I = oracle.map_adaptive(f[None], g[None], [[origin, spacing]], grid, n_levels=2,
                            halfwidth=0.6, fade_lo=8.0, fade_hi=20.0)[0]
    bright = np.nonzero(I[0] > 0.2)[0]
    lines = [(origin + k * spacing) / a for k in range(-1, 20)]
    expect = sorted({int(round((xl - grid["x0"]) / grid["dx"])) for xl in lines
                     if grid["x0"] - 0.3 * grid["dx"] <= xl <= grid["x0"] + 199.3 * grid["dx"]})
    assert list(bright) == expect
    assert np.all(I >= 0.0) and np.all(I <= 1.0)
    assert np.array_equal(I[0], I[3])          # constant along y


def test_adaptive_value_on_a_line_and_between(oracle):
    """A node exactly on a level-0 value has intensity 1; a node half way
    between two level-0 values (finer levels faded out) has 0; the
    intensity falls off linearly with the pixel distance to the line."""
    grid = pixel_grid(8)
    spacing = 0.5
    f = np.array([[[1.0, 1.25, 1.0 + 0.5 * 0.3]]], np.float32)   # on, half way, 0.3 of a step
    g = np.zeros((1, 2, 1, 3), np.float32)
    g[0, 0] = 1.0 * 8 * 0.5 / 10.0    # level-0 lines 10 px apart
    I = oracle.map_adaptive(f, g, [[0.0, spacing]], grid, n_levels=1, halfwidth=4.0,
                            fade_lo=100.0, fade_hi=200.0)[0, 0]
    assert I[0] == 1.0
    assert I[1] == 0.0
    assert I[2] == pytest.approx(1.0 - 3.0 / 4.0, abs=1e-6)   # 0.3 of 10 px = 3 px


def test_adaptive_finer_levels_fade_in(oracle):
    """Shallow plane (space expanded): level-1 lines appear between the
    level-0 lines with opacity clamp((s_1 - fade_lo) / (fade_hi - fade_lo)),
    s_1 the level-1 spacing in pixels; fully visible ones double the line
    count."""
    grid = pixel_grid(400, 2)
    spacing = 0.5
    for a, expect_a1 in ((0.5 / (40 * grid["dx"]), 1.0),      # s_0 = 40 px, s_1 = 20 px
                         (0.5 / (24 * grid["dx"]), 0.5)):     # s_1 = 12 px: half way in [8, 16]
        # f = a (x - x0): every line falls on a node column
        f, g = planar(grid, a, c=-a * grid["x0"])
        I = oracle.map_adaptive(f[None], g[None], [[0.0, spacing]], grid, n_levels=2,
                                halfwidth=0.75, fade_lo=8.0, fade_hi=16.0)[0, 0]
        # level-1 values half way between level-0 values: x = x0 + (k + 1/2) spacing / a
        xs = [grid["x0"] + (k + 0.5) * spacing / a for k in range(0, 20)]
        cols = [int(round((x - grid["x0"]) / grid["dx"])) for x in xs
                if 0 <= (x - grid["x0"]) / grid["dx"] <= 399]
        peaks = [I[c] for c in cols]
        # the nearest column is within half a pixel of the line (float32 values)
        for pk in peaks:
            assert expect_a1 * (1 - 0.5 / 0.75) - 1e-4 <= pk <= expect_a1 + 1e-4
        assert min(peaks) == pytest.approx(expect_a1, abs=1e-4)
        # the level-0 columns stay at full intensity
        assert I[0] == pytest.approx(1.0, abs=1e-4)


def test_adaptive_invariances(oracle):
    """Scaling values, gradients, origin and spacing by one factor, or
    shifting values and origin by whole level-0 steps, leaves the
    intensity unchanged; NaN values give NaN, zero gradients 0."""
    rng = np.random.default_rng(3)
    grid = pixel_grid(30, 20)
    f = smooth_field(rng, grid)
    g = (rng.standard_normal((2, 20, 30)) * 2.0).astype(np.float32)
    kw = dict(n_levels=3, halfwidth=1.0, fade_lo=4.0, fade_hi=12.0)
    base = oracle.map_adaptive(f[None], g[None], [[0.1, 0.125]], grid, **kw)[0]
    scaled = oracle.map_adaptive((4 * f)[None], (4 * g)[None], [[0.4, 0.5]], grid, **kw)[0]
    assert np.allclose(base, scaled, atol=1e-9)
    shifted = oracle.map_adaptive((f + np.float32(0.25))[None], g[None], [[0.35, 0.125]], grid,
                                  **kw)[0]
    assert np.allclose(base, shifted, atol=1e-5)
    f2 = f.copy()
    f2[3, 4] = np.nan
    g2 = g.copy()
    g2[:, 5, 6] = 0.0
    out = oracle.map_adaptive(f2[None], g2[None], [[0.1, 0.125]], grid, **kw)[0]
    assert np.isnan(out[3, 4]) and out[5, 6] == 0.0
    assert np.all((out[~np.isnan(out)] >= 0) & (out[~np.isnan(out)] <= 1))
