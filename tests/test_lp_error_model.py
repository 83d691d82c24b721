"""Where the error of the 16-bit contraction comes from (CPU, no GPU).

tests/lp_model.py reproduces the 16-bit path's rounding steps with numpy
and lets each be switched to exact arithmetic.  On the clustered, noisy
quadratic case that bounds the 16-bit path (the C2 point and attribute
generator, 2,000 points, 13 attributes, h = 0.06 on a 256^2 grid), compared
with the oracle over the nodes where the oracle accepts the quadratic
basis:

* with exact arithmetic the model is the oracle's fit (to the float32
  rounding of the tile-frame coordinates);
* the float32 accumulation of the moments is the dominant error source:
  alone it gives most of the full model's error, while the 16-bit feature
  terms and the split weight with exact sums stay two orders of magnitude
  below it;
* the error grows with the conditioning as 1 / d_min^2 (d_min: the
  oracle's smallest equilibrated Cholesky pivot), the normal equations
  squaring the basis' conditioning: err * d_min^2 stays below 2e-6 in every
  d_min bin from 1e-4 up;
* the consistent weight split (lo times every term but the last) is at
  least five times more accurate than lo times the first term alone.
Tiles: every fourth tile of the grid (64 of 256), which holds the worst
node of the full grid.
"""
import numpy as np
import pytest

from tests import lp_model


@pytest.fixture(scope="module")
def case(oracle):
    from paper_1408_0677_amd import workloads as wl
    w = wl.c2(grid_side=256, n=2000)
    h = 0.06
    of, od, dm = oracle.fit_grid(w.points, w.values, w.grid, basis="quadratic", h=h)
    S = w.values.max(0).astype(np.float64) - w.values.min(0)
    return w, h, of, od, dm, S, list(range(0, 256, 4))


def errors(case, **kw):
    w, h, of, od, dm, S, tiles = case
    f = lp_model.fit_tiles(w.points, w.values, w.grid, h, tiles, **kw)
    err = (np.abs(f - of) / S[:, None, None]).max(axis=0)
    ok = (od == 2) & np.isfinite(f[0])
    return err, ok, dm


def test_model_error_sources(case):
    exact, ok, dm = errors(case, features="f64", weight="exact", accumulate="f64")
    sel = ok & (dm >= 1e-2)
    assert sel.sum() > 5000
    assert exact[sel].max() < 1e-6
    full, _, _ = errors(case)
    acc_only, _, _ = errors(case, features="f32", weight="exact", accumulate="f32")
    terms_only, _, _ = errors(case, accumulate="f64")
    e_full, e_acc, e_terms = full[sel].max(), acc_only[sel].max(), terms_only[sel].max()
    print(f"d_min >= 1e-2: full model {e_full:.2e}, float32 sums alone {e_acc:.2e}, "
          f"16-bit terms and split with exact sums {e_terms:.2e}")
    assert e_acc >= 0.3 * e_full
    assert e_terms <= 0.05 * e_full
    for lo, hi in ((1e-1, 2.0), (1e-2, 1e-1), (1e-3, 1e-2), (1e-4, 1e-3)):
        b = ok & (dm >= lo) & (dm < hi)
        scaled = (full[b] * dm[b] ** 2).max()
        print(f"d_min in [{lo:.0e}, {hi:.0e}): {b.sum()} nodes, max {full[b].max():.2e}, "
              f"max err * d_min^2 {scaled:.2e}")
        assert scaled < 2e-6


def test_consistent_weight_split(case):
    split, ok, dm = errors(case)
    lo1, _, _ = errors(case, weight="lo1")
    sel = ok & (dm >= 1e-2)
    print(f"max error: consistent split {split[sel].max():.2e}, lo x first term only "
          f"{lo1[sel].max():.2e}")
    assert lo1[sel].max() >= 5 * split[sel].max()


def test_attribute_terms_and_lo_weight_are_needed(case):
    """Cheaper carries, with exact sums, against the built scheme with exact
    sums: dropping the third BF16 term of the basis x attribute columns
    (moments keep three), or the lo part of the weight (hi alone on every
    term, still one weight for all features), each costs more than an order
    of magnitude of the terms' error, which is then no longer small beside
    the float32 sums.  Both carries stay."""
    built, ok, dm = errors(case, accumulate="f64")
    rhs2, _, _ = errors(case, accumulate="f64", rhs_terms=2)
    hi, _, _ = errors(case, accumulate="f64", weight="hi")
    full, _, _ = errors(case)
    sel = ok & (dm >= 1e-2)
    e_built, e_rhs2, e_hi, e_full = (x[sel].max() for x in (built, rhs2, hi, full))
    print(f"exact sums: built {e_built:.2e}, two attribute terms {e_rhs2:.2e}, "
          f"hi weight only {e_hi:.2e}; full model {e_full:.2e}")
    assert e_rhs2 >= 10 * e_built
    assert e_hi >= 5 * e_built
    assert e_rhs2 >= 0.3 * e_full
