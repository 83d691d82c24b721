"""GPU parity of mls_contour against the oracle's marching squares.

Same input (the oracle's binary32 variant on the very fields the GPU reads):
cases, segment order and ids equal everywhere, endpoints bit-identical.
Oracle fields vs GPU fields (both from their own fit): cases equal on every
cell whose corners and saddle centre are farther than the fit tolerance
from the isovalue.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def gpu_contour(torch, fields, grid, iso, **kw):
    from paper_1408_0677_amd import api
    F = torch.from_numpy(np.ascontiguousarray(fields, np.float32)).cuda()
    I = torch.from_numpy(np.ascontiguousarray(iso, np.float32)).cuda()
    segs, ids, cases = api.contour(F, grid, I, **kw)
    torch.cuda.synchronize()
    return (segs.cpu().numpy(), None if ids is None else ids.cpu().numpy(),
            None if cases is None else cases.cpu().numpy())


def same_input_check(torch, oracle, fields, grid, iso):
    segs, ids, cases = gpu_contour(torch, fields, grid, iso)
    oc, os_, oi = oracle.contour(fields, grid, iso, f32=True)
    assert np.array_equal(cases, oc)
    assert np.array_equal(ids, oi)
    assert segs.shape == os_.shape
    assert np.array_equal(segs, os_.astype(np.float32)), np.abs(segs - os_).max()
    return len(segs)


@pytest.mark.parametrize("shape", [(2, 2, 1, 1), (7, 5, 2, 3), (64, 33, 3, 4), (300, 257, 2, 5)])
def test_random_fields_same_input(torch_dev, oracle, shape):
    W, H, D, n_iso = shape
    note(f"case random fields W={W} H={H} D={D} n_iso={n_iso}")
    rng = np.random.default_rng(W + H)
    f = rng.standard_normal((D, H, W)).astype(np.float32)
    f[:, ::7, ::5] = np.nan if W > 10 else f[:, ::7, ::5]
    iso = (rng.standard_normal((D, n_iso)) * 0.5).astype(np.float32)
    grid = {"x0": 0.1, "y0": -0.2, "dx": 0.013, "dy": 0.021, "width": W, "height": H}
    same_input_check(torch_dev, oracle, f, grid, iso)


def test_many_isovalues_without_cases(torch_dev, oracle):
    """The launch configuration without the case array, where a wave visits
    only the isovalues inside its corner range, with 150 isovalues per field
    (three batches of 64, one per lane) on smooth fields, so that a chunk
    crosses many isovalues and its queue of crossed cells is drained several
    times: segments and ids equal the oracle's on the same input."""
    note("case 150 isovalues, no case array")
    rng = np.random.default_rng(5)
    W, H, D, n_iso = 203, 151, 2, 150
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    f = np.stack([np.sin(xx / 9.0) * np.cos(yy / 7.0) * 3.0 + 0.01 * rng.standard_normal((H, W)),
                  (xx - 100.0) ** 2 / 900.0 - (yy - 70.0) ** 2 / 700.0]).astype(np.float32)
    f[1, 40, 40:60] = np.nan
    iso = np.stack([np.linspace(-3.0, 3.0, n_iso), np.linspace(-8.0, 12.0, n_iso)]).astype(
        np.float32)
    grid = {"x0": -1.0, "y0": 0.5, "dx": 0.01, "dy": 0.02, "width": W, "height": H}
    segs, ids, cases = gpu_contour(torch_dev, f, grid, iso, want_cases=False)
    assert cases is None
    oc, os_, oi = oracle.contour(f, grid, iso, f32=True)
    note(f"{len(segs)} segments")
    assert len(segs) > 10000
    assert np.array_equal(ids, oi)
    assert np.array_equal(segs, os_.astype(np.float32))


def test_every_case_and_saddle(torch_dev, oracle):
    """A field built to contain all 16 cases and both saddle resolutions,
    plus corners equal to the isovalue."""
    note("case exhaustive cells")
    rng = np.random.default_rng(1)
    f = rng.choice(np.array([-2.0, -1.0, 0.0, 1.0, 2.0], np.float32), size=(40, 40))
    f = f.astype(np.float32)
    iso = np.array([[0.0, 0.5, -1.0]], np.float32)
    grid = {"x0": 0.0, "y0": 0.0, "dx": 1.0, "dy": 1.0, "width": 40, "height": 40}
    same_input_check(torch_dev, oracle, f[None], grid, iso)
    _, _, cases = gpu_contour(torch_dev, f[None], grid, iso)
    assert set(np.unique(cases)) >= set(range(16))


def test_capacity_protocol(torch_dev, oracle):
    import torch
    from paper_1408_0677_amd import api
    note("case capacity protocol")
    rng = np.random.default_rng(2)
    f = rng.standard_normal((1, 30, 30)).astype(np.float32)
    iso = np.zeros((1, 1), np.float32)
    grid = {"x0": 0.0, "y0": 0.0, "dx": 1.0, "dy": 1.0, "width": 30, "height": 30}
    full, _, _ = gpu_contour(torch_dev, f, grid, iso)
    with pytest.raises(api.MlsError) as ei:
        gpu_contour(torch_dev, f, grid, iso, capacity=len(full) - 1)
    assert "CAPACITY" in str(ei.value)
    segs, _, _ = gpu_contour(torch_dev, f, grid, iso, capacity=len(full) + 5)
    assert np.array_equal(segs, full)


def test_c2_fields_contours(torch_dev, oracle):
    """Contours of the 1024^2 workload's fitted fields, 10 isovalues per field:
    same-input exactness on the GPU fields, and agreement with contours of the
    oracle's own fields away from the isovalues (checked on a window)."""
    from paper_1408_0677_amd import api, workloads as wl
    import torch
    w = wl.c2()
    note(f"case c2 contours {w.name}")
    P = torch.from_numpy(w.points).cuda()
    V = torch.from_numpy(w.values).cuda()
    F, deg = api.fit(P, V, w.grid, basis=w.basis, h=w.h)
    iso = torch.from_numpy(w.iso()).cuda()
    segs, ids, cases = api.contour(F, w.grid, iso)
    torch.cuda.synchronize()
    Fh = F.cpu().numpy()
    # same input on a 3-field subset (keeps the oracle fast)
    oc, os_, oi = oracle.contour(Fh[:3], w.grid, w.iso()[:3], f32=True)
    n3 = int(np.sum(ids.cpu().numpy()[:, 0] < 3))
    assert np.array_equal(cases.cpu().numpy()[:3], oc)
    assert np.array_equal(ids.cpu().numpy()[:n3], oi)
    assert np.array_equal(segs.cpu().numpy()[:n3], os_.astype(np.float32))
    # oracle fields on a 96 x 96 window: cases agree away from the isovalue
    W = w.grid["width"]
    r0, c0, k = 400, 500, 96
    rows, cols = np.arange(r0, r0 + k), np.arange(c0, c0 + k)
    pix = (rows[:, None] * W + cols[None, :]).ravel()
    of, od, _ = oracle.fit_grid(w.points, w.values, w.grid, basis=w.basis, h=w.h, pixels=pix)
    of = of.reshape(w.d, k, k)
    sub = {"x0": w.grid["x0"] + c0 * w.grid["dx"], "y0": w.grid["y0"] + r0 * w.grid["dy"],
           "dx": w.grid["dx"], "dy": w.grid["dy"], "width": k, "height": k}
    isoh = w.iso()
    ocase, _, _ = oracle.contour(of, sub, isoh)
    gcase = cases.cpu().numpy()[:, :, r0:r0 + k - 1, c0:c0 + k - 1]
    S = (w.values.max(0) - w.values.min(0)).astype(np.float64)
    tol = 1e-5 * S[:, None, None, None]
    v0, v1, v3, v2 = of[:, None, :-1, :-1], of[:, None, :-1, 1:], of[:, None, 1:, :-1], of[:, None, 1:, 1:]
    centre = ((v0 + v1) + (v2 + v3)) * 0.25
    lv = isoh[:, :, None, None].astype(np.float64)
    far = np.ones_like(gcase, dtype=bool)
    for v in (v0, v1, v2, v3, centre):
        far &= np.abs(v - lv) > tol
    assert far.mean() > 0.99
    assert np.array_equal(gcase[far], ocase[far])


def test_c5_fields_contours_same_input(torch_dev, oracle):
    """Contours at the 4096^2 / 16-field / 16-isovalue shape the bench times,
    in its launch configuration (no cases): the first field's segments and
    ids equal the oracle's on the same fields, bit for bit, and the segment
    count over all fields equals the oracle's count field by field on two
    more fields."""
    from paper_1408_0677_amd import api, workloads as wl
    import torch
    w = wl.c5()
    note(f"case c5 contours {w.name}")
    P = torch.from_numpy(w.points).cuda()
    V = torch.from_numpy(w.values).cuda()
    F, _ = api.fit(P, V, w.grid, basis=w.basis, weight=w.weight, h=w.h, precision="bf16")
    iso = torch.from_numpy(w.iso()).cuda()
    segs, ids, _ = api.contour(F, w.grid, iso, want_cases=False)
    torch.cuda.synchronize()
    ids_h = ids.cpu().numpy()
    segs_h = segs.cpu().numpy()
    Fh = F.cpu().numpy()
    for d in (0, 7, 15):
        _, os_, oi = oracle.contour(Fh[d:d + 1], w.grid, w.iso()[d:d + 1], f32=True)
        mine = ids_h[:, 0] == d
        note(f"field {d}: {int(mine.sum())} segments")
        assert mine.sum() == oi.shape[0] and oi.shape[0] > 1000
        assert np.array_equal(ids_h[mine][:, 1:], oi[:, 1:])
        assert np.array_equal(segs_h[mine], os_.astype(np.float32))
