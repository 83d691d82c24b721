"""GPU parity of mls_fit against the FP64 oracle (through the C ABI).

Tolerance (the plain path, float64 contraction, float32 output): on every
node where both sides are determined and accept the same degree,
|f_gpu - f_oracle| / S_d <= 1e-5 (S_d = range of attribute d's inputs).
The pass set (oracle d_min >= 1e-3) is reported as well.  Degree codes may
differ only where a pivot sits within rounding of the threshold.
"""
import sys

import numpy as np
import pytest

from tests.parity import compare

pytestmark = pytest.mark.gpu
TOL = 1e-5


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def gpu_fit(torch, pts, vals, grid, **kw):
    from paper_1408_0677_amd import api
    P = torch.from_numpy(np.ascontiguousarray(pts, np.float32)).cuda()
    V = torch.from_numpy(np.ascontiguousarray(vals, np.float32)).cuda()
    f, d = api.fit(P, V, grid, **kw)
    torch.cuda.synchronize()
    return f.cpu().numpy(), d.cpu().numpy()


def check(stats, max_mismatch_frac=1e-3):
    assert stats["nan_ok"], stats
    assert stats["nan_mismatch"] <= max(2, max_mismatch_frac * stats["nodes"]), stats
    assert stats["degree_mismatch"] <= max(2, max_mismatch_frac * stats["nodes"]), stats
    assert stats["max_err_same_degree"] <= TOL, stats


def test_c1_full_grid(torch_dev, oracle):
    from paper_1408_0677_amd import workloads as wl
    w = wl.c1()
    note(f"case c1 full grid {w.name}")
    F, deg = gpu_fit(torch_dev, w.points, w.values, w.grid, basis=w.basis, h=w.h)
    of, od, dm = oracle.fit_grid(w.points, w.values, w.grid, basis=w.basis, h=w.h)
    st = compare(F.reshape(w.d, -1), deg, of.reshape(w.d, -1), od, dm, w.values)
    note(str(st))
    check(st)
    assert st["pass_set"] > 0.5 * st["nodes"]


@pytest.mark.parametrize("basis", ["constant", "linear", "quadratic"])
@pytest.mark.parametrize("shape", [(37, 29, 150, 3), (16, 16, 64, 1), (50, 7, 333, 5),
                                   (1, 1, 5, 2), (3, 70, 65, 4)])
def test_ragged_shapes(torch_dev, oracle, basis, shape):
    """Grids that are not multiples of the tile, point counts that are not
    multiples of the chunk, single nodes."""
    W, H, n, D = shape
    note(f"case ragged basis={basis} W={W} H={H} n={n} D={D}")
    rng = np.random.default_rng(W * 1000 + H + n)
    pts = rng.random((n, 2))
    vals = rng.standard_normal((n, D))
    grid = {"x0": 0.02, "y0": 0.03, "dx": 0.96 / max(W - 1, 1), "dy": 0.94 / max(H - 1, 1),
            "width": W, "height": H}
    h = 0.25 if n < 100 else 0.12
    F, deg = gpu_fit(torch_dev, pts, vals, grid, basis=basis, h=h)
    of, od, dm = oracle.fit_grid(pts, vals, grid, basis=basis, h=h)
    st = compare(F.reshape(D, -1), deg, of.reshape(D, -1), od, dm,
                 vals.astype(np.float32))
    note(str(st))
    check(st)


@pytest.mark.parametrize("basis,D", [("linear", 83), ("quadratic", 40), ("constant", 255),
                                     ("linear", 1), ("quadratic", 1)])
def test_attribute_count_limits(torch_dev, oracle, basis, D):
    note(f"case D-limit basis={basis} D={D}")
    rng = np.random.default_rng(D)
    n = 300
    pts = rng.random((n, 2))
    vals = rng.standard_normal((n, D))
    grid = {"x0": 0.1, "y0": 0.1, "dx": 0.8 / 23, "dy": 0.8 / 19, "width": 24, "height": 20}
    F, deg = gpu_fit(torch_dev, pts, vals, grid, basis=basis, h=0.1)
    of, od, dm = oracle.fit_grid(pts, vals, grid, basis=basis, h=0.1)
    st = compare(F.reshape(D, -1), deg, of.reshape(D, -1), od, dm, vals.astype(np.float32))
    note(str({k: v for k, v in st.items() if k != "per_field_max_pass"}))
    check(st)


def test_single_point_and_collinear(torch_dev, oracle):
    """Degenerate inputs: one point (degree 0 everywhere it is seen),
    collinear points (the linear system is singular: degree 0)."""
    grid = {"x0": 0.0, "y0": 0.0, "dx": 0.1, "dy": 0.1, "width": 11, "height": 11}
    pts = np.array([[0.5, 0.5]])
    vals = np.array([[2.5, -1.0]])
    F, deg = gpu_fit(torch_dev, pts, vals, grid, basis="quadratic", h=0.3)
    of, od, dm = oracle.fit_grid(pts, vals, grid, basis="quadratic", h=0.3)
    assert np.array_equal(deg, od)
    det = od != 255
    assert np.all(deg[det] == 0)
    np.testing.assert_array_equal(F[:, det], of[:, det].astype(np.float32))
    t = np.linspace(0.1, 0.9, 40)
    pts = np.stack([t, 0.3 + 0.5 * t], 1)
    vals = np.sin(5 * t)[:, None]
    F, deg = gpu_fit(torch_dev, pts, vals, grid, basis="linear", h=0.2)
    of, od, dm = oracle.fit_grid(pts, vals, grid, basis="linear", h=0.2)
    st = compare(F.reshape(1, -1), deg, of.reshape(1, -1), od, dm, vals.astype(np.float32))
    check(st)
    assert np.all(deg[deg != 255] == 0)


def test_c2_full_size_sampled(torch_dev, oracle):
    """The 1024^2, N = 5,000, D = 13 workload in the benchmark's launch
    configuration, checked on 3,000 random nodes and one full 64 x 64 window."""
    from paper_1408_0677_amd import workloads as wl
    w = wl.c2()
    note(f"case c2 sampled {w.name}")
    F, deg = gpu_fit(torch_dev, w.points, w.values, w.grid, basis=w.basis, h=w.h)
    W = w.grid["width"]
    rng = np.random.default_rng(5)
    win = (np.arange(448, 512)[:, None] * W + np.arange(300, 364)[None, :]).ravel()
    pix = np.unique(np.concatenate([rng.choice(W * W, 3000, replace=False), win]))
    of, od, dm = oracle.fit_grid(w.points, w.values, w.grid, basis=w.basis, h=w.h,
                                 pixels=pix)
    Fg = F.reshape(w.d, -1)[:, pix]
    st = compare(Fg, deg.ravel()[pix], of, od, dm, w.values)
    note(str({k: v for k, v in st.items() if k != "per_field_max_pass"}))
    check(st)
    assert st["pass_set"] > 0.5 * st["nodes"]


@pytest.mark.parametrize("basis", ["linear", "quadratic"])
def test_factor_generation_beyond_the_table_cap(torch_dev, oracle, basis):
    """Where the Gaussian factor tables would pass their 512 MiB cap (here
    70,000 points on a 512^2 grid: 573 MB) the kernel generates the factors
    per tile; checked on sampled nodes and a window like the table path."""
    from paper_1408_0677_amd import api, workloads as wl
    w = wl.c2(grid_side=512, n=70_000)
    assert api.fit_scratch_bytes(w.n, w.d, w.grid, "f64") == 0    # no tables
    note(f"case f64 without tables {basis} n={w.n}")
    h = 0.01 if basis == "linear" else 0.02    # most nodes well conditioned
    F, deg = gpu_fit(torch_dev, w.points, w.values, w.grid, basis=basis, h=h)
    W = w.grid["width"]
    rng = np.random.default_rng(9)
    win = (np.arange(200, 216)[:, None] * W + np.arange(100, 116)[None, :]).ravel()
    pix = np.unique(np.concatenate([rng.choice(W * W, 300, replace=False), win]))
    of, od, dm = oracle.fit_grid(w.points, w.values, w.grid, basis=basis, h=h, pixels=pix)
    st = compare(F.reshape(w.d, -1)[:, pix], deg.ravel()[pix], of, od, dm, w.values)
    note(str({k: v for k, v in st.items() if k != "per_field_max_pass"}))
    check(st)
    assert st["pass_set"] > 0.5 * st["nodes"]


def test_deterministic(torch_dev):
    from paper_1408_0677_amd import workloads as wl
    w = wl.c2(grid_side=256)
    note("case determinism c2@256")
    a, da = gpu_fit(torch_dev, w.points, w.values, w.grid, basis=w.basis, h=w.h)
    b, db = gpu_fit(torch_dev, w.points, w.values, w.grid, basis=w.basis, h=w.h)
    assert np.array_equal(da, db)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_host_pointer_rejected(torch_dev):
    import torch
    from paper_1408_0677_amd import api
    note("case host pointer")
    pts = torch.rand(10, 2)
    vals = torch.rand(10, 1)
    grid = {"x0": 0.0, "y0": 0.0, "dx": 0.1, "dy": 0.1, "width": 4, "height": 4}
    out = torch.empty(1, 4, 4, device="cuda")
    # the binding refuses host tensors before the call ...
    with pytest.raises(ValueError, match="device tensor"):
        api.fit(pts, vals, grid, out=out, want_degree=False)
    # ... and the library itself refuses a host pointer passed straight
    # through the C ABI
    import ctypes
    from paper_1408_0677_amd import _lib
    lib = _lib.load()
    ctx = api.default_context(0)
    w = _lib.MlsWeight(0, 0.1, 1.0)
    g = _lib.MlsGrid(0.0, 0.0, 0.1, 0.1, 4, 4)
    st = lib.mls_fit(ctx.handle, ctypes.c_void_p(pts.data_ptr()),
                     ctypes.c_void_p(vals.data_ptr()), 10, 1, 1, ctypes.byref(w),
                     ctypes.byref(g), 0, None, ctypes.c_void_p(out.data_ptr()), None, None)
    assert st == -1 and b"d_points" in lib.mls_last_error()
    # mis-sized or mistyped outputs, and points/values of different lengths
    P = pts.cuda()
    V = vals.cuda()
    with pytest.raises(ValueError, match="elements"):
        api.fit(P, V, grid, out=torch.empty(1, 4, 3, device="cuda"))
    with pytest.raises(ValueError, match="float32"):
        api.fit(P, V, grid, out=torch.empty(1, 4, 4, device="cuda", dtype=torch.float16))
    with pytest.raises(ValueError, match="elements"):
        api.fit(P, V, grid, degree_out=torch.empty(15, device="cuda", dtype=torch.uint8))
    with pytest.raises(ValueError, match="rows"):
        api.fit(P[:9], V, grid)
    with pytest.raises(ValueError, match="shape"):
        api.fit(P.view(-1), V, grid)


def test_unsupported_weight_reported(torch_dev):
    import torch
    from paper_1408_0677_amd import api
    pts = torch.rand(10, 2, device="cuda")
    vals = torch.rand(10, 1, device="cuda")
    grid = {"x0": 0.0, "y0": 0.0, "dx": 0.1, "dy": 0.1, "width": 4, "height": 4}
    with pytest.raises(api.MlsError) as ei:
        api.fit(pts, vals, grid, weight="wendland", precision="f64")
    assert "UNSUPPORTED" in str(ei.value)
