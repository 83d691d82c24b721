"""GPU parity of the inverse-distance weight (Eq. 4) on the float64 path,
including the exact-hit rule (a node on data points takes their mean,
degree code 254), against the FP64 oracle.  Bound: 1e-5 relative to the
attribute range on the nodes where both sides agree on the degree and the
oracle's d_min >= 1e-3 (the weight itself is formed with float32 exp2/log2,
a common relative error of about 1e-7 per pair)."""
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


@pytest.mark.parametrize("alpha", [0.5, 1.0, 1.5, 2.0])
@pytest.mark.parametrize("basis", ["constant", "linear", "quadratic"])
def test_invpow_matches_oracle(torch_dev, oracle, basis, alpha):
    from paper_1408_0677_amd import workloads as wl
    note(f"case invpow {basis} alpha={alpha}")
    rng = np.random.default_rng(int(alpha * 10) + len(basis))
    pts = rng.random((300, 2))
    vals = wl.analytic_fields(rng, pts)
    grid = {"x0": 0.013, "y0": 0.021, "dx": 0.0151, "dy": 0.0137, "width": 70, "height": 53}
    F, deg = gpu_fit(torch_dev, pts, vals, grid, basis=basis, weight="invpow", h=0.05,
                     alpha=alpha)
    of, od, dm = oracle.fit_grid(pts, vals, grid, basis=basis, weight="invpow", h=0.05,
                                 alpha=alpha)
    st = compare(F.reshape(4, -1), deg, of.reshape(4, -1), od, dm, vals.astype(np.float32))
    note(str({k: v for k, v in st.items() if k != "per_field_max_pass"}))
    assert st["nan_ok"] and st["nan_mismatch"] == 0
    assert st["degree_mismatch"] <= 2
    assert st["max_err_pass"] <= TOL


@pytest.mark.parametrize("extra", [200, 5000])
def test_exact_hits_take_the_mean(torch_dev, oracle, extra):
    """Points placed exactly on grid nodes (pixel centres are dyadic, so the
    float32 point equals the float64 node position): single hits, a double
    and a triple hit with different values, and near misses 1e-6 away, among
    `extra` random points (211 points in all take the one-workgroup hit
    pass, 5,011 the radix-sorted one)."""
    from paper_1408_0677_amd import workloads as wl
    note(f"case invpow exact hits, {extra} extra points")
    rng = np.random.default_rng(9)
    # spacings 1/64 and 1/32: node positions are exact in float32 and float64
    grid = wl.pixel_grid(64, 32)
    W, H = 64, 32
    node = lambda r, c: (grid["x0"] + c * grid["dx"], grid["y0"] + r * grid["dy"])
    hits = [node(3, 5), node(10, 60), node(31, 0), node(0, 63), node(20, 20), node(20, 20),
            node(25, 7), node(25, 7), node(25, 7)]
    near = [(x + 1e-6, y) for x, y in [node(5, 5), node(28, 40)]]
    pts = np.concatenate([np.array(hits), np.array(near), rng.random((extra, 2))])
    vals = rng.standard_normal((pts.shape[0], 3))
    F, deg = gpu_fit(torch_dev, pts, vals, grid, basis="linear", weight="invpow", h=0.05)
    of, od, dm = oracle.fit_grid(pts, vals, grid, basis="linear", weight="invpow", h=0.05)
    hit_nodes = [(3, 5), (10, 60), (31, 0), (0, 63), (20, 20), (25, 7)]
    for r, c in hit_nodes:
        assert deg[r, c] == 254 and od[r, c] == 254, (r, c)
        assert np.allclose(F[:, r, c], of[:, r, c], rtol=0, atol=1e-6), (r, c)
    assert np.allclose(F[:, 20, 20], vals[4:6].astype(np.float32).astype(np.float64).mean(0),
                       atol=1e-6)
    assert int((deg == 254).sum()) == len(hit_nodes)
    st = compare(F.reshape(3, -1), deg, of.reshape(3, -1), od, dm, vals.astype(np.float32))
    note(str({k: v for k, v in st.items() if k != "per_field_max_pass"}))
    assert st["degree_mismatch"] == 0 and st["nan_mismatch"] == 0
    assert st["max_err_pass"] <= TOL


@pytest.mark.parametrize("basis", ["linear", "constant"])
@pytest.mark.parametrize("n", [306, 2245])
def test_table1_shapes_sampled(torch_dev, oracle, n, basis):
    """The timing-table shape (600 x 600, N uniform, D = 2, alpha = 1) on
    sampled nodes: Affine MLS (linear basis) and Mean MLS (constant
    basis), as the bench times them."""
    from paper_1408_0677_amd import workloads as wl
    w = wl.t1(n)
    note(f"case {w.name} {basis}")
    F, deg = gpu_fit(torch_dev, w.points, w.values, w.grid, basis=basis, weight=w.weight,
                     h=w.h, alpha=w.alpha)
    rng = np.random.default_rng(n)
    pix = rng.choice(600 * 600, 3000, replace=False)
    of, od, dm = oracle.fit_grid(w.points, w.values, w.grid, basis=basis, weight=w.weight,
                                 h=w.h, alpha=w.alpha, pixels=pix)
    st = compare(F.reshape(2, -1)[:, pix], deg.ravel()[pix], of, od, dm, w.values)
    note(str({k: v for k, v in st.items() if k != "per_field_max_pass"}))
    assert st["degree_mismatch"] == 0 and st["nan_ok"]
    assert st["max_err_pass"] <= TOL


def test_invpow_refused_where_unsupported(torch_dev):
    import torch
    from paper_1408_0677_amd import api
    P = torch.rand(50, 2, device="cuda")
    V = torch.rand(50, 2, device="cuda")
    grid = {"x0": 0.0, "y0": 0.0, "dx": 0.05, "dy": 0.05, "width": 8, "height": 8}
    for prec in ("bf16", "fp16"):
        with pytest.raises(api.MlsError) as ei:
            api.fit(P, V, grid, weight="invpow", h=0.05, precision=prec)
        assert "UNSUPPORTED" in str(ei.value)
    flat = dict(grid, dx=0.0)
    with pytest.raises(api.MlsError) as ei:
        api.fit(P, V, flat, weight="invpow", h=0.05)
    assert "UNSUPPORTED" in str(ei.value)
    torch.cuda.synchronize()
