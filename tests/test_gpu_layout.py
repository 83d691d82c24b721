"""GPU parity of the planarity-preserving layout (mls_layout, Sec. 3.2
Eq. 1-3) against the oracle's iteration, and the planarity guarantee on a
long hot run.  Positions are float32 at the boundary (float64 inside); the
bound is 2e-6 of the point cloud's extent after 1 and 25 iterations."""
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


def to_dev(torch, mesh):
    return {k: torch.from_numpy(np.ascontiguousarray(mesh[k])).cuda()
            for k in ("adj_start", "adj", "fan_start", "fan")}


def signed_areas(x, tri):
    a, b, c = x[tri[:, 0]], x[tri[:, 1]], x[tri[:, 2]]
    return (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])


def params_for(pts, mesh):
    src = np.repeat(np.arange(pts.shape[0]), np.diff(mesh["adj_start"]))
    D = float(np.linalg.norm(pts[src] - pts[mesh["adj"]], axis=1).mean())
    return dict(C=D ** 3, D=D, eta=1e-3 * D, t0=0.25 * D, lam=0.99)


@pytest.mark.parametrize("iters", [1, 25])
def test_layout_matches_oracle(torch_dev, oracle, iters):
    from paper_1408_0677_amd import api, workloads as wl
    note(f"case layout parity {iters} iterations")
    rng = np.random.default_rng(iters)
    pts = rng.random((300, 2)).astype(np.float32)
    mesh = wl.mesh_arrays(pts)
    prm = params_for(pts.astype(np.float64), mesh)
    P = torch_dev.from_numpy(pts.copy()).cuda()
    api.layout(P, to_dev(torch_dev, mesh), iterations=iters, **prm)
    torch_dev.cuda.synchronize()
    got = P.cpu().numpy().astype(np.float64)
    ref = oracle.layout(pts.astype(np.float64), mesh, iterations=iters, **prm)
    err = np.abs(got - ref).max()
    note(f"max position error {err:.3e}, moved {np.abs(ref - pts).max():.3e}")
    assert np.abs(ref - pts).max() > 1e-4
    assert err <= 2e-6


def test_layout_keeps_planarity(torch_dev):
    from paper_1408_0677_amd import api, workloads as wl
    note("case layout planarity 2000 points x 300 iterations")
    rng = np.random.default_rng(11)
    pts = rng.random((2000, 2)).astype(np.float32)
    mesh = wl.mesh_arrays(pts)
    prm = params_for(pts.astype(np.float64), mesh)
    prm["t0"] = prm["D"]            # hot start
    P = torch_dev.from_numpy(pts.copy()).cuda()
    api.layout(P, to_dev(torch_dev, mesh), iterations=300, **prm)
    torch_dev.cuda.synchronize()
    out = P.cpu().numpy().astype(np.float64)
    tri = mesh["triangles"]
    s0 = np.sign(signed_areas(pts.astype(np.float64), tri))
    s1 = np.sign(signed_areas(out, tri))
    assert np.all(np.isfinite(out))
    assert np.all(s0 == s1)
    assert np.abs(out - pts).max() > 1e-3


def test_layout_ignores_malformed_lists(torch_dev):
    """Indices outside [0, n) and ranges past the arrays are skipped."""
    import torch
    from paper_1408_0677_amd import api
    note("case layout malformed lists")
    n = 50
    pts = torch.rand(n, 2, device="cuda")
    adj_start = torch.tensor([0] + [3] * (n - 1) + [10_000], dtype=torch.int32, device="cuda")
    adj = torch.tensor([1, -5, 99999], dtype=torch.int32, device="cuda")
    fan_start = torch.tensor([-7] + [1] * n, dtype=torch.int32, device="cuda")
    fan = torch.tensor([[2, 70000]], dtype=torch.int32, device="cuda")
    api.layout(pts, {"adj_start": adj_start, "adj": adj, "fan_start": fan_start, "fan": fan},
               C=1e-3, D=0.1, eta=1e-4, t0=0.01, lam=0.9, iterations=3)
    torch.cuda.synchronize()
    assert torch.isfinite(pts).all()


def test_layout_bench_shape(torch_dev, oracle):
    """The 2245-node timing-table mesh with the bench's parameters: parity
    after 10 iterations, and no flipped triangle after the bench's 1000."""
    from paper_1408_0677_amd import api, workloads as wl
    note("case layout 2245 nodes, bench parameters")
    pts, mesh, prm = wl.layout_workload(2245)
    p32 = pts.astype(np.float32)
    M = to_dev(torch_dev, mesh)
    P = torch_dev.from_numpy(p32.copy()).cuda()
    api.layout(P, M, iterations=10, **prm)
    torch_dev.cuda.synchronize()
    ref = oracle.layout(p32.astype(np.float64), mesh, iterations=10, **prm)
    err = np.abs(P.cpu().numpy().astype(np.float64) - ref).max() / 600.0
    note(f"10 iterations: max position error {err:.3e} of the canvas")
    assert err <= 2e-6
    P = torch_dev.from_numpy(p32.copy()).cuda()
    api.layout(P, M, iterations=1000, **prm)
    torch_dev.cuda.synchronize()
    out = P.cpu().numpy().astype(np.float64)
    tri = mesh["triangles"]
    assert np.all(np.isfinite(out))
    assert np.all(np.sign(signed_areas(p32.astype(np.float64), tri)) ==
                  np.sign(signed_areas(out, tri)))


@pytest.mark.parametrize("n", [65536, 300000])
def test_layout_large_meshes_sampled(torch_dev, oracle, n):
    """Meshes large enough for the 16- and 64-node workgroup layouts: one
    iteration, checked against the oracle on a sample of nodes."""
    from paper_1408_0677_amd import api, workloads as wl
    note(f"case layout {n} nodes, sampled")
    rng = np.random.default_rng(n)
    p32 = (rng.random((n, 2)) * 600.0).astype(np.float32)
    mesh = wl.mesh_arrays(p32.astype(np.float64))
    prm = params_for(p32.astype(np.float64), mesh)
    P = torch_dev.from_numpy(p32.copy()).cuda()
    api.layout(P, to_dev(torch_dev, mesh), iterations=1, **prm)
    torch_dev.cuda.synchronize()
    got = P.cpu().numpy().astype(np.float64)
    nodes = np.unique(np.concatenate([[0, n - 1], rng.integers(0, n, 1000)]))
    ref = oracle.layout_step_nodes(p32.astype(np.float64), mesh, C=prm["C"], D=prm["D"],
                                   eta=prm["eta"], t=prm["t0"], nodes=nodes)
    err = np.abs(got[nodes] - ref).max() / 600.0
    moved = np.abs(ref - p32[nodes]).max()
    note(f"max position error {err:.3e} of the canvas over {nodes.size} nodes, moved {moved:.3e}")
    assert moved > 1e-3
    assert err <= 2e-6


def test_layout_binding_checks_mesh_arrays(torch_dev):
    """Mesh arrays of the wrong type, place or length are refused by the
    binding instead of being read as something else."""
    import torch
    from paper_1408_0677_amd import api, workloads as wl
    note("case layout binding checks")
    rng = np.random.default_rng(2)
    pts = rng.random((40, 2)).astype(np.float32)
    mesh = to_dev(torch, wl.mesh_arrays(pts))
    P = torch.from_numpy(pts).cuda()
    prm = dict(C=1e-3, D=0.1, eta=1e-4, t0=0.01, lam=0.9, iterations=1)
    bad = dict(mesh, adj=mesh["adj"].long())
    with pytest.raises(ValueError, match="int32"):
        api.layout(P, bad, **prm)
    bad = dict(mesh, fan=mesh["fan"].cpu())
    with pytest.raises(ValueError, match="int32"):
        api.layout(P, bad, **prm)
    bad = dict(mesh, adj_start=mesh["adj_start"][:-1].contiguous())
    with pytest.raises(ValueError, match="n \\+ 1"):
        api.layout(P, bad, **prm)
    api.layout(P, mesh, **prm)
    torch.cuda.synchronize()
    assert torch.isfinite(P).all()
