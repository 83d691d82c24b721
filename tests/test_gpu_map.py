"""GPU parity of the space mappings (Sec. 3.4, Fig. 5b, 5d) against the
oracle on the same float32 fields: bands and colours bit for bit, adaptive
line intensities within 1e-6 (both sides in float64 per node; the output
is float32)."""
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


def fitted(torch, w, grid=None, basis="linear", h=None):
    from paper_1408_0677_amd import api
    P = torch.from_numpy(w.points).cuda()
    V = torch.from_numpy(w.values).cuda()
    return api.fit_grad(P, V, grid or w.grid, basis=basis, h=h or w.h)


@pytest.mark.parametrize("side", [(37, 29), (256, 256), (1024, 1024)])
def test_bands_and_colours(torch_dev, oracle, side):
    import torch
    from paper_1408_0677_amd import api, workloads as wl
    W, H = side
    note(f"case map bands {W}x{H}")
    w = wl.c2(grid_side=W, n=3000)
    grid = wl.pixel_grid(W, H)
    F, _, _ = fitted(torch, w, grid=grid)
    F[0, 3, 4] = float("nan")
    iso = torch.from_numpy(w.iso()).cuda()
    n_iso = iso.shape[1]
    rng = np.random.default_rng(1)
    cmap = torch.from_numpy(rng.integers(-2**31, 2**31 - 1, (w.d, n_iso + 1), dtype=np.int64)
                            .astype(np.int32)).cuda()
    bands, rgba = api.map_bands(F, grid, iso, colormap=cmap)
    torch.cuda.synchronize()
    ob = oracle.map_bands(F.cpu().numpy(), w.iso())
    gb = bands.cpu().numpy()
    assert np.array_equal(gb, ob)
    cm = cmap.cpu().numpy()
    expect = np.where(ob == 255, 0, np.take_along_axis(
        cm, np.where(ob == 255, 0, ob).reshape(w.d, -1).astype(np.int64), axis=1).reshape(ob.shape))
    assert np.array_equal(rgba.cpu().numpy(), expect)
    # bands only, no colours
    b2, r2 = api.map_bands(F, grid, iso)
    assert r2 is None and torch.equal(b2, bands)


@pytest.mark.parametrize("side,basis", [((37, 29), "linear"), ((256, 256), "quadratic"),
                                        ((1024, 1024), "linear")])
def test_adaptive_lines(torch_dev, oracle, side, basis):
    import torch
    from paper_1408_0677_amd import api, workloads as wl
    W, H = side
    note(f"case map adaptive {W}x{H} {basis}")
    w = wl.c2(grid_side=W, n=3000)
    grid = wl.pixel_grid(W, H)
    F, G, _ = fitted(torch, w, grid=grid, basis=basis, h=0.06)
    G[1, :, 5, 6] = 0.0
    lo, hi = w.values.min(0), w.values.max(0)
    levels = np.stack([lo, (hi - lo) / 11.0], axis=1).astype(np.float32)
    L = torch.from_numpy(levels).cuda()
    kw = dict(n_levels=4, halfwidth=1.0, fade_lo=4.0, fade_hi=12.0)
    I = api.map_adaptive(F, G, grid, L, **kw)
    torch.cuda.synchronize()
    oi = oracle.map_adaptive(F.cpu().numpy(), G.cpu().numpy(), levels, grid, **kw)
    gi = I.cpu().numpy().astype(np.float64)
    assert np.array_equal(np.isnan(gi), np.isnan(oi))
    ok = ~np.isnan(oi)
    err = np.abs(gi[ok] - oi[ok]).max()
    note(f"max |intensity - oracle| = {err:.2e}; mean intensity {oi[ok].mean():.3f}")
    assert err <= 1e-6
    assert gi[1, 5, 6] == 0.0


def test_map_arguments_rejected(torch_dev):
    import ctypes
    import torch
    from paper_1408_0677_amd import _lib, api
    lib = _lib.load()
    ctx = api.default_context(0)
    F = torch.zeros((1, 8, 8), device="cuda")
    g = _lib.MlsGrid(0.0, 0.0, 0.1, 0.1, 8, 8)
    iso = torch.zeros((1, 2), device="cuda")
    st = lib.mls_map_bands(ctx.handle, ctypes.c_void_p(F.data_ptr()), 1, ctypes.byref(g),
                           ctypes.c_void_p(iso.data_ptr()), 255, None,
                           ctypes.c_void_p(F.data_ptr()), None, None)
    assert st == -1 and b"n_iso" in lib.mls_last_error()
    prm = _lib.MlsAdaptiveParams(0, 1.0, 1.0, 2.0)
    st = lib.mls_map_adaptive(ctx.handle, ctypes.c_void_p(F.data_ptr()),
                              ctypes.c_void_p(F.data_ptr()), 1, ctypes.byref(g),
                              ctypes.c_void_p(F.data_ptr()), ctypes.byref(prm),
                              ctypes.c_void_p(F.data_ptr()), None)
    assert st == -1 and b"levels" in lib.mls_last_error()
