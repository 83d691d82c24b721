"""The allocation-free contour entry point (mls_contour_static) against
mls_contour, through the C ABI: two calls in a row on one device, the second
on a smaller input, each bit for bit equal to mls_contour's segments, ids,
cases and count; a short buffer still receives the first segments; a call
whose scratch would exceed the fixed array is refused before any work."""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def fields_for(torch, w, D):
    from paper_1408_0677_amd import api
    P = torch.from_numpy(w.points).cuda()
    V = torch.from_numpy(np.ascontiguousarray(w.values[:, :D])).cuda()
    F, _ = api.fit(P, V, w.grid, basis=w.basis, h=w.h)
    iso = torch.from_numpy(np.ascontiguousarray(w.iso()[:D])).cuda()
    return F, iso


def static_call(torch, lib, ctx, F, grid, iso, cap, with_cases=True):
    from paper_1408_0677_amd import _lib
    D, H, W = F.shape
    n_iso = iso.shape[1]
    segs = torch.full((max(cap, 1), 4), -1.0, device="cuda")
    ids = torch.full((max(cap, 1), 3), -1, dtype=torch.int32, device="cuda")
    cases = (torch.zeros((D, n_iso, H - 1, W - 1), dtype=torch.uint8, device="cuda")
             if with_cases else None)
    count = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    g = _lib.MlsGrid(grid["x0"], grid["y0"], grid["dx"], grid["dy"], W, H)
    stream = torch.cuda.current_stream().cuda_stream
    st = lib.mls_contour_static(ctx.handle, ctypes.c_void_p(F.data_ptr()), D, ctypes.byref(g),
                                ctypes.c_void_p(iso.data_ptr()), n_iso,
                                ctypes.c_void_p(cases.data_ptr()) if with_cases else None,
                                ctypes.c_void_p(segs.data_ptr()) if cap else None,
                                ctypes.c_void_p(ids.data_ptr()) if cap else None, cap,
                                ctypes.c_void_p(count.data_ptr()), ctypes.c_void_p(stream))
    return st, segs, ids, cases, count


def test_static_contour_equals_contour():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1408_0677_amd import _lib, api, workloads as wl
    lib = _lib.load()
    ctx = api.Context(0)
    big = wl.c2(grid_side=512, n=3000)
    small = wl.c1()
    for label, w, D in (("512^2 x 13 fields", big, 13), ("128^2 x 4 fields", small, 4)):
        note(f"case contour_static {label}")
        F, iso = fields_for(torch, w, D)
        ref_segs, ref_ids, ref_cases = api.contour(F, w.grid, iso, ctx=ctx)
        torch.cuda.synchronize()
        n = ref_segs.shape[0]
        cap = n + 100
        st, segs, ids, cases, count = static_call(torch, lib, ctx, F, w.grid, iso, cap)
        assert st == 0, lib.mls_last_error()
        torch.cuda.synchronize()
        assert int(count.item()) == n
        assert torch.equal(segs[:n].view(torch.int32), ref_segs.view(torch.int32))
        assert torch.equal(ids[:n], ref_ids)
        assert torch.equal(cases, ref_cases)
        assert bool((segs[n:] == -1.0).all()) and bool((ids[n:] == -1).all())
        # a short buffer: the count is still the full one, the first segments
        # are written in order, nothing past the buffer
        short = n // 3
        st, segs2, ids2, _, count2 = static_call(torch, lib, ctx, F, w.grid, iso, short,
                                                 with_cases=False)
        assert st == 0
        torch.cuda.synchronize()
        assert int(count2.item()) == n
        assert torch.equal(segs2[:short].view(torch.int32), ref_segs[:short].view(torch.int32))
        assert torch.equal(ids2[:short], ref_ids[:short])
    # more fields x isovalues than the fixed scratch holds: refused up front
    F = torch.zeros((64, 2048, 2048), device="cuda")
    iso = torch.zeros((64, 16), device="cuda")
    grid = wl.pixel_grid(2048)
    st, segs, _, _, count = static_call(torch, lib, ctx, F, grid, iso, 16, with_cases=False)
    assert st == -1 and b"static scratch holds" in lib.mls_last_error()
    torch.cuda.synchronize()
    assert int(count.item()) == -1
    ctx.close()
