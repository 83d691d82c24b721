"""The C ABI library loads, exports every symbol include/mls.h declares, and
rejects bad arguments before touching the device (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mls.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mls_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1408_0677_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1408_0677_amd import build
        build.build()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert {"mls_fit", "mls_context_create", "mls_context_destroy"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    from paper_1408_0677_amd import _lib
    assert set(_lib.EXPORTS) == set(names)


def test_status_strings(lib):
    assert lib.mls_status_string(0) == b"MLS_OK"
    assert lib.mls_status_string(-1) == b"MLS_ERR_INVALID_ARG"
    assert lib.mls_status_string(-3) == b"MLS_ERR_CAPACITY"
    assert lib.mls_status_string(12345) == b"MLS_UNKNOWN_STATUS"


def _fit(lib, n=10, d=2, basis=1, kind=0, h=0.1, alpha=1.0, grid=(0.0, 0.0, 0.1, 0.1, 8, 8),
         precision=0, opts=None, pts=1, vals=1, fields=1, ctx=None):
    from paper_1408_0677_amd import _lib
    w = _lib.MlsWeight(kind, h, alpha)
    g = _lib.MlsGrid(*grid)
    o = None if opts is None else ctypes.byref(_lib.MlsSolveOpts(*opts))
    fake = ctypes.c_void_p(0x1000)
    return lib.mls_fit(ctx, fake if pts else None, fake if vals else None, n, d, basis,
                       ctypes.byref(w), ctypes.byref(g), precision, o,
                       fake if fields else None, None, None)


@pytest.mark.parametrize("kwargs,needle", [
    (dict(n=0), b"n = 0"),
    (dict(d=0), b"d = 0"),
    (dict(d=84), b"d = 84"),
    (dict(basis=2, d=41), b"d = 41"),
    (dict(basis=4), b"basis 4"),
    (dict(basis=3, d=3), b"2-vector values"),
    (dict(kind=7), b"weight kind 7"),
    (dict(h=0.0), b"h = 0"),
    (dict(h=float("nan")), b"h = nan"),
    (dict(h=float("inf")), b"h = inf"),
    (dict(kind=2, alpha=-1.0), b"alpha"),
    (dict(grid=(0.0, 0.0, 0.1, 0.1, 0, 8)), b"need width"),
    (dict(grid=(float("nan"), 0.0, 0.1, 0.1, 8, 8)), b"finite"),
    (dict(precision=9), b"precision 9"),
    (dict(precision=1, d=1025), b"d = 1025"),
    (dict(opts=(0.0, 1e-6, 0)), b"pivot_tol"),
    (dict(opts=(1e-8, -1.0, 0)), b"weight_floor"),
    (dict(opts=(1e-8, 1e-6, 4)), b"lp_terms"),
    (dict(opts=(1e-8, 1e-6, 0, -1)), b"lp_slab"),
    (dict(basis=2, opts=(1e-8, 1e-6, 0, 19)), b"lp_slab"),
    (dict(basis=1, opts=(1e-8, 1e-6, 0, 41)), b"lp_slab"),
    (dict(pts=0), b"d_points is NULL"),
    (dict(vals=0), b"d_values is NULL"),
    (dict(fields=0), b"d_fields is NULL"),
    (dict(), b"ctx is NULL"),
])
def test_invalid_arguments_rejected_before_device(lib, kwargs, needle):
    st = _fit(lib, **kwargs)
    assert st == -1, (st, lib.mls_last_error())
    assert needle in lib.mls_last_error(), lib.mls_last_error()


def test_context_create_rejects_null_out(lib):
    assert lib.mls_context_create(0, None) == -1


def _contour(lib, d=1, grid=(0.0, 0.0, 0.1, 0.1, 8, 8), n_iso=2, capacity=10, fields=1,
             iso=1, segs=1, count=True, ctx=None, seg_addr=0x1000):
    from paper_1408_0677_amd import _lib
    g = _lib.MlsGrid(*grid)
    fake = ctypes.c_void_p(0x1000)
    cnt = ctypes.c_int64(-7)
    st = lib.mls_contour(ctx, fake if fields else None, d, ctypes.byref(g),
                         fake if iso else None, n_iso, None,
                         ctypes.c_void_p(seg_addr) if segs else None, None, capacity,
                         ctypes.byref(cnt) if count else None, None)
    return st, cnt.value


@pytest.mark.parametrize("kwargs,needle", [
    (dict(d=0), b"d = 0"),
    (dict(grid=(0.0, 0.0, 0.1, 0.1, 1, 8)), b"width, height >= 2"),
    (dict(grid=(0.0, float("inf"), 0.1, 0.1, 8, 8)), b"finite"),
    (dict(n_iso=0), b"n_iso = 0"),
    (dict(capacity=-1), b"capacity"),
    (dict(count=False), b"h_count is NULL"),
    (dict(fields=0), b"d_fields is NULL"),
    (dict(iso=0), b"d_iso is NULL"),
    (dict(segs=0), b"d_segments is NULL"),
    (dict(seg_addr=0x1004), b"16-byte aligned"),
    (dict(d=100000, grid=(0.0, 0.0, 1.0, 1.0, 1000, 1000)), b"exceed one launch"),
    (dict(), b"ctx is NULL"),
])
def test_contour_invalid_arguments(lib, kwargs, needle):
    st, cnt = _contour(lib, **kwargs)
    assert st == -1, (st, lib.mls_last_error())
    assert needle in lib.mls_last_error(), lib.mls_last_error()
    assert cnt == -7          # nothing written on rejection


def test_fit_scratch_plan(lib):
    """Host-only scratch plan: the Gaussian factor tables for float64 (up to
    the cap, none beyond it), staging for 16-bit paths, more with the cell
    list."""
    from paper_1408_0677_amd import api
    grid = {"x0": 0.0, "y0": 0.0, "dx": 0.01, "dy": 0.01, "width": 100, "height": 100}
    # 8 B x 1024 points (1000 padded to 64) x (112 columns + 112 rows)
    assert api.fit_scratch_bytes(1000, 4, grid, "f64") == 8 * 1024 * (112 + 112)
    # past 512 MiB of tables: generated per tile, no scratch
    big = dict(grid, width=4096, height=4096)
    assert api.fit_scratch_bytes(10 ** 6, 4, big, "f64") == 0
    assert api.fit_scratch_bytes(1000, 4, grid, "f64", weight="invpow") > 0
    lp = api.fit_scratch_bytes(1000, 4, grid, "bf16")
    assert lp >= 4 * 1000 * 4
    wd = api.fit_scratch_bytes(1000, 4, grid, "bf16", weight="wendland", h=0.05)
    assert wd > lp + 2 * 4 * 1000 * 4


def test_server_arguments_rejected_without_device(lib):
    from paper_1408_0677_amd import _lib
    out = ctypes.c_void_p()
    assert lib.mls_server_create(0, 1 << 20, 0, 0, ctypes.byref(out)) == -1
    assert b"slots" in lib.mls_server_last_error()
    assert lib.mls_server_create(0, 1 << 20, 4, 1 << 20, ctypes.byref(out)) == -5
    assert b"exceed the budget" in lib.mls_server_last_error()
    assert lib.mls_server_create(0, 1 << 20, 1, 0, None) == -1
    pid = ctypes.c_uint64()
    assert lib.mls_server_put_points(None, None, None, 1, 1, ctypes.byref(pid)) == -1
    req = _lib.MlsRequest()
    t = ctypes.c_uint64()
    assert lib.mls_server_submit(None, ctypes.byref(req), ctypes.byref(t)) == -1
    res = _lib.MlsResult()
    assert lib.mls_server_poll(None, 1, ctypes.byref(res)) == -1
    assert lib.mls_server_tuning(None, 1, None) == -1
    assert lib.mls_server_tuned_classes(None) == 0
    assert lib.mls_server_tuning_pending(None) == 0
    assert lib.mls_server_cancel(None, 1) == -1
    assert lib.mls_status_string(-5) == b"MLS_ERR_OVER_BUDGET"
    assert lib.mls_status_string(-6) == b"MLS_ERR_CANCELLED"
    assert lib.mls_status_string(1) == b"MLS_PENDING"


def _layout(lib, n=10, n_adj=4, n_fan=2, prm=(1.0, 0.1, 1e-4, 0.01, 0.99), iters=5,
            pos=1, starts=1, arrays=1, ctx=None):
    from paper_1408_0677_amd import _lib
    fake = ctypes.c_void_p(0x1000)
    p = None if prm is None else ctypes.byref(_lib.MlsLayoutParams(*prm))
    return lib.mls_layout(ctx, fake if pos else None, n, fake if starts else None,
                          fake if arrays else None, n_adj, fake if starts else None,
                          fake if arrays else None, n_fan, p, iters, None)


@pytest.mark.parametrize("kwargs,needle", [
    (dict(n=0), b"n = 0"),
    (dict(n_adj=-1), b"n_adj"),
    (dict(iters=-2), b"iterations"),
    (dict(prm=None), b"params is NULL"),
    (dict(prm=(1.0, 0.1, 0.0, 0.01, 0.99)), b"layout parameters"),
    (dict(prm=(1.0, 0.1, 1e-4, 0.01, 1.5)), b"layout parameters"),
    (dict(prm=(1.0, -0.1, 1e-4, 0.01, 0.9)), b"layout parameters"),
    (dict(pos=0), b"required device array"),
    (dict(arrays=0), b"required device array"),
    (dict(), b"ctx is NULL"),
])
def test_layout_arguments_rejected_before_device(lib, kwargs, needle):
    assert _layout(lib, **kwargs) == -1
    assert needle in lib.mls_last_error(), lib.mls_last_error()


def test_layout_binding_rejects_host_and_mistyped_arrays():
    """The binding refuses host tensors and mesh arrays of the wrong type or
    length before anything reaches the library."""
    import torch
    from paper_1408_0677_amd import api
    mesh = {"adj_start": torch.zeros(4, dtype=torch.int32), "adj": torch.zeros(0, dtype=torch.int32),
            "fan_start": torch.zeros(4, dtype=torch.int32), "fan": torch.zeros(0, dtype=torch.int32)}
    with pytest.raises(ValueError, match="device tensor"):
        api.layout(torch.zeros(3, 2), mesh, C=1.0, D=1.0, eta=1e-3, t0=0.1, lam=0.9,
                   iterations=1)
    with pytest.raises(ValueError, match="device tensor"):
        api.layout(torch.zeros(3, 2, dtype=torch.float64), mesh, C=1.0, D=1.0, eta=1e-3,
                   t0=0.1, lam=0.9, iterations=1)


def test_fit_binding_rejects_host_and_mistyped_tensors():
    """The fit binding refuses host tensors, other dtypes, mis-shaped points
    and points/values of different lengths before anything reaches the
    library (a wrong buffer would be read or written past its end)."""
    import torch
    from paper_1408_0677_amd import api
    grid = {"x0": 0.0, "y0": 0.0, "dx": 0.1, "dy": 0.1, "width": 8, "height": 8}
    with pytest.raises(ValueError, match="device tensor"):
        api.fit(torch.zeros(10, 2), torch.zeros(10, 3), grid)
    with pytest.raises(ValueError, match="device tensor"):
        api.fit_grad(torch.zeros(10, 2), torch.zeros(10, 3), grid)
    with pytest.raises(ValueError, match="device tensor"):
        api.contour(torch.zeros(1, 8, 8), grid, torch.zeros(1, 1))


def test_contour_static_arguments_rejected_before_device(lib):
    """The allocation-free contour shares mls_contour's checks; it names its
    device count output."""
    from paper_1408_0677_amd import _lib
    g = _lib.MlsGrid(0.0, 0.0, 0.1, 0.1, 8, 8)
    fake = ctypes.c_void_p(0x1000)
    st = lib.mls_contour_static(None, fake, 1, ctypes.byref(g), fake, 2, None, fake, None, 10,
                                None, None)
    assert st == -1 and b"d_count is NULL" in lib.mls_last_error()
    st = lib.mls_contour_static(None, fake, 1, ctypes.byref(g), fake, 0, None, fake, None, 10,
                                fake, None)
    assert st == -1 and b"n_iso = 0" in lib.mls_last_error()
    st = lib.mls_contour_static(None, fake, 1, ctypes.byref(g), fake, 2, None, fake, None, 10,
                                fake, None)
    assert st == -1 and b"ctx is NULL" in lib.mls_last_error()


def test_trace_arguments_rejected(lib):
    from paper_1408_0677_amd import _lib
    assert lib.mls_context_trace(None, 1, None) == -1
    rec = _lib.MlsTraceRecord()
    assert lib.mls_context_trace_last(None, ctypes.byref(rec)) == -1


def test_map_arguments_rejected_before_device(lib):
    from paper_1408_0677_amd import _lib
    g = _lib.MlsGrid(0.0, 0.0, 0.1, 0.1, 8, 8)
    fake = ctypes.c_void_p(0x1000)
    assert lib.mls_map_bands(None, fake, 1, ctypes.byref(g), fake, 0, None, fake, None,
                             None) == -1
    assert b"n_iso" in lib.mls_last_error()
    assert lib.mls_map_bands(None, fake, 1, ctypes.byref(g), fake, 3, None, None, None,
                             None) == -1
    assert b"both NULL" in lib.mls_last_error()
    assert lib.mls_map_bands(None, fake, 1, ctypes.byref(g), fake, 3, None, None, fake,
                             None) == -1
    assert b"colormap" in lib.mls_last_error()
    prm = _lib.MlsAdaptiveParams(3, 1.0, 5.0, 5.0)
    assert lib.mls_map_adaptive(None, fake, fake, 1, ctypes.byref(g), fake, ctypes.byref(prm),
                                fake, None) == -1
    assert b"fade_lo" in lib.mls_last_error()
    prm = _lib.MlsAdaptiveParams(3, 1.0, 4.0, 12.0)
    assert lib.mls_map_adaptive(None, fake, fake, 1, ctypes.byref(g), fake, ctypes.byref(prm),
                                fake, None) == -1
    assert b"ctx is NULL" in lib.mls_last_error()


# binding field names that differ from the header's (Python keywords)
RENAMED = {"lam": "lambda"}


def test_struct_layouts_match_header(tmp_path):
    """Every struct the binding declares has the header's size and field
    offsets (a C program built with gcc from include/mls.h prints them)."""
    import os
    import shutil
    import subprocess
    from paper_1408_0677_amd import _lib
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    pairs = {"mls_grid": _lib.MlsGrid, "mls_weight": _lib.MlsWeight,
             "mls_solve_opts": _lib.MlsSolveOpts, "mls_layout_params": _lib.MlsLayoutParams,
             "mls_adaptive_params": _lib.MlsAdaptiveParams, "mls_request": _lib.MlsRequest,
             "mls_result": _lib.MlsResult, "mls_trace_record": _lib.MlsTraceRecord}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "mls.h"', "int main(void) {"]
    for cname, cls in pairs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            field = RENAMED.get(fname, fname)
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(__file__), "..", "include")
    subprocess.run(["gcc", "-std=c99", "-I", inc, str(src), "-o", str(exe)], check=True)
    got = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    expect = []
    for cname, cls in pairs.items():
        expect.append(f"{cname} size {ctypes.sizeof(cls)}")
        for fname, _ in cls._fields_:
            expect.append(f"{cname} {fname} {getattr(cls, fname).offset}")
    assert [g for g in got if g] == expect
