"""Python access to the FP64 CPU oracle (``mls_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use this module to compute reference values.  The GPU
library never imports it, and it imports nothing from the GPU library.

The oracle evaluates moving-least-squares fits (Muelder et al., Sec. 3.3,
Eq. 4-8) by their plain definition -- per position, sequential FP64 sums of the
weighted normal equations in the position-centred basis, equilibrated Cholesky
with a degree ladder -- and extracts marching-squares contours (Sec. 3.4,
contour lines).  See ``mls_oracle.c`` for the exact rules.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mls_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle_mls.so")
# An alternative build of the same source (used by the planted-mistake test,
# which checks that the pins catch a broken oracle).
_LIB_OVERRIDE = os.environ.get("MLS_ORACLE_LIB")

WEIGHT_KINDS = {"gaussian": 0, "wendland": 1, "invpow": 2}
BASIS_DEGREE = {"constant": 0, "linear": 1, "quadratic": 2}
DEG_NAN = 255
DEG_HIT = 254

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, FP64, no FMA contraction)."""
    if _LIB_OVERRIDE or (not force and os.path.exists(_LIB_PATH)):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _LIB_OVERRIDE:
        lib = ctypes.CDLL(_LIB_OVERRIDE)
    else:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.oracle_fit_at.argtypes = [P, P, i64, i32, i32, i32, f64, f64, P, i64,
                                  f64, f64, i32, P, P, P, P]
    lib.oracle_fit_at.restype = ctypes.c_int
    lib.oracle_fit_grid.argtypes = [P, P, i64, i32, i32, i32, f64, f64, f64, f64,
                                    f64, f64, i32, i32, P, i64, f64, f64, i32, P,
                                    P, P, P]
    lib.oracle_fit_grid.restype = ctypes.c_int
    lib.oracle_rigid_grid.argtypes = [P, P, i64, i32, f64, f64, f64, f64, f64, f64, i32, i32,
                                      P, i64, f64, i32, P, P]
    lib.oracle_rigid_grid.restype = ctypes.c_int
    lib.oracle_layout.argtypes = [P, i64, P, P, P, P, f64, f64, f64, f64, f64, i32, i32, P]
    lib.oracle_layout.restype = ctypes.c_int
    lib.oracle_layout_step_nodes.argtypes = [P, i64, P, P, P, P, f64, f64, f64, f64, P, i64,
                                             i32, P]
    lib.oracle_layout_step_nodes.restype = ctypes.c_int
    lib.oracle_map_bands.argtypes = [P, i32, i64, P, i32, P]
    lib.oracle_map_bands.restype = ctypes.c_int
    lib.oracle_map_adaptive.argtypes = [P, P, i32, i64, P, f64, f64, i32, f64, f64, f64, P]
    lib.oracle_map_adaptive.restype = ctypes.c_int
    for name in ("oracle_contour_f64", "oracle_contour_f32"):
        fn = getattr(lib, name)
        fn.argtypes = [P, i32, i32, f64, f64, f64, f64, P, i32, i32, P, P, P, i64]
        fn.restype = ctypes.c_int64
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _prep(points, values):
    pts = np.ascontiguousarray(points, dtype=np.float32)
    vals = np.ascontiguousarray(values, dtype=np.float32)
    if vals.ndim == 1:
        vals = vals[:, None]
    assert pts.ndim == 2 and pts.shape[1] == 2 and vals.shape[0] == pts.shape[0]
    return pts, vals


def fit_at(points, values, positions, basis="linear", weight="gaussian", h=0.05,
           alpha=1.0, tau=1e-8, weight_floor=1e-6, threads=0, grads=False):
    """MLS values at arbitrary positions.

    ``points`` (N, 2) and ``values`` (N, D) are rounded to float32 first (the
    oracle sees exactly the arrays a GPU caller would hand over); positions
    (P, 2) stay float64.  Returns ``(fields (D, P) float64, degree (P,) uint8,
    dmin (P,) float64)``, plus the gradients (D, 2, P) with ``grads=True``.
    """
    pts, vals = _prep(points, values)
    pos = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1, 2)
    n, D = vals.shape
    P = pos.shape[0]
    fields = np.empty((D, P), np.float64)
    deg = np.empty(P, np.uint8)
    dmin = np.empty(P, np.float64)
    g = np.empty((D, 2, P), np.float64) if grads else None
    rc = _load().oracle_fit_at(_ptr(pts), _ptr(vals), n, D, BASIS_DEGREE[basis],
                               WEIGHT_KINDS[weight], float(h), float(alpha),
                               _ptr(pos), P, float(tau), float(weight_floor),
                               int(threads), _ptr(fields), _ptr(deg), _ptr(dmin), _ptr(g))
    if rc != 0:
        raise ValueError("oracle_fit_at rejected its arguments")
    return (fields, deg, dmin, g) if grads else (fields, deg, dmin)


def fit_grid(points, values, grid, basis="linear", weight="gaussian", h=0.05,
             alpha=1.0, tau=1e-8, weight_floor=1e-6, pixels=None, threads=0, grads=False):
    """MLS values at grid nodes.

    ``grid`` is a dict with x0, y0, dx, dy, width, height; node (r, c) sits at
    (x0 + c*dx, y0 + r*dy).  ``pixels`` is an optional array of linear node
    indices r*W + c.  Returns ``(fields, degree, dmin)`` shaped (D, H, W) /
    (H, W) for the whole grid, or (D, P) / (P,) for a pixel list.  With
    ``grads=True`` a fourth result holds the gradients of the local fits,
    (D, 2, H, W) or (D, 2, P).
    """
    pts, vals = _prep(points, values)
    n, D = vals.shape
    W, H = int(grid["width"]), int(grid["height"])
    if pixels is None:
        pix, P = None, W * H
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        P = pix.shape[0]
    fields = np.empty((D, P), np.float64)
    deg = np.empty(P, np.uint8)
    dmin = np.empty(P, np.float64)
    g = np.empty((D, 2, P), np.float64) if grads else None
    rc = _load().oracle_fit_grid(_ptr(pts), _ptr(vals), n, D, BASIS_DEGREE[basis],
                                 WEIGHT_KINDS[weight], float(h), float(alpha),
                                 float(grid["x0"]), float(grid["y0"]),
                                 float(grid["dx"]), float(grid["dy"]), W, H,
                                 _ptr(pix), P, float(tau), float(weight_floor),
                                 int(threads), _ptr(fields), _ptr(deg), _ptr(dmin),
                                 _ptr(g))
    if rc != 0:
        raise ValueError("oracle_fit_grid rejected its arguments")
    if pixels is None:
        out = (fields.reshape(D, H, W), deg.reshape(H, W), dmin.reshape(H, W))
        return out + (g.reshape(D, 2, H, W),) if grads else out
    return (fields, deg, dmin, g) if grads else (fields, deg, dmin)


def rigid_grid(points, values, grid, weight="invpow", h=0.05, alpha=1.0,
               weight_floor=1e-6, pixels=None, threads=0):
    """Rigid MLS (Eq. 9-10) of 2-vector values (N, 2) at grid nodes.
    Returns ``(fields (2, H, W), degree (H, W))`` (or (2, P) / (P,) for a
    pixel list); degree is 1, 254 at exact hits, 255 where undetermined."""
    pts, vals = _prep(points, values)
    n, D = vals.shape
    assert D == 2
    W, H = int(grid["width"]), int(grid["height"])
    if pixels is None:
        pix, P = None, W * H
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        P = pix.shape[0]
    fields = np.empty((2, P), np.float64)
    deg = np.empty(P, np.uint8)
    rc = _load().oracle_rigid_grid(_ptr(pts), _ptr(vals), n, WEIGHT_KINDS[weight], float(h),
                                   float(alpha), float(grid["x0"]), float(grid["y0"]),
                                   float(grid["dx"]), float(grid["dy"]), W, H, _ptr(pix), P,
                                   float(weight_floor), int(threads), _ptr(fields), _ptr(deg))
    if rc != 0:
        raise ValueError("oracle_rigid_grid rejected its arguments")
    if pixels is None:
        return fields.reshape(2, H, W), deg.reshape(H, W)
    return fields, deg


def layout(pos, mesh, C, D, eta, t0, lam, iterations, threads=0):
    """Planarity-preserving layout iterations (Sec. 3.2, Eq. 1-3) from
    positions (n, 2) on a mesh given as a dict of int32 arrays adj_start,
    adj, fan_start, fan (see mesh_arrays).  Returns the positions (n, 2)
    after `iterations` iterations, float64."""
    x = np.ascontiguousarray(pos, dtype=np.float64)
    n = x.shape[0]
    arrs = [np.ascontiguousarray(mesh[k], dtype=np.int32)
            for k in ("adj_start", "adj", "fan_start", "fan")]
    out = np.empty_like(x)
    rc = _load().oracle_layout(_ptr(x), n, *[_ptr(a) for a in arrs], float(C), float(D),
                               float(eta), float(t0), float(lam), int(iterations), int(threads),
                               _ptr(out))
    if rc != 0:
        raise ValueError("oracle_layout rejected its arguments")
    return out


def layout_step_nodes(pos, mesh, C, D, eta, t, nodes, threads=0):
    """One layout iteration at temperature t (Sec. 3.2) for the listed nodes
    only: their positions (m, 2) after it, float64; the move is the one
    `layout` makes in its first iteration."""
    x = np.ascontiguousarray(pos, dtype=np.float64)
    n = x.shape[0]
    arrs = [np.ascontiguousarray(mesh[k], dtype=np.int32)
            for k in ("adj_start", "adj", "fan_start", "fan")]
    idx = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.empty((idx.size, 2), dtype=np.float64)
    rc = _load().oracle_layout_step_nodes(_ptr(x), n, *[_ptr(a) for a in arrs], float(C),
                                          float(D), float(eta), float(t), _ptr(idx), idx.size,
                                          int(threads), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_layout_step_nodes rejected its arguments")
    return out


def contour(fields, grid, iso, f32=False):
    """Marching-squares contours of fields (D, H, W) at isovalues iso (D, n_iso).

    Returns ``(cases (D, n_iso, H-1, W-1) uint8, segments (S, 4) float64,
    ids (S, 3) int32)`` in (field, iso, cell, k) order.  With ``f32=True``
    the fields and isovalues are taken as binary32 and every step of the case
    and crossing arithmetic is rounded to binary32.
    """
    dt = np.float32 if f32 else np.float64
    F = np.ascontiguousarray(fields, dtype=dt)
    if F.ndim == 2:
        F = F[None]
    D, H, W = F.shape
    iso = np.ascontiguousarray(iso, dtype=dt).reshape(D, -1)
    n_iso = iso.shape[1]
    fn = _load().oracle_contour_f32 if f32 else _load().oracle_contour_f64
    cases = np.empty((D, n_iso, H - 1, W - 1), np.uint8)
    segs_all, ids_all = [], []
    g = [float(grid[k]) for k in ("x0", "y0", "dx", "dy")]
    for d in range(D):
        fd = np.ascontiguousarray(F[d])
        isd = np.ascontiguousarray(iso[d])
        cnt = fn(_ptr(fd), H, W, *g, _ptr(isd), n_iso, d, _ptr(cases[d]), None,
                 None, 0)
        if cnt < 0:
            raise ValueError("oracle contour rejected its arguments")
        segs = np.empty((max(cnt, 1), 4), np.float64)
        ids = np.empty((max(cnt, 1), 3), np.int32)
        cnt2 = fn(_ptr(fd), H, W, *g, _ptr(isd), n_iso, d, None, _ptr(segs),
                  _ptr(ids), cnt)
        assert cnt2 == cnt
        segs_all.append(segs[:cnt])
        ids_all.append(ids[:cnt])
    return cases, np.concatenate(segs_all), np.concatenate(ids_all)


def map_bands(fields, iso):
    """Discrete-colour bands (Sec. 3.4, Fig. 5b) of float32 fields (D, ...)
    at isovalues (D, n_iso): per value the number of isovalues at or below
    it, 255 for NaN.  Returns uint8 of the fields' shape."""
    f = np.ascontiguousarray(fields, dtype=np.float32)
    D = f.shape[0]
    lv = np.ascontiguousarray(np.asarray(iso, dtype=np.float32).reshape(D, -1))
    out = np.empty(f.shape, np.uint8)
    P = f.size // D
    rc = _load().oracle_map_bands(_ptr(f), D, P, _ptr(lv), lv.shape[1], _ptr(out))
    if rc != 0:
        raise ValueError("oracle_map_bands rejected its arguments")
    return out


def map_adaptive(fields, grads, levels, grid, n_levels=3, halfwidth=1.0, fade_lo=4.0,
                 fade_hi=12.0):
    """Adaptive contour-line intensity (Sec. 3.4, Fig. 5d) of float32 fields
    (D, H, W) with gradients (D, 2, H, W) and levels (D, 2) = (origin,
    spacing) per field.  Returns float64 (D, H, W)."""
    f = np.ascontiguousarray(fields, dtype=np.float32)
    D = f.shape[0]
    g = np.ascontiguousarray(grads, dtype=np.float32)
    lv = np.ascontiguousarray(np.asarray(levels, dtype=np.float32).reshape(D, 2))
    out = np.empty(f.shape, np.float64)
    P = f.size // D
    rc = _load().oracle_map_adaptive(_ptr(f), _ptr(g), D, P, _ptr(lv), float(grid["dx"]),
                                     float(grid["dy"]), int(n_levels), float(halfwidth),
                                     float(fade_lo), float(fade_hi), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_map_adaptive rejected its arguments")
    return out
