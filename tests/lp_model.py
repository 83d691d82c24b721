"""A numpy model of the arithmetic of the 16-bit contraction paths (test
infrastructure, CPU only).

It follows the rounding steps the 16-bit fit takes, not its code: tile
frames anchored at the centre of 16 x 16 node tiles, attributes mapped to
[-1, 1], float32 tile-frame coordinates, separable float32 Gaussian
factors multiplied into a float32 weight, features carried as S bfloat16
terms, the weight as a hi + lo pair of bfloat16 numbers, products summed
into float32 accumulators once per 32-point step and matrix instruction.
Each ingredient can be switched to exact (float64) arithmetic, so that the
error of the full model can be split among its sources.  The normal
equations are solved in float64 in the tile frame and evaluated at the
node's offset, which is the same polynomial as the node-frame fit.

Nothing here comes from, or feeds, the HIP library: the model reads the
seeded workload and is compared with the oracle.
"""
from __future__ import annotations

import numpy as np

# monomials u_x^a u_y^b of degree <= 4, in the order the moments are kept;
# the quadratic basis is the first six
EXPONENTS = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1), (1, 2), (0, 3),
             (4, 0), (3, 1), (2, 2), (1, 3), (0, 4)]
MONO = {e: i for i, e in enumerate(EXPONENTS)}
BASIS = EXPONENTS[:6]
KSTEP = 32      # points per matrix instruction (16 x 16 x 32)


def bf16(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float32."""
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def fit_tiles(points, values, grid, h, tiles, terms=3, features="bf16", weight="split",
              accumulate="f32", rhs_terms=None):
    """Quadratic-basis Gaussian MLS fields on the nodes of the given 16 x 16
    tiles, under the chosen arithmetic:

    features    "bf16" (S = terms bfloat16 terms of float32 features),
                "f32" (float32 features), "f64" (exact features)
    weight      "split" (hi + lo, lo times every term but the last),
                "lo1" (hi + lo, lo times the first term only),
                "hi" (the bfloat16 rounding of the weight alone, every term),
                "exact" (the float32 weight, or float64 with features="f64")
    accumulate  "f32" (one float32 rounding per step and product) or "f64"
    rhs_terms   with features="bf16": the basis x attribute columns keep only
                their first rhs_terms terms (default: all `terms`)

    Returns fields (D, H, W), NaN outside the tiles.
    """
    pts = np.asarray(points, np.float32)
    vals = np.asarray(values, np.float32)
    n, D = vals.shape
    W, H = int(grid["width"]), int(grid["height"])
    x0, y0, dx, dy = (float(grid[k]) for k in ("x0", "y0", "dx", "dy"))
    lo = vals.min(0).astype(np.float64)
    hi = vals.max(0).astype(np.float64)
    shift = (0.5 * (lo + hi)).astype(np.float32)
    scale = (0.5 * (hi - lo)).astype(np.float32)
    staged = ((vals.astype(np.float64) - shift) / scale).astype(np.float32)
    inv_hd = 1.0 / h
    inv_h = np.float32(inv_hd)
    tiles_x = (W + 15) // 16
    out = np.full((D, H, W), np.nan)
    for t in tiles:
        c0, r0 = (t % tiles_x) * 16, (t // tiles_x) * 16
        ax = np.float32(x0 + (c0 + 8) * dx)
        ay = np.float32(y0 + (r0 + 8) * dy)
        col_off = (x0 + (c0 + np.arange(16)) * dx - float(ax)) * inv_hd
        row_off = (y0 + (r0 + np.arange(16)) * dy - float(ay)) * inv_hd
        if features == "f64":
            ux = (pts[:, 0].astype(np.float64) - float(ax)) * inv_hd
            uy = (pts[:, 1].astype(np.float64) - float(ay)) * inv_hd
            gx = np.exp(-(ux[None, :] - col_off[:, None]) ** 2)
            gy = np.exp(-(uy[None, :] - row_off[:, None]) ** 2)
            mono = [ux ** a * uy ** b for a, b in EXPONENTS]
            sv = (vals.astype(np.float64) - shift) / scale
        else:
            ux = (pts[:, 0] - ax) * inv_h
            uy = (pts[:, 1] - ay) * inv_h
            gx = np.exp(-(ux[None, :] - col_off.astype(np.float32)[:, None]) ** 2).astype(
                np.float32)
            gy = np.exp(-(uy[None, :] - row_off.astype(np.float32)[:, None]) ** 2).astype(
                np.float32)
            # the monomials as successive float32 products
            m = {(0, 0): np.ones(n, np.float32), (1, 0): ux, (0, 1): uy}
            for a, b in EXPONENTS[3:]:
                m[(a, b)] = m[(a - 1, b)] * ux if a > 0 and b == 0 else m[(a, b - 1)] * uy
            mono = [m[e] for e in EXPONENTS]
            sv = staged
        wgt = (gy[:, None, :] * gx[None, :, :]).reshape(256, n)    # node = row * 16 + col
        G = np.stack(mono + [mono[j] * sv[:, d] for j in range(6) for d in range(D)], 1)
        if features == "bf16":
            terms_g, rest = [], G.astype(np.float32)
            for _ in range(terms):
                q = bf16(rest)
                terms_g.append(q)
                rest = (rest - q).astype(np.float32)
            if rhs_terms is not None:
                for s in range(rhs_terms, terms):
                    terms_g[s] = terms_g[s].copy()
                    terms_g[s][:, 15:] = 0.0
        else:
            terms_g = [G]
        if weight == "exact":
            products = [(wgt, s) for s in range(len(terms_g))]
        else:
            whi = bf16(wgt)
            wlo = bf16((wgt - whi).astype(np.float32))
            products = []
            for s in range(len(terms_g)):
                products.append((whi, s))
                if (weight == "split" and s + 1 < len(terms_g)) or (weight == "lo1" and s == 0):
                    products.append((wlo, s))
        F = G.shape[1]
        if accumulate == "f64":
            A = np.zeros((256, F))
            for wm, s in products:
                A += wm.astype(np.float64) @ terms_g[s].astype(np.float64)
        else:
            A = np.zeros((256, F), np.float32)
            for k in range(0, n, KSTEP):
                for wm, s in products:
                    part = wm[:, k:k + KSTEP].astype(np.float64) @ \
                        terms_g[s][k:k + KSTEP].astype(np.float64)
                    A = (A.astype(np.float64) + part).astype(np.float32)
            A = A.astype(np.float64)
        for node in range(256):
            r, c = r0 + node // 16, c0 + node % 16
            if r >= H or c >= W:
                continue
            g = A[node]
            M = np.array([[g[MONO[(a1 + a2, b1 + b2)]] for a2, b2 in BASIS] for a1, b1 in BASIS])
            R = g[15:].reshape(6, D)
            try:
                coef = np.linalg.solve(M, R)
            except np.linalg.LinAlgError:
                continue
            ex, ey = col_off[node % 16], row_off[node // 16]
            phi = np.array([ex ** a * ey ** b for a, b in BASIS])
            out[:, r, c] = (phi @ coef) * scale.astype(np.float64) + \
                shift.astype(np.float64)
    return out
