"""Seeded synthetic workloads for MLS field evaluation.

This module only draws inputs: scattered 2-D points, attribute values per
point, grid descriptions and isovalues.  It contains none of the fitting or
contouring arithmetic, so both the GPU library's callers and the independent
CPU oracle can take their inputs from here.

The paper's datasets are not available; these generators stand in for them
with the shapes its workloads have (Muelder et al., Sec. 4.5: a few hundred to
a few thousand projected points at screen resolution), widened to the sizes
the GPU path is measured on:

* ``c1``  200 uniform points, 4 analytic attributes, 128^2 grid (CPU scale).
* ``c2``  5,000 points from an 8-component Gaussian mixture, 13 random smooth
  attributes, linear basis, Gaussian h = 0.03, 1024^2 grid, 10 isovalues.
* ``c3``  50,000 mixture points, 64 attributes, quadratic, h = 0.015, 2048^2.
* ``c4``  256 requests of random size for the served form.
* ``c5``  1,000,000 points (background + 32 tight clusters), 16 attributes,
  Wendland C2 support 0.01, quadratic, 4096^2, 16 isovalues.

Coordinates and values are generated in float64 and returned as float32:
those float32 arrays are exactly what every consumer sees.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def pixel_grid(width: int, height: int | None = None) -> dict:
    """Grid of pixel centres over the unit square: node (r, c) at
    ((c + 0.5) / W, (r + 0.5) / H), rows increasing in y."""
    height = width if height is None else height
    return {"x0": 0.5 / width, "y0": 0.5 / height, "dx": 1.0 / width,
            "dy": 1.0 / height, "width": int(width), "height": int(height)}


def uniform_points(rng, n):
    return rng.random((n, 2))


def mixture_points(rng, n, k=8, centre_lo=0.15, centre_hi=0.85, sigma_lo=0.03,
                   sigma_hi=0.1):
    """Isotropic Gaussian mixture with equal component weights; samples that
    fall outside the unit square are drawn again from the same component."""
    centres = rng.uniform(centre_lo, centre_hi, size=(k, 2))
    sigmas = rng.uniform(sigma_lo, sigma_hi, size=k)
    comp = rng.integers(0, k, size=n)
    pts = centres[comp] + sigmas[comp, None] * rng.standard_normal((n, 2))
    bad = np.any((pts < 0.0) | (pts > 1.0), axis=1)
    while bad.any():
        idx = np.nonzero(bad)[0]
        pts[idx] = centres[comp[idx]] + sigmas[comp[idx], None] * \
            rng.standard_normal((idx.size, 2))
        bad = np.any((pts < 0.0) | (pts > 1.0), axis=1)
    return pts


def clustered_points(rng, n, n_clusters=32, background=0.2, sigma_lo=0.002,
                     sigma_hi=0.02):
    """Uniform background plus tight isotropic clusters (large compact-support
    case)."""
    n_bg = int(round(background * n))
    n_cl = n - n_bg
    bg = rng.random((n_bg, 2))
    centres = rng.uniform(0.05, 0.95, size=(n_clusters, 2))
    sigmas = rng.uniform(sigma_lo, sigma_hi, size=n_clusters)
    comp = np.repeat(np.arange(n_clusters), n_cl // n_clusters)
    comp = np.concatenate([comp, rng.integers(0, n_clusters, n_cl - comp.size)])
    pts = centres[comp] + sigmas[comp, None] * rng.standard_normal((n_cl, 2))
    bad = np.any((pts < 0.0) | (pts > 1.0), axis=1)
    while bad.any():
        idx = np.nonzero(bad)[0]
        pts[idx] = centres[comp[idx]] + sigmas[comp[idx], None] * \
            rng.standard_normal((idx.size, 2))
        bad = np.any((pts < 0.0) | (pts > 1.0), axis=1)
    allp = np.concatenate([bg, pts])
    return allp[rng.permutation(n)]


def smooth_fields(rng, pts, d, n_waves=8, kmax=3, noise=0.01):
    """D random smooth fields: sums of plane waves with integer wave vectors
    in [-kmax, kmax]^2 \\ {0}, amplitude N(0,1)/|k|, random phase, plus
    Gaussian noise of standard deviation noise * (range of the clean field)."""
    n = pts.shape[0]
    out = np.empty((n, d))
    for j in range(d):
        acc = np.zeros(n)
        for _ in range(n_waves):
            while True:
                kv = rng.integers(-kmax, kmax + 1, size=2)
                if kv[0] != 0 or kv[1] != 0:
                    break
            a = rng.standard_normal() / math.hypot(kv[0], kv[1])
            phi = rng.uniform(0.0, 2.0 * math.pi)
            acc += a * np.sin(2.0 * math.pi * (pts @ kv) + phi)
        rng_span = acc.max() - acc.min()
        out[:, j] = acc + noise * rng_span * rng.standard_normal(n)
    return out


def analytic_fields(rng, pts, noise_sigma=0.01, noise=True):
    """The four analytic attributes of the CPU-scale case: a plane, a
    quadratic, a product of sinusoids and a Gaussian bump."""
    x, y = pts[:, 0], pts[:, 1]
    f = np.stack([1.0 + 2.0 * x - 3.0 * y,
                  x * x - x * y + 0.5 * y * y,
                  np.sin(2 * math.pi * x) * np.cos(2 * math.pi * y),
                  np.exp(-((x - 0.3) ** 2 + (y - 0.7) ** 2) / 0.05)], axis=1)
    if noise:
        f = f + noise_sigma * rng.standard_normal(f.shape)
    return f


def isovalues(values, n_iso):
    """n_iso isovalues per attribute, evenly spaced strictly inside the range
    of the input values: lo + (k + 1) (hi - lo) / (n_iso + 1)."""
    v = np.asarray(values, dtype=np.float64)
    lo, hi = v.min(axis=0), v.max(axis=0)
    k = np.arange(1, n_iso + 1, dtype=np.float64)
    return (lo[:, None] + k[None, :] * (hi - lo)[:, None] / (n_iso + 1)).astype(
        np.float32)


@dataclass
class Workload:
    name: str
    points: np.ndarray            # (N, 2) float32
    values: np.ndarray            # (N, D) float32
    basis: str                    # "constant" | "linear" | "quadratic"
    weight: str                   # "gaussian" | "wendland" | "invpow"
    h: float
    grid: dict
    precision: str = "fp32"
    n_iso: int = 0
    alpha: float = 1.0
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.points.shape[0]

    @property
    def d(self):
        return self.values.shape[1]

    def iso(self):
        return isovalues(self.values, self.n_iso) if self.n_iso else None


def c1(seed=0, noise=True):
    rng = np.random.default_rng(seed)
    pts = uniform_points(rng, 200)
    vals = analytic_fields(rng, pts, noise=noise)
    return Workload("c1_n200_d4_linear_gauss_h0.05_128", pts.astype(np.float32),
                    vals.astype(np.float32), "linear", "gaussian", 0.05,
                    pixel_grid(128), "fp64", n_iso=10)


def c2(seed=0, grid_side=1024, n=5000):
    rng = np.random.default_rng(seed)
    pts = mixture_points(rng, n, k=8)
    vals = smooth_fields(rng, pts, 13)
    return Workload(f"c2_n{n}_d13_linear_gauss_h0.03_{grid_side}",
                    pts.astype(np.float32), vals.astype(np.float32), "linear",
                    "gaussian", 0.03, pixel_grid(grid_side), "fp32", n_iso=10)


def c3(seed=0, grid_side=2048, n=50000, d=64):
    rng = np.random.default_rng(seed)
    pts = mixture_points(rng, n, k=8)
    vals = smooth_fields(rng, pts, d)
    return Workload(f"c3_n{n}_d{d}_quadratic_gauss_h0.015_{grid_side}",
                    pts.astype(np.float32), vals.astype(np.float32), "quadratic",
                    "gaussian", 0.015, pixel_grid(grid_side), "bf16", n_iso=0)


def c5(seed=0, grid_side=4096, n=1_000_000, d=16):
    rng = np.random.default_rng(seed)
    pts = clustered_points(rng, n)
    vals = smooth_fields(rng, pts, d)
    return Workload(f"c5_n{n}_d{d}_quadratic_wendland_h0.01_{grid_side}",
                    pts.astype(np.float32), vals.astype(np.float32), "quadratic",
                    "wendland", 0.01, pixel_grid(grid_side), "bf16", n_iso=16)


def t1(n, seed=0):
    """Shape of the paper's timing table (Table 1): a 600 x 600 canvas, N
    uniform points, two attributes, the linear basis with the paper's own
    inverse-distance weight (Eq. 4, alpha = 1)."""
    rng = np.random.default_rng(seed + n)
    pts = uniform_points(rng, n)
    vals = smooth_fields(rng, pts, 2)
    return Workload(f"t1_n{n}_d2_linear_invpow_a1_600", pts.astype(np.float32),
                    vals.astype(np.float32), "linear", "invpow", 0.05, pixel_grid(600),
                    "fp64", n_iso=10, alpha=1.0)


def mesh_arrays(points):
    """Delaunay triangulation of (N, 2) points (the paper's upstream step,
    done here on the host with scipy) as the layout's inputs: CSR
    neighbour lists (adj_start[N+1], adj) and triangle fans (fan_start[N+1],
    fan[2 T_v]: the other two vertices of each triangle around a node), all
    int32, plus the triangles (T, 3)."""
    from scipy.spatial import Delaunay
    pts = np.asarray(points, dtype=np.float64)
    n = pts.shape[0]
    tri = Delaunay(pts).simplices.astype(np.int64)
    nb = [set() for _ in range(n)]
    fans = [[] for _ in range(n)]
    for a, b, c in tri:
        nb[a].update((b, c)); nb[b].update((a, c)); nb[c].update((a, b))
        fans[a].append((b, c)); fans[b].append((c, a)); fans[c].append((a, b))
    adj_start = np.zeros(n + 1, np.int32)
    adj_start[1:] = np.cumsum([len(x) for x in nb])
    adj = np.array([u for x in nb for u in sorted(x)], np.int32)
    fan_start = np.zeros(n + 1, np.int32)
    fan_start[1:] = np.cumsum([len(x) for x in fans])
    fan = np.array([v for x in fans for pr in x for v in pr], np.int32)
    return {"adj_start": adj_start, "adj": adj, "fan_start": fan_start, "fan": fan,
            "triangles": tri.astype(np.int32)}


def layout_workload(n, seed=0, canvas=600.0):
    """Timing-table layout shape: n uniform points on a canvas x canvas
    square, their Delaunay mesh, and parameters in canvas units: D the mean
    edge length, C = D^3 (repulsion of about D at distance D), eta = 1e-3 D,
    t0 = D / 4, lambda = 0.995."""
    rng = np.random.default_rng(seed + n)
    pts = rng.random((n, 2)) * canvas
    mesh = mesh_arrays(pts)
    src = np.repeat(np.arange(n), np.diff(mesh["adj_start"]))
    D = float(np.linalg.norm(pts[src] - pts[mesh["adj"]], axis=1).mean())
    params = {"C": D ** 3, "D": D, "eta": 1e-3 * D, "t0": 0.25 * D, "lam": 0.995}
    return pts, mesh, params


def c4_requests(seed=0, count=256):
    """Request mix of the served form: sizes, bases and bandwidths drawn at
    random; the bandwidth puts about 20 (linear) or 40 (quadratic) points
    inside radius h for uniform density."""
    rng = np.random.default_rng(seed)
    reqs = []
    for q in range(count):
        n = int(rng.integers(500, 20001))
        d = int(rng.integers(4, 33))
        side = int(rng.integers(256, 1025))
        basis = "linear" if rng.random() < 0.5 else "quadratic"
        if rng.random() < 0.5:
            pts = mixture_points(rng, n, k=int(rng.integers(1, 9)))
        else:
            pts = uniform_points(rng, n)
        vals = smooth_fields(rng, pts, d)
        target = 20.0 if basis == "linear" else 40.0
        h = math.sqrt(target / (math.pi * n))
        reqs.append(Workload(f"c4_req{q}", pts.astype(np.float32),
                             vals.astype(np.float32), basis, "gaussian", h,
                             pixel_grid(side), "fp16"))
    return reqs


def poisson_arrivals(rng_seed, count, rate_per_s):
    """Arrival times (seconds from 0) of a Poisson process."""
    rng = np.random.default_rng(rng_seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))
