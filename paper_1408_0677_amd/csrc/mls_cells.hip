// Device cell list for compactly supported weights (Wendland C2), the
// localised sampling that replaces the all-points loop (the paper notes the
// per-pixel O(n) cost as its limitation and names localised sampling as the
// way past it, Sec. 4.6 / Sec. 5).
//
// Cells are squares of side h (the support radius) over the points'
// bounding box, so a node's support touches at most 3 x 3 cells and a
// 16 x 16 node tile a small block of cells.  Binning is a stable counting
// sort by cell id, written as an LSD radix sort with 8-bit digits:
//   upsweep    per-block digit histograms,
//   scan       exclusive scan in (digit, block) order,
//   downsweep  stable scatter: keys are ranked inside a block round by round
//              (one key per thread per round, in index order) with wave
//              ballots and per-wave digit counts in LDS,
// so points of one cell keep their input order and every run produces the
// same payload.  Then per-cell counts (cell_start by exclusive scan) and a
// gather of coordinates and normalised attributes into cell order.  Then
// per node tile the list of points within h of its nodes (from the cells
// the tile's support reaches, so a tile's fit touches no point that cannot
// weigh in; the cells alone hold 2-4x more), and a second sort that orders
// node tiles by descending list length, so that the heavy tiles of dense
// clusters start first.
// All of it is bound by HBM and launch latency, not arithmetic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mls_internal.h"

namespace mls {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;                              // keys per thread per block
constexpr int kSortTile = kSortThreads * kSortRounds;       // 2048 keys per block
constexpr int kDigits = 256;

__device__ __forceinline__ uint32_t digit_of(uint32_t key, int shift) {
  return (key >> shift) & (kDigits - 1);
}

__global__ __launch_bounds__(kSortThreads) void radix_upsweep_kernel(const uint32_t* keys,
                                                                     int64_t n, int shift,
                                                                     uint32_t* hist, int nblk) {
  __shared__ uint32_t h[kDigits];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + r * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[digit_of(keys[i], shift)], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of `count` uint32 values in place, one block of 1024
// threads (sequential runs per thread, then a block scan of the run sums).
__global__ __launch_bounds__(1024) void scan_u32_kernel(uint32_t* v, int64_t count,
                                                        uint32_t* total) {
  __shared__ uint32_t wsum[16];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t per = (count + 1023) / 1024;
  const int64_t lo = t * per, hi = lo + per < count ? lo + per : count;
  uint32_t s = 0;
  for (int64_t q = lo; q < hi; ++q) s += v[q];
  uint32_t incl = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t nb = __shfl_up(incl, o, 64);
    if (lane >= o) incl += nb;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t wbase = 0, tot = 0;
  for (int w = 0; w < 16; ++w) {
    if (w < wave) wbase += wsum[w];
    tot += wsum[w];
  }
  uint32_t run = wbase + incl - s;
  for (int64_t q = lo; q < hi; ++q) {
    const uint32_t x = v[q];
    v[q] = run;
    run += x;
  }
  if (t == 0 && total) *total = tot;
}

__global__ __launch_bounds__(kSortThreads) void radix_downsweep_kernel(
    const uint32_t* keys_in, const uint32_t* vals_in, int64_t n, int shift, const uint32_t* offs,
    int nblk, uint32_t* keys_out, uint32_t* vals_out) {
  __shared__ uint32_t wave_cnt[4][kDigits];   // keys per digit in each wave, this pass
  __shared__ uint32_t running[kDigits];       // keys per digit in earlier rounds of this block
  __shared__ uint32_t wave_base[4][kDigits];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  running[t] = 0;
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t i = base + r * kSortThreads + t;
    const bool valid = i < n;
    const uint32_t key = valid ? keys_in[i] : 0u;
    const uint32_t val = valid ? vals_in[i] : 0u;
    const uint32_t d = valid ? digit_of(key, shift) : 0xFFFFFFFFu;
    for (int q = t; q < 4 * kDigits; q += kSortThreads) (&wave_cnt[0][0])[q] = 0;
    __syncthreads();
    // peers: lanes of this wave with the same digit
    uint64_t remaining = __ballot(valid);
    uint64_t peers = 0;
    while (remaining) {
      const int leader = __ffsll((unsigned long long)remaining) - 1;
      const uint32_t ld = __shfl(d, leader, 64);
      const uint64_t m = __ballot(d == ld) & remaining;
      if (d == ld) peers = m;
      remaining &= ~m;
    }
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint32_t rank_in_wave = (uint32_t)__popcll(peers & lt);
    if (valid && rank_in_wave == 0) wave_cnt[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    // per digit: bases of the four waves after the earlier rounds
    {
      uint32_t acc = running[t];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        wave_base[w][t] = acc;
        acc += wave_cnt[w][t];
      }
      running[t] = acc;
    }
    __syncthreads();
    if (valid) {
      const uint32_t pos = offs[(int64_t)d * nblk + blockIdx.x] + wave_base[wave][d] + rank_in_wave;
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    __syncthreads();
  }
}

// Cell id of every point; iota of the point indices.
__global__ __launch_bounds__(256) void cell_ids_kernel(const float* pts, int64_t n, double ox,
                                                       double oy, double inv_cell, int ncx,
                                                       int ncy, uint32_t* keys, uint32_t* idx) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  int cx = (int)floor(((double)pts[2 * i] - ox) * inv_cell);
  int cy = (int)floor(((double)pts[2 * i + 1] - oy) * inv_cell);
  cx = cx < 0 ? 0 : (cx >= ncx ? ncx - 1 : cx);
  cy = cy < 0 ? 0 : (cy >= ncy ? ncy - 1 : cy);
  keys[i] = (uint32_t)(cy * ncx + cx);
  idx[i] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void cell_count_kernel(const uint32_t* sorted_keys, int64_t n,
                                                         uint32_t* counts) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) atomicAdd(&counts[sorted_keys[i]], 1u);
}

// Sorted payload: coordinates and the attribute-major normalised values.
__global__ __launch_bounds__(256) void gather_points_kernel(const float* pts, const uint32_t* perm,
                                                            int64_t n, float* pts_s) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t j = perm[i];
  pts_s[2 * i] = pts[2 * j];
  pts_s[2 * i + 1] = pts[2 * j + 1];
}

__global__ __launch_bounds__(256) void gather_values_kernel(const float* vals_t, const uint32_t* perm,
                                                            int64_t n, int D, float* vals_ts) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int d = blockIdx.y;
  if (i >= n) return;
  vals_ts[(int64_t)d * n + i] = vals_t[(int64_t)d * n + perm[i]];
}

__global__ __launch_bounds__(256) void iota_u32_kernel(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = (uint32_t)i;
}

// Per-tile point lists.  One wave per node tile walks the cell runs the
// tile's support can reach and keeps the points within h of the tile's
// node rectangle (a point farther than that has zero weight at every node
// of the tile), in cell order.  Count pass (list == null): the number of
// such points goes to counts[tile] and, as a descending-work sort key, to
// keys[tile].  Fill pass: the indices are written from tile_start[tile] on.
// The test runs in float64 with a relative margin of 1e-4 on h^2, so that
// a point the fit kernel's float32 distance could still place inside the
// support is never dropped; the extra points get zero weight there.
__global__ __launch_bounds__(256) void tile_list_kernel(const uint32_t* cell_start,
                                                        const float* pts_s, int ncx, int ncy,
                                                        CellGeom g, int tiles_x, int tiles,
                                                        uint32_t* counts, uint32_t* keys,
                                                        const uint32_t* tile_start,
                                                        uint32_t* list, int64_t list_cap) {
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= tiles) return;   // whole wave; no barrier below
  const int tc = tile % tiles_x, tr = tile / tiles_x;
  int cx0, cx1, cy0, cy1;
  tile_cell_range(g, tc, tr, ncx, ncy, &cx0, &cx1, &cy0, &cy1);
  const double xa = g.x0 + (double)(tc * kTileCols) * g.dx;
  const double xb = g.x0 + (double)(tc * kTileCols + kTileCols - 1) * g.dx;
  const double ya = g.y0 + (double)(tr * kTileRows) * g.dy;
  const double yb = g.y0 + (double)(tr * kTileRows + kTileRows - 1) * g.dy;
  const double xlo = fmin(xa, xb), xhi = fmax(xa, xb), ylo = fmin(ya, yb), yhi = fmax(ya, yb);
  const double reach2 = g.h * g.h * (1.0 + 1e-4);
  const uint64_t below = (1ull << lane) - 1ull;
  int64_t out = list ? (int64_t)tile_start[tile] : 0;
  uint32_t cnt = 0;
  for (int cy = cy0; cy <= cy1; ++cy) {
    const int64_t a = cell_start[cy * ncx + cx0];
    const int64_t b = cell_start[cy * ncx + cx1 + 1];
    for (int64_t k0 = a; k0 < b; k0 += 64) {
      const int64_t k = k0 + lane;
      bool in = false;
      if (k < b) {
        const double x = (double)pts_s[2 * k], y = (double)pts_s[2 * k + 1];
        const double ex = fmax(fmax(xlo - x, x - xhi), 0.0);
        const double ey = fmax(fmax(ylo - y, y - yhi), 0.0);
        in = ex * ex + ey * ey < reach2;
      }
      const uint64_t m = __ballot(in);
      if (list && in) {
        const int64_t o = out + __popcll(m & below);
        if (o < list_cap) list[o] = (uint32_t)k;
      }
      out += __popcll(m);
      cnt += (uint32_t)__popcll(m);
    }
  }
  if (!list && lane == 0) {
    counts[tile] = cnt;
    keys[tile] = 0xFFFFFFFFu - cnt;
  }
}

}  // namespace

int64_t tile_list_bound(int64_t n, double h, double dx, double dy, int tiles_x, int tiles_y) {
  // a point is listed by tile t when it lies within h of t's node
  // rectangle: along x that is a window of 2 h + 15 |dx| for the tiles'
  // first nodes, which are 16 |dx| apart (likewise along y)
  const double hh = h * 1.0001;
  auto per_axis = [&](double d, int tiles) -> int64_t {
    const double w = 16.0 * fabs(d);
    if (!(w > 0.0)) return tiles;
    const double k = floor((2.0 * hh + w) / w) + 1.0;
    return k < (double)tiles ? (int64_t)k : (int64_t)tiles;
  };
  return n * per_axis(dx, tiles_x) * per_axis(dy, tiles_y);
}

int64_t radix_blocks(int64_t n) { return (n + kSortTile - 1) / kSortTile; }

// Stable sort of (key, val) pairs by the low `bits` bits of key.  On return
// the result is in (k0, v0); (k1, v1) are scratch of the same size; hist
// holds 256 * radix_blocks(n) words.
hipError_t radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n,
                            int bits, uint32_t* hist, hipStream_t s) {
  const int nblk = (int)radix_blocks(n);
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(radix_upsweep_kernel, dim3(nblk), dim3(kSortThreads), 0, s, k0, n, shift,
                       hist, nblk);
    hipLaunchKernelGGL(scan_u32_kernel, dim3(1), dim3(1024), 0, s, hist,
                       (int64_t)kDigits * nblk, (uint32_t*)nullptr);
    hipLaunchKernelGGL(radix_downsweep_kernel, dim3(nblk), dim3(kSortThreads), 0, s, k0, v0, n,
                       shift, hist, nblk, k1, v1);
    uint32_t* tk = k0; k0 = k1; k1 = tk;
    uint32_t* tv = v0; v0 = v1; v1 = tv;
  }
  // an odd number of passes leaves the result in the scratch pair
  if (((bits + 7) / 8) % 2 == 1) {
    hipMemcpyAsync(k1, k0, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s);
    hipMemcpyAsync(v1, v0, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s);
  }
  return hipGetLastError();
}

hipError_t launch_cells(const CellArgs& a, hipStream_t s) {
  const int64_t n = a.n;
  const unsigned gb = (unsigned)((n + 255) / 256);
  const int ncells = a.ncx * a.ncy;
  hipLaunchKernelGGL(cell_ids_kernel, dim3(gb), dim3(256), 0, s, a.pts, n, a.geom.ox, a.geom.oy,
                     1.0 / a.geom.cell, a.ncx, a.ncy, a.keys, a.perm);
  int bits = 0;
  while ((1 << bits) < ncells) ++bits;
  if (bits < 8) bits = 8;
  hipError_t e = radix_sort_pairs(a.keys, a.perm, a.keys2, a.perm2, n, bits, a.hist, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((ncells + 1 + 255) / 256)), dim3(256), 0, s,
                     a.cell_start, (int64_t)ncells + 1, 0u);
  hipLaunchKernelGGL(cell_count_kernel, dim3(gb), dim3(256), 0, s, a.keys, n, a.cell_start);
  hipLaunchKernelGGL(scan_u32_kernel, dim3(1), dim3(1024), 0, s, a.cell_start,
                     (int64_t)ncells + 1, (uint32_t*)nullptr);
  hipLaunchKernelGGL(gather_points_kernel, dim3(gb), dim3(256), 0, s, a.pts, a.perm, n, a.pts_s);
  hipLaunchKernelGGL(gather_values_kernel, dim3(gb, a.D), dim3(256), 0, s, a.vals_t, a.perm, n,
                     a.D, a.vals_ts);
  // per-tile point lists: counts (and the work keys), starts, entries
  const unsigned lb = (unsigned)((a.tiles + 3) / 4);
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((a.tiles + 1 + 255) / 256)), dim3(256), 0,
                     s, a.tile_start, (int64_t)a.tiles + 1, 0u);
  hipLaunchKernelGGL(tile_list_kernel, dim3(lb), dim3(256), 0, s, a.cell_start, a.pts_s, a.ncx,
                     a.ncy, a.geom, a.tiles_x, a.tiles, a.tile_start, a.tkeys,
                     (const uint32_t*)nullptr, (uint32_t*)nullptr, (int64_t)0);
  hipLaunchKernelGGL(scan_u32_kernel, dim3(1), dim3(1024), 0, s, a.tile_start,
                     (int64_t)a.tiles + 1, (uint32_t*)nullptr);
  hipLaunchKernelGGL(tile_list_kernel, dim3(lb), dim3(256), 0, s, a.cell_start, a.pts_s, a.ncx,
                     a.ncy, a.geom, a.tiles_x, a.tiles, (uint32_t*)nullptr, (uint32_t*)nullptr,
                     (const uint32_t*)a.tile_start, a.tile_list, a.list_cap);
  // tile order by descending work (list length)
  const int tb = (a.tiles + 255) / 256;
  hipLaunchKernelGGL(iota_u32_kernel, dim3(tb), dim3(256), 0, s, a.torder, (int64_t)a.tiles);
  e = radix_sort_pairs(a.tkeys, a.torder, a.tkeys2, a.torder2, a.tiles, 32, a.thist, s);
  return e != hipSuccess ? e : hipGetLastError();
}

}  // namespace mls
