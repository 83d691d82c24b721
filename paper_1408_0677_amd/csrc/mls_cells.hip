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
// clusters start first; the order keeps 4 x 4 supertiles of neighbouring
// tiles together on one XCD, so that their shared points stay in its L2.
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

// Multi-block exclusive scan, in place: each block scans 1024 values and
// writes its total; then each block adds the sum of the totals before it.
constexpr int kScanBlock = 1024;

__global__ __launch_bounds__(256) void scan_blocks_u32_kernel(uint32_t* v, int64_t count,
                                                              uint32_t* sums) {
  __shared__ uint32_t wsum[4];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + 4 * t;
  uint32_t x[4], sum = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    x[q] = base + q < count ? v[base + q] : 0u;
    sum += x[q];
  }
  uint32_t incl = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t nb = __shfl_up(incl, o, 64);
    if (lane >= o) incl += nb;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  uint32_t run = incl - sum, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    if (w < wave) run += wsum[w];
    tot += wsum[w];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (base + q < count) v[base + q] = run;
    run += x[q];
  }
  if (t == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void scan_add_u32_kernel(uint32_t* v, int64_t count,
                                                           const uint32_t* sums) {
  __shared__ uint32_t wsum[4];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int b = blockIdx.x;
  uint32_t s = 0;
  for (int j = t; j < b; j += 256) s += sums[j];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) wsum[wave] = s;
  __syncthreads();
  const uint32_t prefix = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  const int64_t base = (int64_t)b * kScanBlock;
  for (int q = t; q < kScanBlock; q += 256)
    if (base + q < count) v[base + q] += prefix;
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

// cell_start from the sorted cell ids: the first point of each run of ids
// writes its index into the start of every cell from the previous run's id
// + 1 up to its own (empty cells between take the same start); the last
// point closes the cells after it.  No atomics.
__global__ __launch_bounds__(256) void cell_start_kernel(const uint32_t* sorted_keys, int64_t n,
                                                         int64_t ncells, uint32_t* cell_start) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int64_t k = sorted_keys[i];
  const int64_t prev = i == 0 ? -1 : (int64_t)sorted_keys[i - 1];
  for (int64_t c = prev + 1; c <= k; ++c) cell_start[c] = (uint32_t)i;
  if (i == n - 1)
    for (int64_t c = k + 1; c <= ncells; ++c) cell_start[c] = (uint32_t)n;
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

// Work of each 4 x 4 supertile (the sum of its tiles' list lengths, from
// the scanned list starts), as a descending sort key; iota of the ids.
__global__ __launch_bounds__(256) void supertile_work_kernel(const uint32_t* tile_start,
                                                             int tiles_x, int tiles_y,
                                                             int super_x, int nsuper,
                                                             uint32_t* keys, uint32_t* ids) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= nsuper) return;
  const int sx = s % super_x, sy = s / super_x;
  uint64_t work = 0;
  for (int k = 0; k < kSuperTile * kSuperTile; ++k) {
    const int tc = sx * kSuperTile + k % kSuperTile, tr = sy * kSuperTile + k / kSuperTile;
    if (tc < tiles_x && tr < tiles_y) {
      const int t = tr * tiles_x + tc;
      work += tile_start[t + 1] - tile_start[t];
    }
  }
  keys[s] = 0xFFFFFFFFu - (work > 0xFFFFFFFEull ? 0xFFFFFFFEu : (uint32_t)work);
  ids[s] = (uint32_t)s;
}

// Supertile of rank j (heaviest first) goes to XCD j % 8, as its slot
// j / 8 there; its tiles take 16 consecutive workgroups of that XCD
// (workgroup b runs on XCD b % 8).
__global__ __launch_bounds__(256) void tile_slots_kernel(const uint32_t* sorder, int tiles_x,
                                                         int tiles_y, int super_x, int nsuper,
                                                         uint32_t* torder) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  constexpr int kPer = kSuperTile * kSuperTile;
  const int64_t j = i / kPer;
  const int k = (int)(i % kPer);
  if (j >= nsuper) return;
  const int s = (int)sorder[j];
  const int tc = (s % super_x) * kSuperTile + k % kSuperTile;
  const int tr = (s / super_x) * kSuperTile + k / kSuperTile;
  const int64_t slot = 8 * (kPer * (j / 8) + k) + j % 8;
  torder[slot] = (tc < tiles_x && tr < tiles_y) ? (uint32_t)(tr * tiles_x + tc) : 0xFFFFFFFFu;
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

int64_t scan_sums_words(int64_t count) { return (count + kScanBlock - 1) / kScanBlock; }

hipError_t scan_u32(uint32_t* v, int64_t count, uint32_t* sums, hipStream_t s) {
  const unsigned nb = (unsigned)scan_sums_words(count);
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(scan_blocks_u32_kernel, dim3(nb), dim3(256), 0, s, v, count, sums);
  hipLaunchKernelGGL(scan_add_u32_kernel, dim3(nb), dim3(256), 0, s, v, count,
                     (const uint32_t*)sums);
  return hipGetLastError();
}

// Stable sort of (key, val) pairs by the low `bits` bits of key.  On return
// the result is in (k0, v0); (k1, v1) are scratch of the same size; hist
// holds 256 * radix_blocks(n) words.
hipError_t radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n,
                            int bits, uint32_t* hist, uint32_t* sums, hipStream_t s) {
  const int nblk = (int)radix_blocks(n);
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(radix_upsweep_kernel, dim3(nblk), dim3(kSortThreads), 0, s, k0, n, shift,
                       hist, nblk);
    scan_u32(hist, (int64_t)kDigits * nblk, sums, s);
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
  hipError_t e = radix_sort_pairs(a.keys, a.perm, a.keys2, a.perm2, n, bits, a.hist, a.ssum, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cell_start_kernel, dim3(gb), dim3(256), 0, s, a.keys, n, (int64_t)ncells,
                     a.cell_start);
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
  scan_u32(a.tile_start, (int64_t)a.tiles + 1, a.ssum, s);
  hipLaunchKernelGGL(tile_list_kernel, dim3(lb), dim3(256), 0, s, a.cell_start, a.pts_s, a.ncx,
                     a.ncy, a.geom, a.tiles_x, a.tiles, (uint32_t*)nullptr, (uint32_t*)nullptr,
                     (const uint32_t*)a.tile_start, a.tile_list, a.list_cap);
  // workgroup order: supertiles by descending work, dealt to the XCDs
  const int tiles_y = a.tiles / a.tiles_x;
  const int super_x = (a.tiles_x + kSuperTile - 1) / kSuperTile;
  const int nsuper = super_x * ((tiles_y + kSuperTile - 1) / kSuperTile);
  const int64_t slots = tile_order_slots(a.tiles_x, tiles_y);
  hipLaunchKernelGGL(supertile_work_kernel, dim3((unsigned)((nsuper + 255) / 256)), dim3(256), 0,
                     s, a.tile_start, a.tiles_x, tiles_y, super_x, nsuper, a.tkeys, a.sorder);
  e = radix_sort_pairs(a.tkeys, a.sorder, a.tkeys2, a.torder2, nsuper, 32, a.thist, a.ssum, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((slots + 255) / 256)), dim3(256), 0, s,
                     a.torder, slots, 0xFFFFFFFFu);
  hipLaunchKernelGGL(tile_slots_kernel,
                     dim3((unsigned)(((int64_t)nsuper * kSuperTile * kSuperTile + 255) / 256)),
                     dim3(256), 0, s, a.sorder, a.tiles_x, tiles_y, super_x, nsuper, a.torder);
  return hipGetLastError();
}

}  // namespace mls
