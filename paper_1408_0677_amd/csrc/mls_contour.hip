// Marching-squares contour lines of MLS fields (Muelder et al., Sec. 3.4:
// contour lines are the simplest rendering of the MLS output; the
// extraction rule below is this library's choice).
//
// Cell (i, j) of an H x W field has corners v0 = f[i][j], v1 = f[i][j+1],
// v2 = f[i+1][j+1], v3 = f[i+1][j]; bit k of its case is (v_k >= iso).  A NaN
// corner (undetermined node) gives case 255 and no segment.  Saddles 5 and 10
// join the above corners when the centre ((v0 + v1) + (v2 + v3)) / 4 >= iso.
// A crossing on an edge is interpolated from the edge endpoint with the
// smaller (row, col), so the two cells sharing an edge produce the same bits.
// Segments run with the >= iso side on their left.  Edge numbering:
// 0 bottom (v0-v1), 1 right (v1-v2), 2 top (v3-v2), 3 left (v0-v3).
//
// Three passes keep the output in (field, iso, cell, segment) order without
// atomics, so it is deterministic:
//   count:  a wave owns a chunk of 256 consecutive cells of one field (four
//           per lane, lane l holding cells l, l + 64, l + 128, l + 192, so
//           the corner loads coalesce) and visits every isovalue with the
//           corners in registers; the chunk's segment count per isovalue is
//           two ballots and two population counts per cell group, with no
//           shuffles and no barriers.  An isovalue outside every lane's
//           [min, max] corner range is skipped with one wave-wide test;
//   scan:   exclusive scan of the counts in (field, iso, chunk) order;
//   emit:   recompute; a segment's slot is the chunk's scanned offset plus
//           the ballot prefix of the cells before it; crossed cells are
//           queued in LDS and their segments and ids written one cell per
//           lane.
// Reading the fields is one pass of HBM traffic per kernel; with many
// isovalues the per-(cell, iso) tests dominate (vector ALU).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/mls.h"
#include "mls_internal.h"

namespace mls {
namespace {

constexpr int kCellsPerLane = 4;
constexpr int kCellsPerWave = 64 * kCellsPerLane;   // one count entry per wave chunk
constexpr int kWavesPerBlock = 4;
constexpr int kScanTile = 1024;      // entries per block of the first scan level

// Segments per case: from-edge, to-edge pairs; cases 5 and 10 are resolved
// by the saddle rule in case_segments().
__constant__ signed char kOneSegment[16][2] = {
    {-1, -1}, {0, 3}, {1, 0}, {1, 3}, {2, 1}, {-1, -1}, {2, 0}, {2, 3},
    {3, 2},   {0, 2}, {-1, -1}, {1, 2}, {3, 1}, {0, 1}, {3, 0}, {-1, -1}};

struct Corners {
  float v0, v1, v2, v3;
  bool valid;
};

__device__ __forceinline__ int cell_case(const Corners& c, float iso) {
  if (!c.valid) return 255;
  return (c.v0 >= iso ? 1 : 0) | (c.v1 >= iso ? 2 : 0) | (c.v2 >= iso ? 4 : 0) |
         (c.v3 >= iso ? 8 : 0);
}

// (from, to) edges of the case's segments in (a0, a1) and (b0, b1);
// returns the segment count.  Scalars, not an array, so that nothing of a
// cell's state needs addressable (scratch) storage.
__device__ __forceinline__ int case_segments(int cs, const Corners& c, float iso, int& a0,
                                             int& a1, int& b0, int& b1) {
#pragma clang fp contract(off)
  a0 = a1 = b0 = b1 = 0;
  if (cs == 5 || cs == 10) {
    const float centre = ((c.v0 + c.v1) + (c.v2 + c.v3)) * 0.25f;
    const bool joined = centre >= iso;
    if (cs == 5) {
      a0 = 0; a1 = joined ? 1 : 3;
      b0 = 2; b1 = joined ? 3 : 1;
    } else {
      a0 = joined ? 3 : 1; a1 = 0;
      b0 = joined ? 1 : 3; b1 = 2;
    }
    return 2;
  }
  if (cs == 255 || kOneSegment[cs][0] < 0) return 0;
  a0 = kOneSegment[cs][0];
  a1 = kOneSegment[cs][1];
  return 1;
}

struct GridD {
  double x0, y0, dx, dy;
};

// World position of the crossing on edge e of cell (i, j).
__device__ __forceinline__ void edge_point(int e, const Corners& c, float iso, int i, int j,
                                           const GridD& g, float* x, float* y) {
#pragma clang fp contract(off)
  float va, vb;
  switch (e) {
    case 0: va = c.v0; vb = c.v1; break;
    case 1: va = c.v1; vb = c.v2; break;
    case 2: va = c.v3; vb = c.v2; break;
    default: va = c.v0; vb = c.v3; break;
  }
  const float t = (iso - va) / (vb - va);
  double px, py;
  switch (e) {
    case 0: px = g.x0 + ((double)j + (double)t) * g.dx; py = g.y0 + (double)i * g.dy; break;
    case 1: px = g.x0 + (double)(j + 1) * g.dx; py = g.y0 + ((double)i + (double)t) * g.dy; break;
    case 2: px = g.x0 + ((double)j + (double)t) * g.dx; py = g.y0 + (double)(i + 1) * g.dy; break;
    default: px = g.x0 + (double)j * g.dx; py = g.y0 + ((double)i + (double)t) * g.dy; break;
  }
  *x = (float)px;
  *y = (float)py;
}

struct ContourParams {
  const float* fields;
  const float* iso;      // [D][n_iso]
  int D, n_iso, W, H;
  int64_t cells;         // (H - 1) * (W - 1)
  int64_t nchunk;        // wave chunks (of kCellsPerWave cells) per field
  int64_t bpf;           // blocks per field
  uint8_t* cases;        // [D][n_iso][cells] or null
  int32_t* counts;       // [D][n_iso][nchunk]
  const int32_t* offsets;  // [D][n_iso][nchunk], exclusive within scan tiles
  const int64_t* tile_prefix;  // exclusive prefix of scan tiles
  float* segs;           // [cap][4]
  int32_t* ids;          // [cap][3] or null
  int64_t capacity;
  GridD g;
};

// Workgroups are dispatched round-robin over the eight XCDs (block b runs on
// XCD b % 8), each with its own L2.  Renumbering so that every XCD works
// through one contiguous eighth of the logical blocks keeps the chunk that
// reads rows i and i + 1 on the XCD that read row i a few blocks earlier,
// so the second read of a row hits that XCD's L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t n) {
  const int64_t per = n / 8, rem = n % 8, x = b % 8, i = b / 8;
  return x * per + (x < rem ? x : rem) + i;
}

// The cells of one wave chunk: corners in registers, and the range of the
// lane's valid corners (an isovalue outside it crosses none of them).
struct WaveCells {
  Corners c[kCellsPerLane];
  // corner range of each cell (+inf, -inf when the cell is outside the grid
  // or has a NaN corner): the cell has segments iff clo < iso <= chi
  float clo[kCellsPerLane], chi[kCellsPerLane];
  int i[kCellsPerLane], j[kCellsPerLane];
  int64_t cell[kCellsPerLane];
  bool in[kCellsPerLane];
  float lo, hi;
};

__device__ __forceinline__ void load_wave_cells(const ContourParams& p, const float* f,
                                                int64_t chunk, int lane, WaveCells& w) {
  const int cw = p.W - 1;
  w.lo = __builtin_inff();
  w.hi = -__builtin_inff();
  // row and column of the chunk's first cell: one division per wave; each
  // lane's cells lie at most kCellsPerWave further on, so a few steps of
  // one row reach them
  const int64_t base = chunk * kCellsPerWave;
  const int64_t row0 = base / cw;
  const int col0 = (int)(base - row0 * cw);
  int64_t at[kCellsPerLane];    // index of corner 0; cells past the grid read cell 0
#pragma unroll
  for (int q = 0; q < kCellsPerLane; ++q) {
    const int64_t cell = base + q * 64 + lane;
    w.cell[q] = cell;
    w.in[q] = cell < p.cells;
    int col = col0 + q * 64 + lane;
    int row = (int)row0;
    while (col >= cw) {
      col -= cw;
      ++row;
    }
    if (!w.in[q]) row = col = 0;
    w.i[q] = row;
    w.j[q] = col;
    at[q] = (int64_t)row * p.W + col;
  }
  // every corner load in flight before the first is used
  float v[kCellsPerLane][4];
#pragma unroll
  for (int q = 0; q < kCellsPerLane; ++q) {
    v[q][0] = f[at[q]];
    v[q][1] = f[at[q] + 1];
    v[q][2] = f[at[q] + p.W + 1];
    v[q][3] = f[at[q] + p.W];
  }
  // keep the scheduler from moving a use of the first loads above the
  // later loads (which would wait for the first before issuing the rest)
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int q = 0; q < kCellsPerLane; ++q) {
    Corners c{v[q][0], v[q][1], v[q][2], v[q][3], false};
    c.valid = w.in[q] && !(isnan(c.v0) || isnan(c.v1) || isnan(c.v2) || isnan(c.v3));
    w.c[q] = c;
    w.clo[q] = c.valid ? fminf(fminf(c.v0, c.v1), fminf(c.v2, c.v3)) : __builtin_inff();
    w.chi[q] = c.valid ? fmaxf(fmaxf(c.v0, c.v1), fmaxf(c.v2, c.v3)) : -__builtin_inff();
    w.lo = fminf(w.lo, w.clo[q]);
    w.hi = fmaxf(w.hi, w.chi[q]);
  }
}

// One step of a wave reduction: x combined with the value the DPP control
// moves in (lanes the row mask leaves out combine x with itself).
template <int CTRL, int ROWS, bool MAX>
__device__ __forceinline__ float dpp_step(float x) {
  const int xi = __builtin_bit_cast(int, x);
  const float y = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(xi, xi, CTRL, ROWS, 0xF, false));
  return MAX ? fmaxf(x, y) : fminf(x, y);
}

// Minimum or maximum over the wave, by lane moves within rows (quad
// permutations, half-row and row mirrors) and the two row broadcasts;
// lane 63 ends with the whole wave's value.  Short dependent steps of the
// vector unit, where lane shuffles through LDS wait on its latency.
template <bool MAX>
__device__ __forceinline__ float wave_reduce(float x) {
  x = dpp_step<0xB1, 0xF, MAX>(x);    // quad_perm 1, 0, 3, 2
  x = dpp_step<0x4E, 0xF, MAX>(x);    // quad_perm 2, 3, 0, 1
  x = dpp_step<0x141, 0xF, MAX>(x);   // row half mirror
  x = dpp_step<0x140, 0xF, MAX>(x);   // row mirror
  x = dpp_step<0x142, 0xA, MAX>(x);   // row broadcast 15 into rows 1 and 3
  x = dpp_step<0x143, 0xC, MAX>(x);   // row broadcast 31 into rows 2 and 3
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 63));
}

// The corner range of the whole wave chunk (NaN-free cells only).
__device__ __forceinline__ void wave_range(const WaveCells& w, float* lo, float* hi) {
  *lo = wave_reduce<false>(w.lo);
  *hi = wave_reduce<true>(w.hi);
}

// Segments of one isovalue in a wave chunk: a cell has segments iff
// min < iso <= max over its corners; it has two iff it is a saddle (case 5
// or 10: diagonal corners on one side, the other diagonal on the other),
// found on whole-wave masks.
__device__ __forceinline__ int64_t wave_segments(const WaveCells& w, float iso) {
  int64_t count = 0;
#pragma unroll
  for (int q = 0; q < kCellsPerLane; ++q) {
    const uint64_t ok = __ballot(w.clo[q] < iso && iso <= w.chi[q]);
    if (ok == 0) continue;
    const Corners& c = w.c[q];
    const uint64_t a0 = __ballot(c.v0 >= iso), a1 = __ballot(c.v1 >= iso);
    const uint64_t a2 = __ballot(c.v2 >= iso), a3 = __ballot(c.v3 >= iso);
    const uint64_t saddle = ok & ~(a0 ^ a2) & ~(a1 ^ a3) & (a0 ^ a1);
    count += __popcll(ok) + __popcll(saddle);
  }
  return count;
}

__global__ __launch_bounds__(64 * kWavesPerBlock) void contour_count_kernel(ContourParams p) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int d = (int)(blk / p.bpf);
  const int64_t chunk = (blk % p.bpf) * kWavesPerBlock + wave;
  if (chunk >= p.nchunk) return;   // whole wave; the kernel has no barrier
  const float* f = p.fields + (int64_t)d * p.W * p.H;
  // the first 64 isovalues, loaded in flight with the corner loads
  const float isov0 = lane < p.n_iso ? p.iso[d * p.n_iso + lane] : 0.0f;
  WaveCells w;
  load_wave_cells(p, f, chunk, lane, w);
  if (p.cases) {
    // with the case array every (isovalue, cell) is written: isovalues one
    // at a time, 64 per vector load, broadcast per iteration
    float isov = 0.0f;
    for (int k = 0; k < p.n_iso; ++k) {
      if ((k & 63) == 0) isov = (k + lane < p.n_iso) ? p.iso[d * p.n_iso + k + lane] : 0.0f;
      const float iso = __builtin_bit_cast(
          float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, isov), k & 63));
#pragma unroll
      for (int q = 0; q < kCellsPerLane; ++q)
        if (w.in[q])
          p.cases[((int64_t)d * p.n_iso + k) * p.cells + w.cell[q]] =
              (uint8_t)cell_case(w.c[q], iso);
      const int64_t count = wave_segments(w, iso);
      if (lane == 0) p.counts[((int64_t)d * p.n_iso + k) * p.nchunk + chunk] = (int32_t)count;
    }
    return;
  }
  // Isovalues 64 at a time, one per lane: the wave's corner range picks the
  // ones that can cross any of its cells (a ballot), only those are
  // counted, and each lane stores its isovalue's count (zero for the rest)
  // in one store.
  float wlo, whi;
  wave_range(w, &wlo, &whi);
  for (int k0 = 0; k0 < p.n_iso; k0 += 64) {
    const bool valid = k0 + lane < p.n_iso;
    const float isov = k0 == 0 ? isov0 : (valid ? p.iso[d * p.n_iso + k0 + lane] : 0.0f);
    uint64_t act = __ballot(valid && isov > wlo && isov <= whi);
    int32_t cnt = 0;
    while (act) {
      const int kk = __builtin_ctzll(act);
      act &= act - 1;
      const float iso = __builtin_bit_cast(
          float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, isov), kk));
      const int64_t count = wave_segments(w, iso);
      if (lane == kk) cnt = (int32_t)count;
    }
    if (valid) p.counts[((int64_t)d * p.n_iso + k0 + lane) * p.nchunk + chunk] = cnt;
  }
}

// First scan level: exclusive scan inside tiles of kScanTile entries (a
// tile holds at most kScanTile * 2 * kCellsPerWave segments, so int32
// offsets suffice).  `out` may alias `in`: every thread reads its four
// entries before it writes them.
__global__ __launch_bounds__(256) void scan_tiles_kernel(const int32_t* in, int32_t* out,
                                                         int64_t* tile_sums, int64_t n) {
  __shared__ int64_t wsum[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  int64_t v[4];
  int64_t s = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t idx = base + 4 * t + q;
    v[q] = idx < n ? (int64_t)in[idx] : 0;
    s += v[q];
  }
  int64_t incl = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t nb = __shfl_up(incl, o, 64);
    if (lane >= o) incl += nb;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int64_t wbase = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    if (w < wave) wbase += wsum[w];
    tot += wsum[w];
  }
  int64_t run = wbase + incl - s;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t idx = base + 4 * t + q;
    if (idx < n) out[idx] = (int32_t)run;
    run += v[q];
  }
  if (t == 0) tile_sums[blockIdx.x] = tot;
}

// Second level: one block scans the tile sums in place and writes the total.
__global__ __launch_bounds__(1024) void scan_sums_kernel(int64_t* sums, int64_t ntiles,
                                                         int64_t* total) {
  __shared__ int64_t wsum[16];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t per = (ntiles + 1023) / 1024;
  const int64_t lo = t * per, hi = lo + per < ntiles ? lo + per : ntiles;
  int64_t s = 0;
  for (int64_t q = lo; q < hi; ++q) s += sums[q];
  int64_t incl = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t nb = __shfl_up(incl, o, 64);
    if (lane >= o) incl += nb;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int64_t wbase = 0, tot = 0;
  for (int w = 0; w < 16; ++w) {
    if (w < wave) wbase += wsum[w];
    tot += wsum[w];
  }
  int64_t run = wbase + incl - s;
  for (int64_t q = lo; q < hi; ++q) {
    const int64_t v = sums[q];
    sums[q] = run;
    run += v;
  }
  if (t == 0) *total = tot;
}

// Emission is done in two steps so that the case and edge work runs on full
// waves: a contour crosses only a few of a chunk's 256 cells per isovalue,
// and working through them where they lie would keep one or two lanes of 64
// busy.  Per isovalue, each crossed cell's output slot is found (the
// chunk's scanned offset plus the ballot prefix of the cells before it) and
// the cell is queued in LDS with its corners and slot; whenever the queue
// might not take another 64 cells, and at the end, the wave drains it, one
// queued cell per lane.  The queue is private to its wave (no barriers).
constexpr int kQueue = 128;   // queued cells per wave

struct QueuedCell {
  float4 c;        // corners v0..v3
  int64_t o;       // output slot of the cell's first segment
  int32_t k;       // isovalue index
  int32_t slot;    // cell within the chunk (q * 64 + lane)
  int32_t i, j;    // row and column
};

struct EmitLds {
  QueuedCell q[kWavesPerBlock][kQueue];
};

// Orders this wave's LDS writes before the reads that follow (LDS requests
// of one wave complete in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Write the segments of the n queued cells, one cell per lane.
__device__ __forceinline__ void drain_queue(const ContourParams& p, EmitLds& L, int wave, int d,
                                            int64_t chunk, int n, int lane) {
  wave_lds_sync();
  for (int e = lane; e < n; e += 64) {
    const QueuedCell qc = L.q[wave][e];
    const Corners cq{qc.c.x, qc.c.y, qc.c.z, qc.c.w, true};
    const float iso = p.iso[d * p.n_iso + qc.k];
    int a0, a1, b0, b1;
    const int ns = case_segments(cell_case(cq, iso), cq, iso, a0, a1, b0, b1);
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
      const int64_t o = qc.o + s2;
      if (s2 < ns && o < p.capacity) {
        float x0, y0, x1, y1;
        edge_point(s2 ? b0 : a0, cq, iso, qc.i, qc.j, p.g, &x0, &y0);
        edge_point(s2 ? b1 : a1, cq, iso, qc.i, qc.j, p.g, &x1, &y1);
        reinterpret_cast<float4*>(p.segs)[o] = make_float4(x0, y0, x1, y1);
        if (p.ids) {
          p.ids[3 * o] = d;
          p.ids[3 * o + 1] = qc.k;
          p.ids[3 * o + 2] = (int32_t)(chunk * kCellsPerWave + qc.slot);
        }
      }
    }
  }
  wave_lds_sync();
}

// Queue the crossed cells of isovalue k of field d in one wave chunk with
// the slots their segments take, in (cell, segment) order from the chunk's
// offset `run` on.  `nq` is the wave's queue length (the same in every
// lane).
__device__ __forceinline__ void queue_iso(const ContourParams& p, const WaveCells& w, EmitLds& L,
                                          int wave, int d, int k, float iso, int64_t chunk,
                                          int64_t run, uint64_t below, int lane, int& nq) {
#pragma unroll
  for (int q = 0; q < kCellsPerLane; ++q) {
    // cells of this group with one segment or more, and the saddles among
    // them (two segments), as whole-wave masks, as in the count pass.  A
    // group no lane's cell crosses has nothing to queue.
    const Corners cq = w.c[q];
    const bool has = w.clo[q] < iso && iso <= w.chi[q];
    const uint64_t one = __ballot(has);
    if (one == 0) continue;
    const uint64_t m0 = __ballot(cq.v0 >= iso), m1 = __ballot(cq.v1 >= iso);
    const uint64_t m2 = __ballot(cq.v2 >= iso), m3 = __ballot(cq.v3 >= iso);
    const uint64_t two = one & ~(m0 ^ m2) & ~(m1 ^ m3) & (m0 ^ m1);
    if (nq > kQueue - 64) {
      drain_queue(p, L, wave, d, chunk, nq, lane);
      nq = 0;
    }
    if (has) {
      QueuedCell qc;
      qc.c = make_float4(cq.v0, cq.v1, cq.v2, cq.v3);
      qc.o = run + __popcll(one & below) + __popcll(two & below);
      qc.k = k;
      qc.slot = q * 64 + lane;
      qc.i = w.i[q];
      qc.j = w.j[q];
      L.q[wave][nq + __popcll(one & below)] = qc;
    }
    nq += __popcll(one);
    run += __popcll(one) + __popcll(two);
  }
}

// five waves per SIMD (at most 96 registers): the pass waits on memory
__global__ __launch_bounds__(64 * kWavesPerBlock) __attribute__((amdgpu_waves_per_eu(5)))
void contour_emit_kernel(ContourParams p) {
  __shared__ EmitLds lds;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int d = (int)(blk / p.bpf);
  const int64_t chunk = (blk % p.bpf) * kWavesPerBlock + wave;
  if (chunk >= p.nchunk) return;   // whole wave; the kernel has no barrier
  const float* f = p.fields + (int64_t)d * p.W * p.H;
  // isovalues 64 at a time, one per lane, with the chunk's output offset of
  // each; the first 64 are loaded here, in flight with the corner loads, so
  // that the wave waits once for all of them
  auto iso_batch = [&](int k0, float& isov, int32_t& off, int64_t& pre) {
    isov = 0.0f;
    off = 0;
    pre = 0;
    if (k0 + lane < p.n_iso) {
      const int64_t slot = ((int64_t)d * p.n_iso + k0 + lane) * p.nchunk + chunk;
      isov = p.iso[d * p.n_iso + k0 + lane];
      off = p.offsets[slot];
      pre = p.tile_prefix[slot / kScanTile];
    }
  };
  float isov0;
  int32_t off0;
  int64_t pre0;
  iso_batch(0, isov0, off0, pre0);
  WaveCells w;
  load_wave_cells(p, f, chunk, lane, w);
  const uint64_t below = (1ull << lane) - 1ull;   // lanes before this one
  int nq = 0;
  // only the isovalues inside the wave's corner range can have segments
  // here (as in the count pass)
  float wlo, whi;
  wave_range(w, &wlo, &whi);
  for (int k0 = 0; k0 < p.n_iso; k0 += 64) {
    float isov = isov0;
    int32_t offk = off0;
    int64_t pre = pre0;
    if (k0 > 0) iso_batch(k0, isov, offk, pre);
    const int64_t off = pre + offk;
    const bool valid = k0 + lane < p.n_iso;
    uint64_t act = __ballot(valid && isov > wlo && isov <= whi);
    while (act) {
      const int kk = __builtin_ctzll(act);
      act &= act - 1;
      const float iso = __builtin_bit_cast(
          float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, isov), kk));
      const uint64_t ou = (uint64_t)off;
      const int64_t run = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(
                                         (int)(uint32_t)(ou >> 32), kk) << 32) |
                                    (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)ou, kk));
      queue_iso(p, w, lds, wave, d, k0 + kk, iso, chunk, run, below, lane, nq);
    }
  }
  if (nq > 0) drain_queue(p, lds, wave, d, chunk, nq, lane);
}

// Fixed scratch of the allocation-free contour entry point: counts,
// offsets and tile sums of one call, MLS_CONTOUR_STATIC_SCRATCH_BYTES in
// all.  Each device holds its own copy for the life of the process.  In
// host code the name stands for a host-side handle only: kernels get the
// device address that contour_static_scratch_resolve() looks up.
static __device__ __align__(256) char scratch[MLS_CONTOUR_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

hipError_t contour_static_scratch_resolve(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* contour_static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  return g_scratch_ptr[device];
}

int64_t contour_scratch_entries(int32_t D, int32_t n_iso, int32_t W, int32_t H) {
  const int64_t cells = (int64_t)(W - 1) * (H - 1);
  const int64_t nchunk = (cells + kCellsPerWave - 1) / kCellsPerWave;
  return (int64_t)D * n_iso * nchunk;
}

int64_t contour_scan_tiles(int64_t entries) { return (entries + kScanTile - 1) / kScanTile; }

hipError_t launch_contour(const ContourArgs& a, hipStream_t s) {
  ContourParams p;
  p.fields = a.fields;
  p.iso = a.iso;
  p.D = a.D;
  p.n_iso = a.n_iso;
  p.W = a.W;
  p.H = a.H;
  p.cells = (int64_t)(a.W - 1) * (a.H - 1);
  p.nchunk = (p.cells + kCellsPerWave - 1) / kCellsPerWave;
  p.bpf = (p.nchunk + kWavesPerBlock - 1) / kWavesPerBlock;
  p.cases = a.cases;
  p.counts = a.counts;
  p.offsets = a.offsets;
  p.tile_prefix = a.tile_sums;
  p.segs = a.segs;
  p.ids = a.ids;
  p.capacity = a.capacity;
  p.g = GridD{a.x0, a.y0, a.dx, a.dy};
  const int64_t blocks = (int64_t)a.D * p.bpf;
  const int64_t entries = (int64_t)a.D * p.nchunk * a.n_iso;
  const int64_t tiles = contour_scan_tiles(entries);
  hipLaunchKernelGGL(contour_count_kernel, dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0,
                     s, p);
  hipLaunchKernelGGL(scan_tiles_kernel, dim3((unsigned)tiles), dim3(256), 0, s, a.counts,
                     a.offsets, a.tile_sums, entries);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, s, a.tile_sums, tiles, a.total);
  if (a.capacity > 0)
    hipLaunchKernelGGL(contour_emit_kernel, dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), 0,
                       s, p);
  return hipGetLastError();
}

}  // namespace mls
