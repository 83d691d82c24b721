// 16-bit matrix-core MLS fit for gfx950 (Muelder et al., Sec. 3.3): the
// weight x feature contraction on v_mfma_f32_16x16x32_{bf16,f16} with
// float32 accumulation, followed by the float64 per-node solve.
//
// Precision design.  The normal equations amplify relative errors of the
// moments by the conditioning of the weighted basis, and a single 16-bit
// rounding of each feature (8 or 11 significant bits) is far too coarse for
// the quadratic basis.  So
//   - every feature g (moment monomial or basis x attribute) is carried as
//     an S-term expansion g = g_1 + ... + g_S of 16-bit numbers (each term
//     the rounding of what the previous terms left), and the contraction
//     issues one MFMA per term into the same float32 accumulator: the
//     products are exact, the accumulator holds about 24 bits;
//   - the weight w(node, point) is rounded once and the same rounded weight
//     multiplies every feature of that pair, so the result is the exact MLS
//     fit for slightly perturbed weights (MLS reproduces its basis for any
//     positive weights);
//   - attributes are staged in [-1, 1] (mls_stage.hip) and mapped back.
//
// Work split.  A workgroup (4 waves) owns a 16 x 16 node tile and one slab
// of attributes: the slab's features are the moment monomials plus
// basis x attribute products for its D_s attributes, at most 16 NTS
// columns, so the per-node accumulators fit in registers (each wave: 4 row
// strips x NTS feature tiles of 16 x 16 float32).  Every slab repeats the
// moments, which lets each slab solve its own nodes.  Points stream through
// double-buffered LDS in chunks of 32 (one MFMA k-step): Gaussian factors
// gx[col][k], gy[row][k] in float32, and the feature terms
// G[s][j][k] in 16 bits; while the MFMAs of one chunk run the workgroup
// fills the next chunk into the other buffer.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mls_internal.h"
#include "mls_solve.h"

namespace mls {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;
constexpr int kWaves = 4;
constexpr int kCols = 16;
constexpr int R = 4;                  // row strips per wave
constexpr int kRows = kWaves * R;     // 16
constexpr int KT = 32;                // points per chunk (one MFMA k-step)
constexpr int KSF = KT + 4;           // float32 table stride (floats)
constexpr int KSH = KT + 8;           // 16-bit feature stride (elements; 80 B rows)
constexpr int kEpiWaves = 2;

template <typename T> struct Vec8;
template <> struct Vec8<__bf16> { typedef bf16x8 type; };
template <> struct Vec8<_Float16> { typedef halfx8 type; };

__device__ __forceinline__ floatx4 mfma16(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma16(halfx8 a, halfx8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

struct LPParams {
  const float* pts;       // [n][2]
  const float* vals_t;    // [D][n] staged attributes in [-1, 1]
  const float* shift;     // [D]
  const float* scale;     // [D]
  int64_t n;
  int D, Ds, nslab, F;    // F = features of a full slab
  float inv_h;
  double inv_hd;
  double x0, y0, dx, dy;
  int W, H, tiles_x, tiles;
  double tau, floor_w;
  float cutoff2;          // points whose u^2 exceeds this for every node get no weight
  float* fields;
  uint8_t* deg_out;
  // compact support: points (and vals_t) in cell order, cell offsets, tiles
  // in the order to run them
  const uint32_t* cell_start;
  const uint32_t* torder;
  int ncx, ncy;
  CellGeom geom;
};

// Chunks of at most KT consecutive points: all points (dense), or the runs
// of cells that a tile's support can reach, one cell row at a time.
struct ChunkCursor {
  int64_t k, kend;   // current chunk starts at k; its run ends at kend
  int cy, cy1;       // cell row of the run, last cell row
  bool done;
};

template <bool CELLS>
__device__ __forceinline__ void cursor_row(const LPParams& p, ChunkCursor& cu, int cx0, int cx1) {
  // advance to the next non-empty run at or after row cu.cy
  while (cu.cy <= cu.cy1) {
    const int64_t a = p.cell_start[cu.cy * p.ncx + cx0];
    const int64_t b = p.cell_start[cu.cy * p.ncx + cx1 + 1];
    if (b > a) {
      cu.k = a;
      cu.kend = b;
      return;
    }
    ++cu.cy;
  }
  cu.done = true;
}

template <bool CELLS>
__device__ __forceinline__ ChunkCursor cursor_begin(const LPParams& p, int cx0, int cx1, int cy0,
                                                    int cy1) {
  ChunkCursor cu;
  cu.done = false;
  if (!CELLS) {
    cu.k = 0;
    cu.kend = p.n;
    cu.cy = 0;
    cu.cy1 = 0;
    return cu;
  }
  cu.cy = cy0;
  cu.cy1 = cy1;
  cursor_row<CELLS>(p, cu, cx0, cx1);
  return cu;
}

template <bool CELLS>
__device__ __forceinline__ void cursor_next(const LPParams& p, ChunkCursor& cu, int cx0, int cx1) {
  cu.k += KT;
  if (cu.k < cu.kend) return;
  if (!CELLS) {
    cu.done = true;
    return;
  }
  ++cu.cy;
  cursor_row<CELLS>(p, cu, cx0, cx1);
}

template <int DEG, int NTS, int S, typename T>
struct LPLayout {
  static constexpr int kFP = NTS * 16;
  static constexpr int kGxB = 0;                                   // [16][KSF] float
  static constexpr int kGyB = kGxB + kCols * KSF * 4;              // [16][KSF] float
  static constexpr int kGB = kGyB + kRows * KSF * 4;               // [S][kFP][KSH] T
  static constexpr int kBuf = kGB + S * kFP * KSH * 2;             // bytes, one buffer
  static constexpr int kEpiStride = kFP + 1;                       // floats
  static constexpr int kEpi = kEpiWaves * 16 * R * kEpiStride * 4;  // bytes
  static constexpr int kBytes = 2 * kBuf > kEpi ? 2 * kBuf : kEpi;
};

// Split v into S 16-bit terms (each the rounding of the remainder).
template <int S, typename T>
__device__ __forceinline__ void split_terms(float v, T* out) {
  float r = v;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const T t = (T)r;
    out[s] = t;
    r = r - (float)t;
  }
}

// Fill one chunk buffer: Gaussian factors and the slab's feature terms for
// points [k0, k0 + KT).  Points past n, and points farther than the cutoff
// from every node of the tile, get zero weight and zero features.
// Offset of node column c0 + col (row r0 + row) from the tile anchor, in
// units of h, computed in float64 from the grid definition.
__device__ __forceinline__ double node_offset_xd(const LPParams& p, int c0, int col, float cxr) {
  return (p.x0 + (double)(c0 + col) * p.dx - (double)cxr) * p.inv_hd;
}
__device__ __forceinline__ double node_offset_yd(const LPParams& p, int r0, int row, float cyr) {
  return (p.y0 + (double)(r0 + row) * p.dy - (double)cyr) * p.inv_hd;
}
__device__ __forceinline__ float node_offset_x(const LPParams& p, int c0, int col, float cxr) {
  return (float)node_offset_xd(p, c0, col, cxr);
}
__device__ __forceinline__ float node_offset_y(const LPParams& p, int r0, int row, float cyr) {
  return (float)node_offset_yd(p, r0, row, cyr);
}

template <int DEG, int NTS, int S, typename T, bool WEND>
__device__ __forceinline__ void stage_chunk(const LPParams& p, char* buf, int64_t k0, int64_t kend,
                                            int slab, int tid, int c0, int r0, float cxr,
                                            float cyr) {
  using L = LPLayout<DEG, NTS, S, T>;
  constexpr int m = DEG == 0 ? 1 : (DEG == 1 ? 3 : 6);
  constexpr int nmom = DEG == 0 ? 1 : (DEG == 1 ? 6 : 15);
  float* gx = (float*)(buf + L::kGxB);
  float* gy = (float*)(buf + L::kGyB);
  T* G = (T*)(buf + L::kGB);
  // Gaussian factors: 32 rows (16 columns, 16 rows) x 32 points = 4 per thread
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int e = tid + it * kThreads;
    const int k = e & (KT - 1), row = e >> 5;
    const int64_t gi = k0 + k;
    // Gaussian: the separable factor exp(-u^2); Wendland: u^2, combined per
    // pair when the A operand is built.  Points past the run: Gaussian 0,
    // Wendland a distance beyond the support.
    float v = WEND ? 4.0f : 0.0f;
    if (gi < kend) {
      float u;
      if (row < kCols) u = (p.pts[2 * gi] - cxr) * p.inv_h - node_offset_x(p, c0, row, cxr);
      else u = (p.pts[2 * gi + 1] - cyr) * p.inv_h - node_offset_y(p, r0, row - kCols, cyr);
      v = WEND ? u * u : __expf(-u * u);
    }
    if (row < kCols) gx[row * KSF + k] = v;
    else gy[(row - kCols) * KSF + k] = v;
  }
  // features: items (feature j, point pair) -> S packed 32-bit writes
  const int d0 = slab * p.Ds;
  const int Ds = min(p.Ds, p.D - d0);
  const int F = nmom + m * Ds;
  for (int e = tid; e < L::kFP * (KT / 2); e += kThreads) {
    const int kp = (e & (KT / 2 - 1)) * 2, j = e / (KT / 2);
    float v[2] = {0.0f, 0.0f};
#pragma unroll
    for (int h2 = 0; h2 < 2; ++h2) {
      const int64_t gi = k0 + kp + h2;
      if (gi < kend && j < F) {
        const float ux = (p.pts[2 * gi] - cxr) * p.inv_h;
        const float uy = (p.pts[2 * gi + 1] - cyr) * p.inv_h;
        if (ux * ux + uy * uy <= p.cutoff2) {
          if (j < nmom) {
            int t = 0;
            while ((t + 1) * (t + 2) / 2 <= j) ++t;
            const int b = j - t * (t + 1) / 2, a = t - b;
            float w = 1.0f;
            for (int q = 0; q < a; ++q) w *= ux;
            for (int q = 0; q < b; ++q) w *= uy;
            v[h2] = w;
          } else {
            const int jj = j - nmom;
            const int bj = jj / Ds, d = jj - bj * Ds;
            const float f = p.vals_t[(int64_t)(d0 + d) * p.n + gi];
            float bv = 1.0f;
            if (bj == 1) bv = ux;
            else if (bj == 2) bv = uy;
            else if (bj == 3) bv = ux * ux;
            else if (bj == 4) bv = ux * uy;
            else if (bj == 5) bv = uy * uy;
            v[h2] = bv * f;
          }
        }
      }
    }
    T t0[S], t1[S];
    split_terms<S, T>(v[0], t0);
    split_terms<S, T>(v[1], t1);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      T* dst = G + ((size_t)s * L::kFP + j) * KSH + kp;
      dst[0] = t0[s];
      dst[1] = t1[s];
    }
  }
}

template <int DEG, int R_, typename Acc>
__device__ void solve_tile_nodes_lp(const LPParams& p, const Acc* epi, int stride, int lane,
                                    int wave, int r0, int c0, int slab, int64_t plane,
                                    float cxr, float cyr) {
  const int d0 = slab * p.Ds;
  const int Ds = min(p.Ds, p.D - d0);
  for (int node = lane; node < 16 * R_; node += 64) {
    const int t = node / 16, col = node % 16;
    const int r = r0 + wave * R_ + t, c = c0 + col;
    if (r >= p.H || c >= p.W) continue;
    const double ex = node_offset_xd(p, c0, col, cxr);
    const double ey = node_offset_yd(p, r0, wave * R_ + t, cyr);
    const int64_t off = (int64_t)r * p.W + c;
    uint8_t code = solve_node<DEG, Acc>(epi + node * stride, Ds, ex, ey, p.tau, p.floor_w,
                                        p.fields + (int64_t)d0 * plane + off, plane,
                                        p.shift + d0, p.scale + d0);
    if (p.deg_out && slab == 0) p.deg_out[off] = code;
  }
}

// Wendland C2 weight (1 - s)^4 (4 s + 1) for s = r / h < 1.
__device__ __forceinline__ float wendland_c2(float s2) {
  const float s = __builtin_sqrtf(s2);
  const float t = 1.0f - s;
  const float t2 = t * t;
  return s < 1.0f ? t2 * t2 * (4.0f * s + 1.0f) : 0.0f;
}

template <int DEG, int NTS, int S, typename T, bool WEND, bool CELLS>
__global__ __launch_bounds__(kThreads, 2) void fit_lp_kernel(LPParams p) {
  using L = LPLayout<DEG, NTS, S, T>;
  typedef typename Vec8<T>::type vec8;
  extern __shared__ __attribute__((aligned(16))) char lds_lp[];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int slab = blockIdx.x / p.tiles;
  const int tile = CELLS ? (int)p.torder[blockIdx.x % p.tiles] : (int)(blockIdx.x % p.tiles);
  const int c0 = (tile % p.tiles_x) * kCols;
  const int r0 = (tile / p.tiles_x) * kRows;
  // tile anchor (rounded to float32: the frame only has to be close to the
  // tile, the offsets below are taken in the same float32 frame)
  const float cxr = (float)(p.x0 + (double)(c0 + kCols / 2) * p.dx);
  const float cyr = (float)(p.y0 + (double)(r0 + kRows / 2) * p.dy);
  int cx0 = 0, cx1 = 0, cy0 = 0, cy1 = 0;
  if (CELLS) tile_cell_range(p.geom, tile % p.tiles_x, tile / p.tiles_x, p.ncx, p.ncy, &cx0, &cx1,
                             &cy0, &cy1);

  floatx4 acc[R][NTS];
#pragma unroll
  for (int t = 0; t < R; ++t)
#pragma unroll
    for (int q = 0; q < NTS; ++q) acc[t][q] = floatx4{0.f, 0.f, 0.f, 0.f};

  ChunkCursor cu = cursor_begin<CELLS>(p, cx0, cx1, cy0, cy1);
  if (!cu.done)
    stage_chunk<DEG, NTS, S, T, WEND>(p, lds_lp, cu.k, cu.kend, slab, tid, c0, r0, cxr, cyr);
  __syncthreads();

  const int i = lane & 15;
  const int k8 = (lane >> 4) * 8;   // this lane's 8 points of the 32
  int c = 0;
  while (!cu.done) {
    const char* cur = lds_lp + (c & 1) * L::kBuf;
    char* nxt = lds_lp + ((c & 1) ^ 1) * L::kBuf;
    const float* gx = (const float*)(cur + L::kGxB);
    const float* gy = (const float*)(cur + L::kGyB);
    const T* G = (const T*)(cur + L::kGB);
    // A operands: weights of the wave's 4 row strips x the lane's 8 points
    float wx[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) wx[q] = gx[i * KSF + k8 + q];
    vec8 a[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const float* gyr = gy + (wave * R + t) * KSF + k8;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        a[t][q] = (T)(WEND ? wendland_c2(wx[q] + gyr[q]) : wx[q] * gyr[q]);
    }
#pragma unroll
    for (int q = 0; q < NTS; ++q) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const vec8 b = *(const vec8*)(G + ((size_t)s * L::kFP + q * 16 + i) * KSH + k8);
#pragma unroll
        for (int t = 0; t < R; ++t) acc[t][q] = mfma16(a[t], b, acc[t][q]);
      }
    }
    cursor_next<CELLS>(p, cu, cx0, cx1);
    if (!cu.done)
      stage_chunk<DEG, NTS, S, T, WEND>(p, nxt, cu.k, cu.kend, slab, tid, c0, r0, cxr, cyr);
    __syncthreads();
    ++c;
  }

  // Epilogue: accumulators -> LDS [node][feature] (float32) -> solve.
  const int64_t plane = (int64_t)p.W * p.H;
  float* epi_all = (float*)lds_lp;
#pragma unroll 1
  for (int g = 0; g < kWaves; g += kEpiWaves) {
    const bool mine = wave >= g && wave < g + kEpiWaves;
    float* epi = epi_all + (wave - g) * 16 * R * L::kEpiStride;
    if (mine) {
#pragma unroll
      for (int t = 0; t < R; ++t)
#pragma unroll
        for (int q = 0; q < NTS; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            // f32 16x16 MFMA result: lane holds row 4 (lane/16) + r, column lane%16
            const int node = t * 16 + 4 * (lane >> 4) + r;
            const int feat = q * 16 + (lane & 15);
            epi[node * L::kEpiStride + feat] = acc[t][q][r];
          }
    }
    __syncthreads();
    if (mine)
      solve_tile_nodes_lp<DEG, R, float>(p, epi, L::kEpiStride, lane, wave, r0, c0, slab, plane,
                                         cxr, cyr);
    __syncthreads();
  }
}

template <int DEG, int NTS, int S, typename T, bool WEND>
hipError_t launch_lp_impl(LPParams p, hipStream_t s) {
  using L = LPLayout<DEG, NTS, S, T>;
  const size_t lds = (size_t)L::kBytes;
  // Wendland weights always walk the cell list; the Gaussian runs dense
  const void* fn = WEND ? (const void*)fit_lp_kernel<DEG, NTS, S, T, true, true>
                        : (const void*)fit_lp_kernel<DEG, NTS, S, T, false, false>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int64_t blocks = (int64_t)p.tiles * p.nslab;
  if (WEND)
    hipLaunchKernelGGL((fit_lp_kernel<DEG, NTS, S, T, true, true>), dim3((unsigned)blocks),
                       dim3(kThreads), lds, s, p);
  else
    hipLaunchKernelGGL((fit_lp_kernel<DEG, NTS, S, T, false, false>), dim3((unsigned)blocks),
                       dim3(kThreads), lds, s, p);
  return hipGetLastError();
}

template <int DEG, int S, typename T, bool WEND>
hipError_t launch_lp_nts(const LPParams& p, int nts, hipStream_t s) {
  switch (nts) {
    case 1: return launch_lp_impl<DEG, 1, S, T, WEND>(p, s);
    case 2: return launch_lp_impl<DEG, 2, S, T, WEND>(p, s);
    case 3: return launch_lp_impl<DEG, 3, S, T, WEND>(p, s);
    case 4: return launch_lp_impl<DEG, 4, S, T, WEND>(p, s);
    case 5: return launch_lp_impl<DEG, 5, S, T, WEND>(p, s);
    case 6: return launch_lp_impl<DEG, 6, S, T, WEND>(p, s);
    case 7: return launch_lp_impl<DEG, 7, S, T, WEND>(p, s);
    default: return launch_lp_impl<DEG, 8, S, T, WEND>(p, s);
  }
}

template <int S, typename T, bool WEND>
hipError_t launch_lp_deg(const LPParams& p, int deg, int nts, hipStream_t s) {
  switch (deg) {
    case 0: return launch_lp_nts<0, S, T, WEND>(p, nts, s);
    case 1: return launch_lp_nts<1, S, T, WEND>(p, nts, s);
    default: return launch_lp_nts<2, S, T, WEND>(p, nts, s);
  }
}

template <typename T, bool WEND>
hipError_t launch_lp_terms(const LPParams& p, int deg, int nts, int terms, hipStream_t s) {
  switch (terms) {
    case 1: return launch_lp_deg<1, T, WEND>(p, deg, nts, s);
    case 2: return launch_lp_deg<2, T, WEND>(p, deg, nts, s);
    default: return launch_lp_deg<3, T, WEND>(p, deg, nts, s);
  }
}

}  // namespace

// Slab plan: feature tiles per slab (1..8) and attributes per slab that cover
// D with the fewest padded columns in total.
void lp_slab_plan(int degree, int D, int* nts_out, int* ds_out, int* nslab_out) {
  const int m = basis_terms(degree), nmom = moment_terms(degree);
  int best_cost = 1 << 30, best_nts = 8, best_ds = 1, best_ns = D;
  for (int nts = 1; nts <= 8; ++nts) {
    const int ds = (nts * 16 - nmom) / m;
    if (ds < 1) continue;
    const int dsu = ds < D ? ds : D;
    const int ns = (D + dsu - 1) / dsu;
    const int cost = ns * nts;
    if (cost < best_cost || (cost == best_cost && nts > best_nts)) {
      best_cost = cost;
      best_nts = nts;
      best_ds = dsu;
      best_ns = ns;
    }
  }
  // the smallest tile count that still holds best_ds attributes
  int nts = 1;
  while (nts * 16 < nmom + m * best_ds) ++nts;
  *nts_out = nts;
  *ds_out = best_ds;
  *nslab_out = best_ns;
}

hipError_t launch_fit_lp(const FitArgs& a, const float* vals_t, const float* shift,
                         const float* scale, bool fp16, int terms, const LPCells* cells,
                         hipStream_t stream) {
  int nts, ds, nslab;
  lp_slab_plan(a.degree, a.D, &nts, &ds, &nslab);
  LPParams p;
  p.pts = a.pts;
  p.vals_t = vals_t;
  p.shift = shift;
  p.scale = scale;
  p.n = a.n;
  p.D = a.D;
  p.Ds = ds;
  p.nslab = nslab;
  p.F = moment_terms(a.degree) + basis_terms(a.degree) * ds;
  p.inv_hd = 1.0 / a.h;
  p.inv_h = (float)p.inv_hd;
  p.x0 = a.x0; p.y0 = a.y0; p.dx = a.dx; p.dy = a.dy;
  p.W = a.W; p.H = a.H;
  p.tiles_x = (a.W + kCols - 1) / kCols;
  p.tiles = p.tiles_x * ((a.H + kRows - 1) / kRows);
  p.tau = a.tau;
  p.floor_w = a.floor_w;
  // weight below exp(-64) ~ 1.6e-28 at every node of the tile: the tile
  // spans at most half its diagonal from the anchor
  const double sxd = a.dx / a.h, syd = a.dy / a.h;
  const double half = 0.5 * sqrt((double)(kCols * kCols) * sxd * sxd +
                                 (double)(kRows * kRows) * syd * syd);
  const double reach = 8.0 + half;
  p.cutoff2 = (float)(reach * reach);
  p.fields = a.fields;
  p.deg_out = a.deg_out;
  p.cell_start = nullptr;
  p.torder = nullptr;
  p.ncx = p.ncy = 0;
  p.geom = CellGeom{0, 0, 1, a.x0, a.y0, a.dx, a.dy, a.h};
  const bool wend = a.wkind == 1;
  if (wend) {
    if (!cells) return hipErrorInvalidValue;
    p.pts = cells->pts_s;
    p.vals_t = cells->vals_ts;
    p.cell_start = cells->cell_start;
    p.torder = cells->torder;
    p.ncx = cells->ncx;
    p.ncy = cells->ncy;
    p.geom = cells->geom;
    return fp16 ? launch_lp_terms<_Float16, true>(p, a.degree, nts, terms, stream)
                : launch_lp_terms<__bf16, true>(p, a.degree, nts, terms, stream);
  }
  return fp16 ? launch_lp_terms<_Float16, false>(p, a.degree, nts, terms, stream)
              : launch_lp_terms<__bf16, false>(p, a.degree, nts, terms, stream);
}

}  // namespace mls
