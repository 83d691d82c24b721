// Float64 matrix-core MLS fit for gfx950 (Muelder et al., Sec. 3.3).
//
// Per node p the fit needs the weighted moments of the basis and of
// basis x attribute products, G_p = sum_i w(p, x_i) g_i with
//   g_i = [u_x^a u_y^b (a + b <= 2 deg) | b_j(u_i) f_{i,d}]   (F features)
// in a tile frame u = (x_i - c_T) / h.  Over a tile of nodes this is the
// product W (nodes x points) . G (points x F): a dense contraction, run here
// on v_mfma_f64_16x16x4f64 with the point index as the reduction dimension.
//
// Workgroup: 256 threads (4 waves) own a tile of 16 columns x 4R rows of
// nodes.  Each wave owns R row-strips of 16 nodes (one MFMA M-tile each) and
// all NT = ceil(F / 16) feature N-tiles, so a wave holds R * NT accumulator
// blocks.  Points stream through LDS in chunks of KT:
//   1. point coordinates -> LDS (tile-frame u, float64),
//   2. Gaussian weight factors gx[col][k] = exp(-((x_k - p_col)/h)^2) and
//      gy[row][k] (the Gaussian separates on a grid, so a tile needs
//      16 + 4R factors per point instead of 64R), and the feature block
//      G[j][k] in float64.  The factors are either copied from tables of
//      every grid column and row built once per launch (when they fit the
//      scratch cap) or generated per tile by a stepping recurrence; the
//      copy costs load and LDS instructions, which overlap the matrix
//      cores, where the recurrence costs vector instructions, which do not,
//   3. MFMA sweep: the A operand (node x point weight) is gx * gy, built in
//      registers; B is read from G.  Within each group of 16 points a lane
//      supplies points k0 + 4 (lane / 16) + j for MFMA j = 0..3, so it reads
//      four consecutive points with one 32-byte LDS access.
// After the last chunk the accumulators go through LDS to one node per
// lane, which runs the float64 degree-ladder solve (mls_solve.h) and stores
// the D fields and the degree code.  Every node sums its points in the same
// fixed order, so results are bit-reproducible run to run.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mls_internal.h"
#include "mls_solve.h"

namespace mls {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

#ifndef MLS_F64_KT
#define MLS_F64_KT 64
#endif
#ifndef MLS_F64_EPI_WAVES
#define MLS_F64_EPI_WAVES 2
#endif

constexpr int kThreads = 256;
constexpr int kWaves = 4;
constexpr int kCols = 16;      // node columns per tile (one M-tile)
constexpr int KT = MLS_F64_KT; // points per LDS chunk
#ifndef MLS_F64_PAD
#define MLS_F64_PAD 2
#endif
#ifndef MLS_F64_KG_UNROLL
#define MLS_F64_KG_UNROLL 1
#endif
#ifndef MLS_F64_SETPRIO
#define MLS_F64_SETPRIO 0
#endif
// LDS row stride in doubles.  A lane reads four consecutive doubles (two
// 16-byte reads) of row i = lane % 16; with a stride of KT + 2 = 66
// doubles (132 dwords, 4 mod 64) the sixteen rows of one read start in
// sixteen different 4-bank groups, so the reads are free of bank
// conflicts (a stride of 68 doubles puts rows i and i + 8 on the same
// banks).
constexpr int KS = KT + MLS_F64_PAD;
static_assert(KS % 2 == 0 && KT % 16 == 0, "rows must start on 16-byte boundaries");
// Waves that run the epilogue at the same time: the epilogue needs a
// [nodes][features] float64 staging area per wave, and sharing it keeps the
// kernel's LDS small enough for two workgroups per CU.
constexpr int kEpiWaves = MLS_F64_EPI_WAVES;

struct F64Params {
  const float* pts;
  const float* vals;
  // Gaussian factor tables (WM_TABLE kernels): rows [0, tab_cols) are the
  // grid columns, rows tab_cols + r the grid rows; tab_n points per row
  const double* tab;
  int64_t tab_n;
  int tab_cols;
  int64_t n;
  int D, F;
  double h, inv_h;
  double alpha;        // inverse-distance exponent (WM_INV kernels)
  double x0, y0, dx, dy;
  int W, H, tiles_x;
  double tau, floor_w;
  float* fields;
  uint8_t* deg_out;
  float* grads;        // [D][2][H][W] or null
  bool rigid;          // rigid map (EPI 2 kernels)
};

// Weight modes of the kernel: the Gaussian with per-tile factors from a
// stepping recurrence, the inverse-distance weight per pair (any exponent,
// or alpha = 1 and alpha = 2 through a reciprocal), the Gaussian with
// factors copied from per-launch tables.
constexpr int WM_GAUSS = 0, WM_INV = 1, WM_TABLE = 2, WM_INV1 = 3, WM_INV2 = 4;

template <int DEG, int NT, int R>
struct F64Layout {
  static constexpr int kRows = kWaves * R;
  static constexpr int kFP = NT * 16;                    // padded features
  static constexpr int m = DEG == 0 ? 1 : (DEG == 1 ? 3 : 6);
  static constexpr int nmom = DEG == 0 ? 1 : (DEG == 1 ? 6 : 15);
  // most attributes NT feature tiles can hold, and the per-thread registers
  // that hold one chunk of their values
  static constexpr int kDMax = (kFP - nmom) / m;
  static constexpr int kValRegs =
      kDMax > 0 ? (KT * kDMax + kThreads - 1) / kThreads : 1;
  // per-thread registers holding one chunk of table factors (16 + 4R rows)
  static constexpr int kTabRegs = ((kCols + kWaves * R) * KT + kThreads - 1) / kThreads;
  // chunk phase
  static constexpr int kUx = 0;                          // [KT] tile-frame u_x
  static constexpr int kUy = kUx + KT;                   // [KT]
  static constexpr int kGx = kUy + KT;                   // [16][KS]
  static constexpr int kGy = kGx + kCols * KS;           // [kRows][KS]
  static constexpr int kG = kGy + kRows * KS;            // [kFP][KS]
  static constexpr int kChunk = kG + kFP * KS;
  // epilogue phase: per solving wave [16R nodes][kFP + 1]
  static constexpr int kEpiStride = kFP + 1;
  static constexpr int kEpi = kEpiWaves * 16 * R * kEpiStride;
  static constexpr int kDoubles = kChunk > kEpi ? kChunk : kEpi;
};

template <int DEG, int R, int EPI>
__device__ void solve_tile_nodes(const F64Params& p, const double* epi, int stride, int lane,
                                 int wave, int r0, int c0, int rows, int64_t plane);

// Inverse-distance weight (Eq. 4) of a node-point offset (ox, oy) in units of
// h: (ox^2 + oy^2)^(-alpha).  log2 of r^2 is taken as its binary exponent
// plus the float32 log2 of its mantissa (so r^2 far outside float32's range
// keeps an exact exponent), and the power is rebuilt as 2^frac scaled by
// ldexp, so it cannot overflow float32 either; the relative error is that
// of the float32 exp2/log2 (about 1e-7), a common factor of all features of
// the pair.  Padding points carry an infinite offset and weigh 0.  A node on
// a point (r^2 = 0) gets the clamp's large finite weight; such nodes are
// overwritten by the exact-hit pass.
__device__ __forceinline__ double invpow_weight(double ox, double oy, double alpha) {
  const double r2 = ox * ox + oy * oy;
  if (!(r2 < 1e300)) return 0.0;
  int ex;
  const double mant = frexp(fmax(r2, 1e-300), &ex);
  const double l2 = (double)ex + (double)__log2f((float)mant);
  const double e = fmin(-alpha * l2, 1000.0);
  const double ip = floor(e);
  return ldexp((double)exp2f((float)(e - ip)), (int)ip);
}

// The same weight for alpha = 1 and alpha = 2: the float32 reciprocal of
// r^2 (about 1 ulp of float32, a common relative error of about 1e-7 per
// pair, as the general form's), squared in float64 for alpha = 2, at about
// half the vector instructions of the float64 reciprocal with its Newton
// steps.  Padding points (infinite offset) get 1 / inf = 0; r^2 below
// float32's smallest normal number is clamped there, so a node on a point
// gets a large finite weight, as in the general form.
template <int ALPHA>
__device__ __forceinline__ double invpow_weight_int(double ox, double oy) {
  const double r2 = ox * ox + oy * oy;
  const double r = (double)__builtin_amdgcn_rcpf(fmaxf((float)r2, 0x1p-126f));
  return ALPHA == 1 ? r : r * r;
}

__device__ __forceinline__ void read4(const double* src, double* dst) {
  const double2* v = reinterpret_cast<const double2*>(src);
  const double2 lo = v[0], hi = v[1];
  dst[0] = lo.x;
  dst[1] = lo.y;
  dst[2] = hi.x;
  dst[3] = hi.y;
}

// Epilogue EPI: 0 fields, 1 fields and the slopes of the local fits (the
// extra solves raise the epilogue's register count, so they are separate
// instantiations and the plain kernels keep two workgroups per CU), 2 the
// rigid map of 2-vector values from the linear moments.
//
// Q4 > 0 (one feature tile, F <= 4 Q4 <= 12): the contraction runs on the
// four-block 4x4x4 FP64 MFMA instead of the 16x16x4 one.  Block b of that
// instruction takes nodes 4b .. 4b + 3, the same four points k and four
// feature columns c: lane l holds A (node l % 16, point l / 16) exactly as
// the 16x16x4 instruction takes it, B (point l / 16, feature l % 4, the
// same in every block) and the result for node 4 ((l / 4) % 4) + l / 16 and
// feature l % 4.  Each instruction covers the same 64 node-point pairs over
// 4 feature columns instead of 16, at about a quarter of the cycles, so the
// small shapes (Mean MLS F = 3, Affine and Rigid MLS F = 12) issue one to
// three short instructions where the 16x16x4 one carries 4 to 13 empty
// columns.
template <int DEG, int NT, int R, int WM, int EPI, int Q4 = 0>
__global__ __launch_bounds__(kThreads) void fit_f64_kernel(F64Params p) {
  static_assert(Q4 == 0 || NT == 1, "the 4x4x4 form covers one feature tile");
  constexpr bool INV = WM == WM_INV || WM == WM_INV1 || WM == WM_INV2;
  using L = F64Layout<DEG, NT, R>;
  constexpr int m = DEG == 0 ? 1 : (DEG == 1 ? 3 : 6);
  constexpr int nmom = DEG == 0 ? 1 : (DEG == 1 ? 6 : 15);
  extern __shared__ double lds[];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int tile_c = blockIdx.x % p.tiles_x;
  const int tile_r = blockIdx.x / p.tiles_x;
  const int c0 = tile_c * kCols;
  const int r0 = tile_r * L::kRows;
  // tile anchor: the node at the tile's centre (may lie beyond the grid)
  const double cx = p.x0 + (double)(c0 + kCols / 2) * p.dx;
  const double cy = p.y0 + (double)(r0 + L::kRows / 2) * p.dy;

  double* ux = lds + L::kUx;
  double* uy = lds + L::kUy;
  double* gx = lds + L::kGx;
  double* gy = lds + L::kGy;
  double* G = lds + L::kG;

  doublex4 acc[R][NT];
  double acc4[R][Q4 > 0 ? Q4 : 1];
#pragma unroll
  for (int t = 0; t < R; ++t) {
#pragma unroll
    for (int q = 0; q < NT; ++q) acc[t][q] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < (Q4 > 0 ? Q4 : 1); ++q) acc4[t][q] = 0.0;
  }

  const int D = p.D, F = p.F;
  // padding features stay zero for the whole kernel
  for (int e = tid; e < (L::kFP - F) * KS; e += kThreads) G[F * KS + e] = 0.0;

  // Raw chunk data is prefetched into registers one chunk ahead, so that
  // the global-memory latency overlaps the previous chunk's MFMA sweep.
  float pf_x = 0.0f, pf_y = 0.0f;
  float pf_v[L::kValRegs];
  auto prefetch = [&](int64_t k0) {
    const int kn = (int)((p.n - k0) < KT ? (p.n - k0) : KT);
    if (tid < KT && tid < kn) {
      pf_x = p.pts[2 * (k0 + tid)];
      pf_y = p.pts[2 * (k0 + tid) + 1];
    }
    // consecutive threads read consecutive values of the chunk (coalesced)
    const float* v = p.vals + k0 * (int64_t)D;
#pragma unroll
    for (int it = 0; it < L::kValRegs; ++it) {
      const int e = tid + it * kThreads;
      pf_v[it] = (e < kn * D) ? v[e] : 0.0f;
    }
  };
  prefetch(0);
  // table factors of a chunk: row e / KT of the tile's 16 + 4R rows, point
  // e % KT (consecutive threads read consecutive points of a row)
  double tv[L::kTabRegs];
  auto tab_load = [&](int64_t k0) {
#pragma unroll
    for (int it = 0; it < L::kTabRegs; ++it) {
      const int e = tid + it * kThreads;
      const int row = e / KT, k = e % KT;
      if (row < kCols + L::kRows) {
        const int64_t trow = row < kCols ? (int64_t)(c0 + row)
                                         : (int64_t)p.tab_cols + r0 + (row - kCols);
        tv[it] = p.tab[trow * p.tab_n + k0 + k];
      }
    }
  };

  // Gaussian step factors of the tile (exp(-2 s^2) per node step)
  const double sx = p.dx * p.inv_h, sy = p.dy * p.inv_h;
  const double qx = exp(-2.0 * sx * sx), qy = exp(-2.0 * sy * sy);

  // 1. tile-frame coordinates of a chunk, from the prefetched raw data;
  //    the first chunk's now, each later one right after the MFMA sweep of
  //    its predecessor (which does not read them)
  auto put_coords = [&](int kn_) {
    if (tid < KT) {
      double x = 0.0, y = 0.0;
      if (tid < kn_) {
        x = ((double)pf_x - cx) * p.inv_h;
        y = ((double)pf_y - cy) * p.inv_h;
      }
      ux[tid] = x;
      uy[tid] = y;
    }
  };
  put_coords((int)(p.n < KT ? p.n : KT));
  __syncthreads();
  // (point, attribute) of this thread's first feature element and the step
  // to its next one (kThreads elements on)
  const int fk0 = tid / D, fd0 = tid - fk0 * D;
  const int fks = kThreads / D, fds = kThreads - fks * D;

  for (int64_t k0 = 0; k0 < p.n; k0 += KT) {
    const int kn = (int)((p.n - k0) < KT ? (p.n - k0) : KT);
    // table factors of this chunk: loaded now, stored after the monomials
    // and features, so that the loads' latency overlaps that work and the
    // registers are not held during the sweep
    if (WM == WM_TABLE) tab_load(k0);
    for (int e = tid; e < (WM == WM_TABLE ? 0 : 4 * KT); e += kThreads) {
      // 2a. separable Gaussian factors g_c = exp(-(u - e_c)^2), e_c = (c - c_mid) s,
      //     for one point, one axis and one direction.  Start at the node
      //     nearest to u (the largest factor) and step outwards:
      //     g_{c+1} / g_c = exp(2 s (u - e_c) - s^2), and that ratio itself
      //     shrinks by exp(-2 s^2) per step, so every exponent is <= 0; one
      //     thread steps up from the nearest node and another down.  Points
      //     past n get weight 0.
      const int k = e & (KT - 1);
      const bool xaxis = (e & KT) == 0;
      const bool up = e < 2 * KT;
      const int cnt = xaxis ? kCols : L::kRows;
      const int mid = cnt / 2;
      const double s = xaxis ? sx : sy;
      const double q = xaxis ? qx : qy;
      double* g = xaxis ? gx : gy;
      // each direction owns half of the row when there is no stepping
      const int h0 = up ? 0 : mid, h1 = up ? mid : cnt;
      if (INV) {
        // inverse-distance weights do not separate: the tables hold the
        // node offsets, and the A operand forms the weight per pair
        const double u = k < kn ? (xaxis ? ux[k] : uy[k]) : 0.0;
        for (int c = h0; c < h1; ++c)
          g[c * KS + k] = k < kn ? u - (double)(c - mid) * s : __builtin_inf();
      } else if (k < kn) {
        const double u = xaxis ? ux[k] : uy[k];
        const double t = u / s + (double)mid;
        const int cs = (int)fmin(fmax(rint(t), 0.0), (double)(cnt - 1));
        const double dc = u - (double)(cs - mid) * s;
        const double gv = exp(-(dc * dc));
        double r = exp((up ? 2.0 : -2.0) * s * dc - s * s);
        double v = gv;
        if (up) {
          g[cs * KS + k] = gv;
          for (int c = cs + 1; c < cnt; ++c) {
            v *= r;
            r *= q;
            g[c * KS + k] = v;
          }
        } else {
          for (int c = cs - 1; c >= 0; --c) {
            v *= r;
            r *= q;
            g[c * KS + k] = v;
          }
        }
      } else {
        for (int c = h0; c < h1; ++c) g[c * KS + k] = 0.0;
      }
    }
    // 2b. moment monomials of the tile-frame coordinates
    for (int e = tid; e < nmom * KT; e += kThreads) {
      const int k = e % KT, j = e / KT;
      // exponents of monomial j (ordered by total degree, then by y power)
      int t = 0;
      while ((t + 1) * (t + 2) / 2 <= j) ++t;
      const int b = j - t * (t + 1) / 2, a = t - b;
      double v = 1.0;
      for (int q = 0; q < a; ++q) v *= ux[k];
      for (int q = 0; q < b; ++q) v *= uy[k];
      G[j * KS + k] = v;
    }
    // 2c. basis x attribute products from the prefetched values
    {
      int k = fk0, d = fd0;
#pragma unroll
      for (int it = 0; it < L::kValRegs; ++it) {
        if (k < KT) {
          const double f = (double)pf_v[it];
          G[(nmom + d) * KS + k] = f;
          if (m >= 3) {
            const double bx = ux[k], by = uy[k];
            G[(nmom + D + d) * KS + k] = bx * f;
            G[(nmom + 2 * D + d) * KS + k] = by * f;
            if (m >= 6) {
              G[(nmom + 3 * D + d) * KS + k] = bx * bx * f;
              G[(nmom + 4 * D + d) * KS + k] = bx * by * f;
              G[(nmom + 5 * D + d) * KS + k] = by * by * f;
            }
          }
        }
        k += fks;
        d += fds;
        if (d >= D) {
          d -= D;
          ++k;
        }
      }
    }
    if (WM == WM_TABLE) {
      // 2a from the tables (zero past n)
#pragma unroll
      for (int it = 0; it < L::kTabRegs; ++it) {
        const int e = tid + it * kThreads;
        const int row = e / KT, k = e % KT;
        if (row < kCols) gx[row * KS + k] = tv[it];
        else if (row < kCols + L::kRows) gy[(row - kCols) * KS + k] = tv[it];
      }
    }
    // next chunk's raw data: in flight during the MFMA sweep
    if (k0 + KT < p.n) prefetch(k0 + KT);
    __syncthreads();

    // 3. MFMA sweep over the chunk
    const int i = lane & 15;        // A row (node column) / B column
    const int kq = (lane >> 4) * 4; // this lane's 4 points in each group of 16
    if (MLS_F64_SETPRIO) __builtin_amdgcn_s_setprio(1);
#pragma unroll MLS_F64_KG_UNROLL
    for (int kg = 0; kg < KT; kg += 16) {
      // four consecutive doubles of a row as two 16-byte reads (rows start
      // on 16-byte boundaries: KS is even and kg + kq a multiple of 4)
      double ax[4], ay[R][4], bv[Q4 > 0 ? Q4 : NT][4];
      read4(gx + i * KS + kg + kq, ax);
#pragma unroll
      for (int t = 0; t < R; ++t) read4(gy + (wave * R + t) * KS + kg + kq, ay[t]);
      if constexpr (Q4 > 0) {
        // feature 4 q + lane % 4 of the lane's four points
#pragma unroll
        for (int q = 0; q < Q4; ++q) read4(G + (q * 4 + (lane & 3)) * KS + kg + kq, bv[q]);
      } else {
#pragma unroll
        for (int q = 0; q < NT; ++q) read4(G + (q * 16 + i) * KS + kg + kq, bv[q]);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const double a = WM == WM_INV1   ? invpow_weight_int<1>(ax[j], ay[t][j])
                           : WM == WM_INV2 ? invpow_weight_int<2>(ax[j], ay[t][j])
                           : INV           ? invpow_weight(ax[j], ay[t][j], p.alpha)
                                           : ax[j] * ay[t][j];
          if constexpr (Q4 > 0) {
#pragma unroll
            for (int q = 0; q < Q4; ++q)
              acc4[t][q] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, bv[q][j], acc4[t][q], 0, 0, 0);
          } else {
#pragma unroll
            for (int q = 0; q < NT; ++q)
              acc[t][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv[q][j], acc[t][q], 0, 0, 0);
          }
        }
      }
    }
    if (MLS_F64_SETPRIO) __builtin_amdgcn_s_setprio(0);
    if (k0 + KT < p.n) put_coords((int)((p.n - k0 - KT) < KT ? (p.n - k0 - KT) : KT));
    __syncthreads();
  }

  // Epilogue: accumulators -> LDS [node][feature] -> one node per lane,
  // kEpiWaves waves at a time.  (The main loop ended with a barrier.)
  const int64_t plane = (int64_t)p.W * p.H;
#pragma unroll 1
  for (int g = 0; g < kWaves; g += kEpiWaves) {
    const bool mine = wave >= g && wave < g + kEpiWaves;
    double* epi = lds + (wave - g) * 16 * R * L::kEpiStride;
    if (mine) {
      if constexpr (Q4 > 0) {
#pragma unroll
        for (int t = 0; t < R; ++t)
#pragma unroll
          for (int q = 0; q < Q4; ++q) {
            // f64 4x4x4 MFMA result: lane holds node 4 ((lane/4) % 4) + lane/16, feature lane%4
            const int node = t * 16 + 4 * ((lane >> 2) & 3) + (lane >> 4);
            const int feat = q * 4 + (lane & 3);
            epi[node * L::kEpiStride + feat] = acc4[t][q];
          }
      } else {
#pragma unroll
        for (int t = 0; t < R; ++t)
#pragma unroll
          for (int q = 0; q < NT; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              // f64 16x16 MFMA result: lane holds row (lane/16 + 4r), column lane%16
              const int node = t * 16 + (lane >> 4) + 4 * r;
              const int feat = q * 16 + (lane & 15);
              epi[node * L::kEpiStride + feat] = acc[t][q][r];
            }
      }
    }
    __syncthreads();
    if (mine)
      solve_tile_nodes<DEG, R, EPI>(p, epi, L::kEpiStride, lane, wave, r0, c0, L::kRows, plane);
    __syncthreads();
  }
}

// One node per lane: the float64 ladder solve of the nodes of one wave.
template <int DEG, int R, int EPI>
__device__ void solve_tile_nodes(const F64Params& p, const double* epi, int stride, int lane,
                                 int wave, int r0, int c0, int rows, int64_t plane) {
  const int D = p.D;
  for (int node = lane; node < 16 * R; node += 64) {
    const int t = node / 16, col = node % 16;
    const int r = r0 + wave * R + t, c = c0 + col;
    if (r >= p.H || c >= p.W) continue;
    // node offset from the anchor, the same expression the weight factors use
    const double ex = (double)(col - kCols / 2) * p.dx * p.inv_h;
    const double ey = (double)(wave * R + t - rows / 2) * p.dy * p.inv_h;
    const int64_t off = (int64_t)r * p.W + c;
    uint8_t code;
    if constexpr (EPI == 2)
      code = rigid_node(epi + node * stride, ex, ey, p.h, p.floor_w, p.fields + off, plane);
    else
      code = solve_node<DEG>(epi + node * stride, D, ex, ey, p.tau, p.floor_w, p.fields + off,
                             plane, nullptr, nullptr, 1.0, EPI == 1 ? p.grads + off : nullptr,
                             p.inv_h);
    if (p.deg_out) p.deg_out[off] = code;
  }
}

template <int DEG, int NT, int R, int WM, int EPI, int Q4 = 0>
hipError_t launch_impl(const F64Params& prm, hipStream_t s) {
  using L = F64Layout<DEG, NT, R>;
  F64Params p = prm;
  const int tiles_x = (p.W + kCols - 1) / kCols;
  const int tiles_y = (p.H + L::kRows - 1) / L::kRows;
  p.tiles_x = tiles_x;
  const size_t lds_bytes = sizeof(double) * (size_t)L::kDoubles;
  hipError_t e = hipFuncSetAttribute((const void*)fit_f64_kernel<DEG, NT, R, WM, EPI, Q4>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds_bytes);
  if (e != hipSuccess) return e;
  const int64_t blocks = (int64_t)tiles_x * tiles_y;
  hipLaunchKernelGGL((fit_f64_kernel<DEG, NT, R, WM, EPI, Q4>), dim3((unsigned)blocks),
                     dim3(kThreads), lds_bytes, s, p);
  return hipGetLastError();
}

// R (row strips per wave) trades accumulator registers against the number
// of Gaussian factors per tile.
template <int DEG, int NT, int WM, int Q4>
hipError_t launch_epi(const F64Params& p, hipStream_t s) {
  constexpr int R = NT <= 3 ? 4 : (NT <= 6 ? 2 : 1);
  if (p.rigid) {
    if constexpr (DEG == 1 && NT == 1) return launch_impl<DEG, NT, R, WM, 2, Q4>(p, s);
    return hipErrorInvalidValue;
  }
  return p.grads ? launch_impl<DEG, NT, R, WM, 1, Q4>(p, s)
                 : launch_impl<DEG, NT, R, WM, 0, Q4>(p, s);
}

// At most 12 features (constant basis with D <= 11, linear basis with
// D <= 2, the timing-table shapes among them) run the 4x4x4 form: the
// 16x16x4 instruction would carry 4 or more empty feature columns.
template <int DEG, int NT, int WM>
hipError_t launch_nt(const F64Params& p, hipStream_t s) {
  if constexpr (NT == 1 && DEG < 2) {
    if (p.F <= 4) return launch_epi<DEG, NT, WM, 1>(p, s);
    if (p.F <= 8) return launch_epi<DEG, NT, WM, 2>(p, s);
    if (p.F <= 12) return launch_epi<DEG, NT, WM, 3>(p, s);
  }
  return launch_epi<DEG, NT, WM, 0>(p, s);
}

template <int DEG, int WM>
hipError_t launch_deg(const F64Params& p, int nt, hipStream_t s) {
  if constexpr (WM == WM_INV1 || WM == WM_INV2) {
    // the reciprocal forms serve one and two feature tiles, where the
    // weight is most of the vector work per matrix instruction
    return nt == 1 ? launch_nt<DEG, 1, WM>(p, s) : launch_nt<DEG, 2, WM>(p, s);
  }
  switch (nt) {
    case 1: return launch_nt<DEG, 1, WM>(p, s);
    case 2: return launch_nt<DEG, 2, WM>(p, s);
    case 3: return launch_nt<DEG, 3, WM>(p, s);
    case 4: return launch_nt<DEG, 4, WM>(p, s);
    case 5: case 6: return launch_nt<DEG, 6, WM>(p, s);
    case 7: case 8: return launch_nt<DEG, 8, WM>(p, s);
    case 9: case 10: case 11: case 12: return launch_nt<DEG, 12, WM>(p, s);
    default: return launch_nt<DEG, 16, WM>(p, s);
  }
}

template <int WM>
hipError_t launch_kind(const F64Params& p, int degree, int nt, hipStream_t s) {
  switch (degree) {
    case 0: return launch_deg<0, WM>(p, nt, s);
    case 1: return launch_deg<1, WM>(p, nt, s);
    default: return launch_deg<2, WM>(p, nt, s);
  }
}

// Gaussian factor tables: row r < cols is exp(-((x_k - (x0 + r dx)) / h)^2)
// over the points k, row cols + r the same with y and y0 + r dy; zero for
// k >= n.  Rows past the grid serve the padding nodes of edge tiles.
__global__ __launch_bounds__(256) void gauss_table_kernel(const float* __restrict__ pts, int64_t n,
                                                          int64_t tab_n, int cols, double x0,
                                                          double dx, double y0, double dy,
                                                          double inv_h, double* __restrict__ tab) {
  const int row = blockIdx.y;
  const bool xr = row < cols;
  const double c = xr ? x0 + (double)row * dx : y0 + (double)(row - cols) * dy;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < tab_n;
       k += (int64_t)gridDim.x * 256) {
    double v = 0.0;
    if (k < n) {
      const double u = ((double)pts[2 * k + (xr ? 0 : 1)] - c) * inv_h;
      v = exp(-(u * u));
    }
    tab[row * tab_n + k] = v;
  }
}

}  // namespace

hipError_t launch_fit_f64(const FitArgs& a, hipStream_t stream) {
  const int F = moment_terms(a.degree) + basis_terms(a.degree) * a.D;
  const int nt = (F + 15) / 16;
  if (nt > 16) return hipErrorInvalidValue;
  F64Params p;
  p.pts = a.pts;
  p.vals = a.vals;
  p.tab = nullptr;
  p.tab_n = 0;
  p.tab_cols = 0;
  p.n = a.n;
  p.D = a.D;
  p.F = F;
  p.h = a.h;
  p.inv_h = 1.0 / a.h;
  p.alpha = a.alpha;
  p.x0 = a.x0; p.y0 = a.y0; p.dx = a.dx; p.dy = a.dy;
  p.W = a.W; p.H = a.H;
  p.tiles_x = 0;
  p.tau = a.tau;
  p.floor_w = a.floor_w;
  p.fields = a.fields;
  p.deg_out = a.deg_out;
  p.grads = a.grads;
  p.rigid = a.rigid;
  if (a.wkind == 2) {   // inverse distance
    if (nt <= 2 && a.alpha == 1.0) return launch_kind<WM_INV1>(p, a.degree, nt, stream);
    if (nt <= 2 && a.alpha == 2.0) return launch_kind<WM_INV2>(p, a.degree, nt, stream);
    return launch_kind<WM_INV>(p, a.degree, nt, stream);
  }
  if (!a.gtab) return launch_kind<WM_GAUSS>(p, a.degree, nt, stream);
  p.tab = a.gtab;
  p.tab_n = f64_table_points(a.n);
  p.tab_cols = f64_table_rows(a.W);
  const int rows = p.tab_cols + f64_table_rows(a.H);
  const int64_t per_row = (p.tab_n + 255) / 256;
  const unsigned bx = (unsigned)(per_row < 64 ? per_row : 64);
  hipLaunchKernelGGL(gauss_table_kernel, dim3(bx, (unsigned)rows), dim3(256), 0, stream, a.pts,
                     a.n, p.tab_n, p.tab_cols, a.x0, a.dx, a.y0, a.dy, p.inv_h, a.gtab);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_kind<WM_TABLE>(p, a.degree, nt, stream);
}

int64_t f64_table_points(int64_t n) { return (n + KT - 1) / KT * KT; }
int f64_table_rows(int cells) { return (cells + kCols - 1) / kCols * kCols; }

size_t f64_table_bytes(int64_t n, int32_t W, int32_t H) {
  const double bytes = 8.0 * (double)f64_table_points(n) *
                       (double)(f64_table_rows(W) + f64_table_rows(H));
  return bytes <= (double)kF64TableCap ? (size_t)bytes : 0;
}

}  // namespace mls
