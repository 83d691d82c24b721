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
// blocks.  Points stream through double-buffered LDS in chunks of KT; a
// chunk buffer holds
//   - Gaussian weight factors gx[col][k] = exp(-((x_k - p_col)/h)^2) and
//     gy[row][k] (the Gaussian separates on a grid, so a tile needs
//     16 + 4R exponentials per point instead of 64R),
//   - the feature block G[j][k] in float64.
// The MFMA sweep over a chunk reads the A operand (node x point weight) as
// gx * gy, built in registers, and B from G.  Within each group of 16 points
// a lane supplies points k0 + 4 (lane / 16) + j for MFMA j = 0..3, so it
// reads four consecutive points with one 32-byte LDS access.  After each
// group's MFMAs the workgroup fills the same 16 points of the next chunk
// into the other buffer, so staging overlaps the matrix work and a chunk
// costs one barrier.
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
#ifndef MLS_F64_PAD
#define MLS_F64_PAD 2
#endif

constexpr int kMmaWaves = 4;             // waves issuing matrix instructions
constexpr int kProdThreads = 256;        // threads of the staging waves
constexpr int kThreads = kMmaWaves * 64 + kProdThreads;
constexpr int kWaves = kMmaWaves;        // waves that own node strips
constexpr int kCols = 16;            // node columns per tile (one M-tile)
constexpr int kPad = MLS_F64_PAD;    // LDS row padding in doubles
constexpr int kEpiWaves = kMmaWaves;     // all accumulators go through LDS at once

struct F64Params {
  const float* pts;
  const float* vals;
  int64_t n;
  int D, F;
  double inv_h, sx, sy;   // 1/h, dx/h, dy/h
  double x0, y0, dx, dy;
  int W, H, tiles_x;
  double tau, floor_w;
  float* fields;
  uint8_t* deg_out;
};

// exp(-a) for a >= 0 in float64 (the device library's exp).
__device__ __forceinline__ double exp_neg(double a) { return exp(-a); }

template <int DEG, int NT, int R>
struct F64Layout {
  static constexpr int kRows = kWaves * R;
  static constexpr int kFP = NT * 16;                    // padded features
  // points per chunk: 64, or 32 where two 64-point buffers would not fit
  static constexpr int KT = (2 * (kCols + kRows + kFP) * (MLS_F64_KT + kPad) * 8 <= 160 * 1024)
                                ? MLS_F64_KT : 32;
  static constexpr int KS = KT + kPad;                   // LDS row stride in doubles
  static constexpr int kParts = KT / 16;                 // MFMA groups per chunk
  static_assert(KT % 16 == 0, "chunk must hold whole MFMA groups");
  // one chunk buffer; the kernel double-buffers it
  static constexpr int kGx = 0;                          // [16][KS]
  static constexpr int kGy = kGx + kCols * KS;           // [kRows][KS]
  static constexpr int kG = kGy + kRows * KS;            // [kFP][KS]
  static constexpr int kBuf = kG + kFP * KS;
  // epilogue phase: per solving wave [16R nodes][kFP + 1]
  static constexpr int kEpiStride = kFP + 1;
  static constexpr int kEpi = kEpiWaves * 16 * R * kEpiStride;
  static constexpr int kDoubles = 2 * kBuf > kEpi ? 2 * kBuf : kEpi;
};

// Fill the LDS entries of points [kb, kb + 16) of the chunk that starts at
// point k0: Gaussian factors for the tile's columns and rows, moment
// monomials and basis x attribute features.  Every entry is computed from
// the inputs in global memory (cached), so the parts of a chunk have no
// dependence on each other and can be spread between MFMA groups.
template <int DEG, int NT, int R>
__device__ __forceinline__ void stage_part(const F64Params& p, double* buf, int64_t k0,
                                           int kb, int tid, double cx, double cy) {
  using L = F64Layout<DEG, NT, R>;
  constexpr int m = DEG == 0 ? 1 : (DEG == 1 ? 3 : 6);
  constexpr int nmom = DEG == 0 ? 1 : (DEG == 1 ? 6 : 15);
  double* gx = buf + L::kGx;
  double* gy = buf + L::kGy;
  double* G = buf + L::kG;
  const int64_t last = p.n - 1;
  // Gaussian factors: (16 + kRows) rows x 16 points
#pragma unroll
  for (int it = 0; it < ((kCols + L::kRows) * 16 + kProdThreads - 1) / kProdThreads; ++it) {
    const int e = tid + it * kProdThreads;
    if (e < (kCols + L::kRows) * 16) {
      const int k = kb + (e & 15), row = e >> 4;
      const int64_t gi = k0 + k;
      const bool valid = gi <= last;
      const int64_t gc = valid ? gi : last;
      if (row < kCols) {
        const double u = ((double)p.pts[2 * gc] - cx) * p.inv_h - (double)(row - kCols / 2) * p.sx;
        gx[row * L::KS + k] = valid ? exp_neg(u * u) : 0.0;
      } else {
        const int rr = row - kCols;
        const double u = ((double)p.pts[2 * gc + 1] - cy) * p.inv_h -
                         (double)(rr - L::kRows / 2) * p.sy;
        gy[rr * L::KS + k] = valid ? exp_neg(u * u) : 0.0;
      }
    }
  }
  // moment monomials u_x^a u_y^b, ordered by total degree then by b
  for (int e = tid; e < nmom * 16; e += kProdThreads) {
    const int k = kb + (e & 15), j = e >> 4;
    const int64_t gi = k0 + k;
    double v = 0.0;
    if (gi <= last) {
      const double ux = ((double)p.pts[2 * gi] - cx) * p.inv_h;
      const double uy = ((double)p.pts[2 * gi + 1] - cy) * p.inv_h;
      int t = 0;
      while ((t + 1) * (t + 2) / 2 <= j) ++t;
      const int b = j - t * (t + 1) / 2, a = t - b;
      v = 1.0;
      for (int q = 0; q < a; ++q) v *= ux;
      for (int q = 0; q < b; ++q) v *= uy;
    }
    G[j * L::KS + k] = v;
  }
  // basis x attribute products; consecutive threads read consecutive values
  // of one point (coalesced)
  const int D = p.D;
  for (int e = tid; e < 16 * D; e += kProdThreads) {
    const int k = kb + e / D, d = e - (e / D) * D;
    const int64_t gi = k0 + k;
    double f = 0.0, ux = 0.0, uy = 0.0;
    if (gi <= last) {
      f = (double)p.vals[gi * (int64_t)D + d];
      ux = ((double)p.pts[2 * gi] - cx) * p.inv_h;
      uy = ((double)p.pts[2 * gi + 1] - cy) * p.inv_h;
    }
    G[(nmom + d) * L::KS + k] = f;
    if (m >= 3) {
      G[(nmom + D + d) * L::KS + k] = ux * f;
      G[(nmom + 2 * D + d) * L::KS + k] = uy * f;
    }
    if (m >= 6) {
      G[(nmom + 3 * D + d) * L::KS + k] = ux * ux * f;
      G[(nmom + 4 * D + d) * L::KS + k] = ux * uy * f;
      G[(nmom + 5 * D + d) * L::KS + k] = uy * uy * f;
    }
  }
}

template <int DEG, int R>
__device__ void solve_tile_nodes(const F64Params& p, const double* epi, int stride, int lane,
                                 int wave, int r0, int c0, int rows, int64_t plane);

template <int DEG, int NT, int R>
__global__ __launch_bounds__(kThreads) void fit_f64_kernel(F64Params p) {
  using L = F64Layout<DEG, NT, R>;
  extern __shared__ double lds[];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  // Waves 0..3 run the matrix cores, waves 4..7 stage the next chunk.
  const bool mma_wave = wave < kMmaWaves;
  const int ptid = tid - kMmaWaves * 64;   // producer thread index (0..255)
  const int tile_c = blockIdx.x % p.tiles_x;
  const int tile_r = blockIdx.x / p.tiles_x;
  const int c0 = tile_c * kCols;
  const int r0 = tile_r * L::kRows;
  // tile anchor: the node at the tile's centre (may lie beyond the grid)
  const double cx = p.x0 + (double)(c0 + kCols / 2) * p.dx;
  const double cy = p.y0 + (double)(r0 + L::kRows / 2) * p.dy;

  doublex4 acc[R][NT];
#pragma unroll
  for (int t = 0; t < R; ++t)
#pragma unroll
    for (int q = 0; q < NT; ++q) acc[t][q] = doublex4{0.0, 0.0, 0.0, 0.0};

  if (!mma_wave) {
    // padding features are zero in both buffers for the whole kernel
    for (int e = ptid; e < (L::kFP - p.F) * L::KT; e += kProdThreads) {
      const int k = e % L::KT, j = p.F + e / L::KT;
      lds[L::kG + j * L::KS + k] = 0.0;
      lds[L::kBuf + L::kG + j * L::KS + k] = 0.0;
    }
#pragma unroll 1
    for (int part = 0; part < L::kParts; ++part)
      stage_part<DEG, NT, R>(p, lds, 0, part * 16, ptid, cx, cy);
  }
  __syncthreads();

  const int i = lane & 15;         // A row (node column) / B column
  const int kq = (lane >> 4) * 4;  // this lane's 4 points in each group of 16
  int c = 0;
  for (int64_t k0 = 0; k0 < p.n; k0 += L::KT, ++c) {
    if (mma_wave) {
      const double* cur = lds + (c & 1) * L::kBuf;
#pragma unroll 1
      for (int kg = 0; kg < L::KT; kg += 16) {
        const double* gxr = cur + L::kGx + i * L::KS + kg + kq;
        double ax[4] = {gxr[0], gxr[1], gxr[2], gxr[3]};
        double ay[R][4];
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const double* gyr = cur + L::kGy + (wave * R + t) * L::KS + kg + kq;
          ay[t][0] = gyr[0]; ay[t][1] = gyr[1]; ay[t][2] = gyr[2]; ay[t][3] = gyr[3];
        }
        if constexpr (NT <= 6) {
          // few feature tiles: read each lane's four points at once
          double bv[NT][4];
#pragma unroll
          for (int q = 0; q < NT; ++q) {
            const double* gr = cur + L::kG + (q * 16 + i) * L::KS + kg + kq;
            bv[q][0] = gr[0]; bv[q][1] = gr[1]; bv[q][2] = gr[2]; bv[q][3] = gr[3];
          }
#pragma unroll
          for (int j = 0; j < 4; ++j) {
#pragma unroll
            for (int t = 0; t < R; ++t) {
              const double a = ax[j] * ay[t][j];
#pragma unroll
              for (int q = 0; q < NT; ++q)
                acc[t][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv[q][j], acc[t][q], 0, 0, 0);
            }
          }
        } else {
          // many feature tiles: one point at a time keeps registers down
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            double bj[NT];
#pragma unroll
            for (int q = 0; q < NT; ++q) bj[q] = cur[L::kG + (q * 16 + i) * L::KS + kg + kq + j];
#pragma unroll
            for (int t = 0; t < R; ++t) {
              const double a = ax[j] * ay[t][j];
#pragma unroll
              for (int q = 0; q < NT; ++q)
                acc[t][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bj[q], acc[t][q], 0, 0, 0);
            }
          }
        }
      }
    } else if (k0 + L::KT < p.n) {
      double* nxt = lds + ((c & 1) ^ 1) * L::kBuf;
#pragma unroll 1
      for (int part = 0; part < L::kParts; ++part)
        stage_part<DEG, NT, R>(p, nxt, k0 + L::KT, part * 16, ptid, cx, cy);
    }
    __syncthreads();
  }

  // Epilogue: accumulators -> LDS [wave][node][feature] -> one node per lane.
  if (mma_wave) {
    double* epi = lds + wave * 16 * R * L::kEpiStride;
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
  __syncthreads();
  if (mma_wave) {
    const double* epi = lds + wave * 16 * R * L::kEpiStride;
    const int64_t plane = (int64_t)p.W * p.H;
    solve_tile_nodes<DEG, R>(p, epi, L::kEpiStride, lane, wave, r0, c0, L::kRows, plane);
  }
}

// One node per lane: the float64 ladder solve of the nodes of one wave.
template <int DEG, int R>
__device__ void solve_tile_nodes(const F64Params& p, const double* epi, int stride, int lane,
                                 int wave, int r0, int c0, int rows, int64_t plane) {
  const int D = p.D;
  for (int node = lane; node < 16 * R; node += 64) {
    const int t = node / 16, col = node % 16;
    const int r = r0 + wave * R + t, c = c0 + col;
    if (r >= p.H || c >= p.W) continue;
    // node offset from the anchor, the same expression the weight factors use
    const double ex = (double)(col - kCols / 2) * p.sx;
    const double ey = (double)(wave * R + t - rows / 2) * p.sy;
    const int64_t off = (int64_t)r * p.W + c;
    uint8_t code = solve_node<DEG>(epi + node * stride, D, ex, ey, p.tau, p.floor_w,
                                   p.fields + off, plane);
    if (p.deg_out) p.deg_out[off] = code;
  }
}

template <int DEG, int NT, int R>
hipError_t launch_impl(const F64Params& prm, hipStream_t s) {
  using L = F64Layout<DEG, NT, R>;
  F64Params p = prm;
  const int tiles_x = (p.W + kCols - 1) / kCols;
  const int tiles_y = (p.H + L::kRows - 1) / L::kRows;
  p.tiles_x = tiles_x;
  const size_t lds_bytes = sizeof(double) * (size_t)L::kDoubles;
  hipError_t e = hipFuncSetAttribute((const void*)fit_f64_kernel<DEG, NT, R>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds_bytes);
  if (e != hipSuccess) return e;
  const int64_t blocks = (int64_t)tiles_x * tiles_y;
  hipLaunchKernelGGL((fit_f64_kernel<DEG, NT, R>), dim3((unsigned)blocks), dim3(kThreads),
                     lds_bytes, s, p);
  return hipGetLastError();
}

// R (row strips per wave) trades accumulator registers against the number
// of Gaussian factors per tile.
template <int DEG, int NT>
hipError_t launch_nt(const F64Params& p, hipStream_t s) {
  constexpr int R = NT <= 3 ? 4 : (NT <= 6 ? 2 : 1);
  return launch_impl<DEG, NT, R>(p, s);
}

template <int DEG>
hipError_t launch_deg(const F64Params& p, int nt, hipStream_t s) {
  switch (nt) {
    case 1: return launch_nt<DEG, 1>(p, s);
    case 2: return launch_nt<DEG, 2>(p, s);
    case 3: return launch_nt<DEG, 3>(p, s);
    case 4: return launch_nt<DEG, 4>(p, s);
    case 5: case 6: return launch_nt<DEG, 6>(p, s);
    case 7: case 8: return launch_nt<DEG, 8>(p, s);
    case 9: case 10: case 11: case 12: return launch_nt<DEG, 12>(p, s);
    default: return launch_nt<DEG, 16>(p, s);
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
  p.n = a.n;
  p.D = a.D;
  p.F = F;
  p.inv_h = 1.0 / a.h;
  p.sx = a.dx * p.inv_h;
  p.sy = a.dy * p.inv_h;
  p.x0 = a.x0; p.y0 = a.y0; p.dx = a.dx; p.dy = a.dy;
  p.W = a.W; p.H = a.H;
  p.tiles_x = 0;
  p.tau = a.tau;
  p.floor_w = a.floor_w;
  p.fields = a.fields;
  p.deg_out = a.deg_out;
  switch (a.degree) {
    case 0: return launch_deg<0>(p, nt, stream);
    case 1: return launch_deg<1>(p, nt, stream);
    default: return launch_deg<2>(p, nt, stream);
  }
}

}  // namespace mls
