// Input staging for the low-precision fit paths.
//
// The attributes are fitted as f' = (f - shift_d) / scale_d with
// shift_d = (max_d + min_d) / 2 and scale_d = (max_d - min_d) / 2 over the
// input values, so every attribute lies in [-1, 1] before it is rounded to a
// 16-bit format.  Moving least squares is affine-equivariant in the values
// (the fit of a f + b is a fit(f) + b: Eq. 5-8 are linear in q and reproduce
// constants), so the solve maps the result back exactly.
//
// The staged payload is attribute-major, vals_t[d][i] = f'_{i,d} (float32),
// so a workgroup reading a chunk of points of one attribute reads one
// contiguous run.  Bound: HBM (one read of values, one write).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mls_internal.h"

namespace mls {
namespace {

constexpr int kRowsPerBlock = 1024;

// Partial min / max of each attribute over a block of rows.  Block (32, 8):
// threadIdx.x walks 32 consecutive attributes of a row (coalesced),
// threadIdx.y strides over the block's rows.
__global__ __launch_bounds__(256) void attr_range_kernel(const float* vals, int64_t n, int D,
                                                         float* pmin, float* pmax) {
  __shared__ float smin[8][33], smax[8][33];
  const int d = blockIdx.y * 32 + threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kRowsPerBlock;
  const int64_t r1 = r0 + kRowsPerBlock < n ? r0 + kRowsPerBlock : n;
  float lo = INFINITY, hi = -INFINITY;
  if (d < D) {
    for (int64_t r = r0 + threadIdx.y; r < r1; r += 8) {
      const float v = vals[r * D + d];
      lo = fminf(lo, v);
      hi = fmaxf(hi, v);
    }
  }
  smin[threadIdx.y][threadIdx.x] = lo;
  smax[threadIdx.y][threadIdx.x] = hi;
  __syncthreads();
  if (threadIdx.y == 0 && d < D) {
    for (int q = 1; q < 8; ++q) {
      lo = fminf(lo, smin[q][threadIdx.x]);
      hi = fmaxf(hi, smax[q][threadIdx.x]);
    }
    pmin[(int64_t)blockIdx.x * D + d] = lo;
    pmax[(int64_t)blockIdx.x * D + d] = hi;
  }
}

// One block per attribute: min / max over the partial ranges (min and max
// are exact, so the order of the reduction does not matter).
__global__ __launch_bounds__(256) void attr_finalize_kernel(const float* pmin, const float* pmax,
                                                            int nblk, int D, float* shift,
                                                            float* scale) {
  __shared__ float slo[4], shi[4];
  const int d = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  float lo = INFINITY, hi = -INFINITY;
  for (int b = t; b < nblk; b += 256) {
    lo = fminf(lo, pmin[(int64_t)b * D + d]);
    hi = fmaxf(hi, pmax[(int64_t)b * D + d]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, o, 64));
    hi = fmaxf(hi, __shfl_xor(hi, o, 64));
  }
  if (lane == 0) {
    slo[wave] = lo;
    shi[wave] = hi;
  }
  __syncthreads();
  if (t != 0) return;
  lo = fminf(fminf(slo[0], slo[1]), fminf(slo[2], slo[3]));
  hi = fmaxf(fmaxf(shi[0], shi[1]), fmaxf(shi[2], shi[3]));
  // float64 midpoint and half-range, rounded once
  const double mid = 0.5 * ((double)lo + (double)hi);
  const double half = 0.5 * ((double)hi - (double)lo);
  shift[d] = (float)mid;
  scale[d] = half > 0.0 ? (float)half : 1.0f;
}

// vals_t[d][i] = (vals[i][d] - shift[d]) / scale[d], through a 32 x 32 LDS
// tile so that both the read and the write are coalesced.
__global__ __launch_bounds__(256) void stage_values_kernel(const float* vals, int64_t n, int D,
                                                           const float* shift, const float* scale,
                                                           float* vals_t) {
  __shared__ float tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.x * 32;
  const int d0 = blockIdx.y * 32;
  for (int q = threadIdx.y; q < 32; q += 8) {
    const int64_t i = i0 + q;
    const int d = d0 + threadIdx.x;
    float v = 0.0f;
    if (i < n && d < D) v = (float)(((double)vals[i * D + d] - (double)shift[d]) / (double)scale[d]);
    tile[q][threadIdx.x] = v;
  }
  __syncthreads();
  for (int q = threadIdx.y; q < 32; q += 8) {
    const int d = d0 + q;
    const int64_t i = i0 + threadIdx.x;
    if (i < n && d < D) vals_t[(int64_t)d * n + i] = tile[threadIdx.x][q];
  }
}

}  // namespace

int64_t stage_partial_blocks(int64_t n) { return (n + kRowsPerBlock - 1) / kRowsPerBlock; }

hipError_t launch_stage(const float* vals, int64_t n, int D, float* pmin, float* pmax,
                        float* shift, float* scale, float* vals_t, hipStream_t s) {
  const int64_t nblk = stage_partial_blocks(n);
  const int dblk = (D + 31) / 32;
  hipLaunchKernelGGL(attr_range_kernel, dim3((unsigned)nblk, dblk), dim3(32, 8), 0, s, vals, n,
                     D, pmin, pmax);
  hipLaunchKernelGGL(attr_finalize_kernel, dim3(D), dim3(256), 0, s, pmin, pmax, (int)nblk, D,
                     shift, scale);
  hipLaunchKernelGGL(stage_values_kernel, dim3((unsigned)((n + 31) / 32), dblk), dim3(32, 8), 0,
                     s, vals, n, D, shift, scale, vals_t);
  return hipGetLastError();
}

}  // namespace mls
