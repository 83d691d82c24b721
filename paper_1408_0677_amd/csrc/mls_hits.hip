// Exact hits of the inverse-distance weight (Muelder et al., Eq. 4 and the
// interpolation property of Sec. 3.3): the weight 1 / |p - x_i|^(2 alpha) is
// infinite where a node coincides with data points, and the field there is
// the mean of those points' values (degree code 254).  The fit kernel gives
// such nodes a large finite weight; this pass overwrites them.
//
// A node coincides with a point when the point lies exactly on the node's
// position x0 + c dx, y0 + r dy (float64, no contraction).  Each point can
// coincide with at most one node of a grid with nonzero spacing: the node
// nearest to it.  Keys (node id, or W*H for none) are radix-sorted with the
// point index as a stable payload, so every hit node sees its points in
// index order and sums them in that order; small point sets do the same in
// one workgroup (hits_small_kernel below).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mls_internal.h"

namespace mls {
namespace {

// Node key of a point: the node it lies on exactly, or none.
__device__ __forceinline__ uint32_t hit_key(const float* pts, int64_t i, double x0, double y0,
                                            double dx, double dy, int W, int H) {
#pragma clang fp contract(off)
  const uint32_t none = (uint32_t)W * (uint32_t)H;
  const double px = (double)pts[2 * i], py = (double)pts[2 * i + 1];
  const double fc = rint((px - x0) / dx), fr = rint((py - y0) / dy);
  uint32_t key = none;
  if (fc >= 0.0 && fc < (double)W && fr >= 0.0 && fr < (double)H) {
    const int c = (int)fc, r = (int)fr;
    const double ex = px - (x0 + (double)c * dx);
    const double ey = py - (y0 + (double)r * dy);
    if (ex * ex + ey * ey == 0.0) key = (uint32_t)r * (uint32_t)W + (uint32_t)c;
  }
  return key;
}

__global__ __launch_bounds__(256) void hit_keys_kernel(const float* pts, int64_t n, double x0,
                                                       double y0, double dx, double dy, int W,
                                                       int H, uint32_t* keys, uint32_t* idx) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  keys[i] = hit_key(pts, i, x0, y0, dx, dy, W, H);
  idx[i] = (uint32_t)i;
}

// One thread per sorted entry; the first entry of each run of equal node
// keys writes the node's mean.
__global__ __launch_bounds__(256) void hit_mean_kernel(const uint32_t* keys, const uint32_t* idx,
                                                       int64_t n, uint32_t none,
                                                       const float* vals, int D, int64_t plane,
                                                       float* fields, uint8_t* deg,
                                                       float* grads) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t k = keys[i];
  if (k == none || (i > 0 && keys[i - 1] == k)) return;
  int64_t end = i + 1;
  while (end < n && keys[end] == k) ++end;
  const double cnt = (double)(end - i);
  for (int d = 0; d < D; ++d) {
    double s = 0.0;
    for (int64_t j = i; j < end; ++j) s += (double)vals[(int64_t)idx[j] * D + d];
    fields[(int64_t)d * plane + k] = (float)(s / cnt);
  }
  if (deg) deg[k] = 254;
  // the field jumps to the points' own value there: no slope
  if (grads)
    for (int d = 0; d < 2 * D; ++d) grads[(int64_t)d * plane + k] = __builtin_nanf("");
}

// Small point sets in one workgroup (one launch instead of a radix sort's
// dozen): each thread keys four consecutive points, the hitting points are
// compacted into LDS in index order, and only when there are any are the
// (node, index) pairs sorted (bitonic, in LDS) and the runs averaged as
// above.  Sorting by (node, index) orders each node's points by index, as
// the stable radix sort does, so the sums and results are the same.
constexpr int kHitSmallThreads = 1024;
constexpr int kHitSmall = 4 * kHitSmallThreads;   // points of the one-workgroup form

__global__ __launch_bounds__(kHitSmallThreads) void hits_small_kernel(
    const float* pts, int n, double x0, double y0, double dx, double dy, int W, int H,
    const float* vals, int D, int64_t plane, float* fields, uint8_t* deg, float* grads) {
  __shared__ uint64_t pair[kHitSmall];   // node << 32 | point index
  __shared__ int wsum[kHitSmallThreads / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const uint32_t none = (uint32_t)W * (uint32_t)H;
  uint32_t key[4];
  int cnt = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = 4 * t + q;
    key[q] = i < n ? hit_key(pts, i, x0, y0, dx, dy, W, H) : none;
    cnt += key[q] != none;
  }
  // exclusive prefix of the counts over the threads, in index order
  int incl = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int base = incl - cnt, m = 0;
#pragma unroll
  for (int w = 0; w < kHitSmallThreads / 64; ++w) {
    if (w < wave) base += wsum[w];
    m += wsum[w];
  }
  if (m == 0) return;   // the same in every thread: no barrier is skipped by some only
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (key[q] != none) pair[base++] = ((uint64_t)key[q] << 32) | (uint32_t)(4 * t + q);
  int P = 1;
  while (P < m) P <<= 1;
  for (int i = m + t; i < P; i += kHitSmallThreads) pair[i] = ~0ull;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = t; i < P; i += kHitSmallThreads) {
        const int ij = i ^ j;
        if (ij > i) {
          const uint64_t a = pair[i], b = pair[ij];
          if (((i & k) == 0) == (a > b)) {
            pair[i] = b;
            pair[ij] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = t; i < m; i += kHitSmallThreads) {
    const uint32_t k = (uint32_t)(pair[i] >> 32);
    if (i > 0 && (uint32_t)(pair[i - 1] >> 32) == k) continue;
    int end = i + 1;
    while (end < m && (uint32_t)(pair[end] >> 32) == k) ++end;
    const double c = (double)(end - i);
    for (int d = 0; d < D; ++d) {
      double sum = 0.0;
      for (int j = i; j < end; ++j) sum += (double)vals[(int64_t)(uint32_t)pair[j] * D + d];
      fields[(int64_t)d * plane + k] = (float)(sum / c);
    }
    if (deg) deg[k] = 254;
    if (grads)
      for (int d = 0; d < 2 * D; ++d) grads[(int64_t)d * plane + k] = __builtin_nanf("");
  }
}

}  // namespace

hipError_t launch_hits(const HitArgs& a, hipStream_t s) {
  if (a.n <= kHitSmall) {
    hipLaunchKernelGGL(hits_small_kernel, dim3(1), dim3(kHitSmallThreads), 0, s, a.pts, (int)a.n,
                       a.x0, a.y0, a.dx, a.dy, a.W, a.H, a.vals, a.D, (int64_t)a.W * a.H,
                       a.fields, a.deg_out, a.grads);
    return hipGetLastError();
  }
  const unsigned gb = (unsigned)((a.n + 255) / 256);
  const uint32_t none = (uint32_t)a.W * (uint32_t)a.H;
  hipLaunchKernelGGL(hit_keys_kernel, dim3(gb), dim3(256), 0, s, a.pts, a.n, a.x0, a.y0, a.dx,
                     a.dy, a.W, a.H, a.keys, a.idx);
  int bits = 8;
  while (bits < 32 && ((uint64_t)1 << bits) <= (uint64_t)none) ++bits;
  hipError_t e = radix_sort_pairs(a.keys, a.idx, a.keys2, a.idx2, a.n, bits, a.hist, a.ssum, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(hit_mean_kernel, dim3(gb), dim3(256), 0, s, a.keys, a.idx, a.n, none, a.vals,
                     a.D, (int64_t)a.W * a.H, a.fields, a.deg_out, a.grads);
  return hipGetLastError();
}

}  // namespace mls
