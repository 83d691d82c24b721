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
// index order and sums them in that order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mls_internal.h"

namespace mls {
namespace {

__global__ __launch_bounds__(256) void hit_keys_kernel(const float* pts, int64_t n, double x0,
                                                       double y0, double dx, double dy, int W,
                                                       int H, uint32_t* keys, uint32_t* idx) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
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
  keys[i] = key;
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

}  // namespace

hipError_t launch_hits(const HitArgs& a, hipStream_t s) {
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
