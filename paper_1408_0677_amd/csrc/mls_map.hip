// Space mappings of the MLS fields (Muelder et al., Sec. 3.4, Fig. 5b-d):
// discrete colour bands and adaptive contour lines, per grid node.
//
// Bands: the band of a value is the number of isovalues at or below it
// (the contour cases' tie rule), 255 for NaN; with a colour map the node
// also takes its band's RGBA colour (0 for NaN).
//
// Adaptive lines: level j = 0 .. L-1 has lines at origin + k spacing / 2^j.
// At a node the field changes by r = |(g_x dx, g_y dy)| per pixel (the
// gradient in pixel coordinates), so level j's lines are s_j = (spacing /
// 2^j) / r pixels apart; level 0 is always drawn, finer levels with opacity
// clamp((s_j - fade_lo) / (fade_hi - fade_lo), 0, 1) -- more lines where
// space is expanded, fewer where it is compressed.  The intensity is the
// largest opacity x (1 - e_j / halfwidth)+ over the levels, e_j the pixel
// distance to the nearest level-j line.  Float64 arithmetic per node.
//
// Both are elementwise: one read of the field (and gradient), one write per
// node, bound by HBM.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mls_internal.h"

namespace mls {
namespace {

__device__ __forceinline__ int value_band(float v, const float* iso, int n_iso) {
  if (isnan(v)) return 255;
  int b = 0;
  for (int k = 0; k < n_iso; ++k) b += v >= iso[k] ? 1 : 0;
  return b;
}

// Four consecutive nodes of one field per thread when P % 4 == 0 and the
// arrays are aligned for it (16-byte loads, 4-byte band and 16-byte colour
// stores), one per thread otherwise.
__global__ __launch_bounds__(256) void map_bands_kernel(MapBandsArgs a, bool vec) {
  const int64_t per = vec ? 4 : 1;
  const int64_t total = (int64_t)a.D * a.P / per;
  for (int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x; u < total;
       u += (int64_t)gridDim.x * 256) {
    const int64_t i = u * per;
    const int d = (int)(i / a.P);
    const float* iso = a.iso + (int64_t)d * a.n_iso;
    const uint32_t* cm = a.colormap ? a.colormap + (int64_t)d * (a.n_iso + 1) : nullptr;
    if (vec) {
      const float4 v = *(const float4*)(a.fields + i);
      const int b0 = value_band(v.x, iso, a.n_iso), b1 = value_band(v.y, iso, a.n_iso);
      const int b2 = value_band(v.z, iso, a.n_iso), b3 = value_band(v.w, iso, a.n_iso);
      if (a.bands)
        *(uint32_t*)(a.bands + i) = (uint32_t)b0 | ((uint32_t)b1 << 8) | ((uint32_t)b2 << 16) |
                                    ((uint32_t)b3 << 24);
      if (a.rgba)
        *(uint4*)(a.rgba + i) = make_uint4(b0 == 255 ? 0u : cm[b0], b1 == 255 ? 0u : cm[b1],
                                           b2 == 255 ? 0u : cm[b2], b3 == 255 ? 0u : cm[b3]);
    } else {
      const int b = value_band(a.fields[i], iso, a.n_iso);
      if (a.bands) a.bands[i] = (uint8_t)b;
      if (a.rgba) a.rgba[i] = b == 255 ? 0u : cm[b];
    }
  }
}

__device__ __forceinline__ float adaptive_intensity(const MapAdaptiveArgs& a, double f, double gx,
                                                    double gy, double origin, double spacing) {
  if (isnan(f)) return __builtin_nanf("");
  const double px = gx * a.dx, py = gy * a.dy;
  const double per_px = sqrt(px * px + py * py);
  if (!(per_px > 0.0) || !isfinite(per_px) || !(spacing > 0.0)) return 0.0f;
  // one division each for the pixel scale and the level index; the levels
  // halve the step exactly
  const double inv_r = 1.0 / per_px;
  const double inv_fade = 1.0 / (a.fade_hi - a.fade_lo);
  const double inv_hw = 1.0 / a.halfwidth;
  double t = (f - origin) / spacing;     // position in level-0 steps
  double s = spacing * inv_r;            // level-0 spacing in pixels
  double best = 0.0;
  for (int j = 0; j < a.n_levels; ++j, t *= 2.0, s *= 0.5) {
    const double op = j == 0 ? 1.0 : fmin(fmax((s - a.fade_lo) * inv_fade, 0.0), 1.0);
    const double e = fabs(t - rint(t)) * s;
    best = fmax(best, op * fmax(1.0 - e * inv_hw, 0.0));
  }
  return (float)best;
}

// Four consecutive nodes of one field per thread when P % 4 == 0 and the
// arrays are 16-byte aligned.
__global__ __launch_bounds__(256) void map_adaptive_kernel(MapAdaptiveArgs a, bool vec) {
  const int64_t per = vec ? 4 : 1;
  const int64_t total = (int64_t)a.D * a.P / per;
  for (int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x; u < total;
       u += (int64_t)gridDim.x * 256) {
    const int64_t i = u * per;
    const int64_t d = i / a.P, q = i - d * a.P;
    const double origin = (double)a.levels[2 * d], spacing = (double)a.levels[2 * d + 1];
    const float* gxp = a.grads + (2 * d) * a.P + q;
    const float* gyp = a.grads + (2 * d + 1) * a.P + q;
    if (vec) {
      const float4 f = *(const float4*)(a.fields + i);
      const float4 gx = *(const float4*)gxp, gy = *(const float4*)gyp;
      float4 o;
      o.x = adaptive_intensity(a, f.x, gx.x, gy.x, origin, spacing);
      o.y = adaptive_intensity(a, f.y, gx.y, gy.y, origin, spacing);
      o.z = adaptive_intensity(a, f.z, gx.z, gy.z, origin, spacing);
      o.w = adaptive_intensity(a, f.w, gx.w, gy.w, origin, spacing);
      *(float4*)(a.out + i) = o;
    } else {
      a.out[i] = adaptive_intensity(a, a.fields[i], gxp[0], gyp[0], origin, spacing);
    }
  }
}

// Enough workgroups to fill the chip several times over (grid-stride
// loops cover the rest).
unsigned elementwise_blocks(int64_t units) {
  const int64_t b = (units + 255) / 256;
  return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

}  // namespace

hipError_t launch_map_bands(const MapBandsArgs& a, hipStream_t s) {
  const bool vec = (a.P & 3) == 0 && ((uintptr_t)a.fields & 15) == 0 &&
                   ((uintptr_t)a.bands & 3) == 0 && ((uintptr_t)a.rgba & 15) == 0;
  const int64_t units = vec ? (int64_t)a.D * a.P / 4 : (int64_t)a.D * a.P;
  hipLaunchKernelGGL(map_bands_kernel, dim3(elementwise_blocks(units)), dim3(256), 0, s, a, vec);
  return hipGetLastError();
}

hipError_t launch_map_adaptive(const MapAdaptiveArgs& a, hipStream_t s) {
  const bool vec = (a.P & 3) == 0 && ((uintptr_t)a.fields & 15) == 0 &&
                   ((uintptr_t)a.grads & 15) == 0 && ((uintptr_t)a.out & 15) == 0;
  const int64_t units = vec ? (int64_t)a.D * a.P / 4 : (int64_t)a.D * a.P;
  hipLaunchKernelGGL(map_adaptive_kernel, dim3(elementwise_blocks(units)), dim3(256), 0, s, a,
                     vec);
  return hipGetLastError();
}

}  // namespace mls
