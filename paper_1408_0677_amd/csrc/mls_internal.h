// Internal declarations shared by the host API and the kernel sources of the
// MLS library.  Nothing here is part of the public ABI (include/mls.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mls {

// Everything a fit kernel needs, resolved and validated on the host.
struct FitArgs {
  const float* pts;     // [n][2]
  const float* vals;    // [n][D]
  int64_t n;
  int32_t D;
  int32_t degree;       // 0, 1, 2
  int32_t wkind;        // mls_weight_kind
  double h, alpha;
  double x0, y0, dx, dy;
  int32_t W, H;
  double tau, floor_w;
  float* fields;        // [D][H][W]
  uint8_t* deg_out;     // [H][W] or null
};

// Number of basis terms m and of distinct moment monomials for a degree.
__host__ __device__ constexpr int basis_terms(int deg) { return deg == 0 ? 1 : (deg == 1 ? 3 : 6); }
__host__ __device__ constexpr int moment_terms(int deg) { return deg == 0 ? 1 : (deg == 1 ? 6 : 15); }

// Float64 matrix-core fit (Gaussian weight).  Returns a hipError_t.
hipError_t launch_fit_f64(const FitArgs& a, hipStream_t stream);

}  // namespace mls
