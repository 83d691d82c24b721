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

// Marching squares over D fields at n_iso isovalues each.
struct ContourArgs {
  const float* fields;   // [D][H][W]
  const float* iso;      // [D][n_iso]
  int32_t D, n_iso, W, H;
  double x0, y0, dx, dy;
  uint8_t* cases;        // [D][n_iso][(H-1)(W-1)] or null
  float* segs;           // [capacity][4]
  int32_t* ids;          // [capacity][3] or null
  int64_t capacity;
  // scratch (library-owned): contour_scratch_entries() int32 counts and
  // int64 offsets, contour_scan_tiles() int64 tile sums, one int64 total
  int32_t* counts;
  int64_t* offsets;
  int64_t* tile_sums;
  int64_t* total;
};
int64_t contour_scratch_entries(int32_t D, int32_t n_iso, int32_t W, int32_t H);
int64_t contour_scan_tiles(int64_t entries);
hipError_t launch_contour(const ContourArgs& a, hipStream_t stream);

}  // namespace mls
