// Internal declarations shared by the host API and the kernel sources of the
// MLS library.  Nothing here is part of the public ABI (include/mls.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mls {

typedef int mls_status_t;   // an mls_status value

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
  int32_t lp_slab;      // 16-bit paths: attributes per slab, 0 = lp_slab_plan's choice
  int32_t lp_form;      // 16-bit paths: 0 the library's choice, 1 one pass, 2 two passes
  float* grads;         // [D][2][H][W] slopes of the local fits, or null
  bool rigid;           // rigid map of 2-vector values (degree 1 moments, D = 2)
  double* gtab;         // float64 Gaussian: factor tables in scratch, or null
};

// Number of basis terms m and of distinct moment monomials for a degree.
__host__ __device__ constexpr int basis_terms(int deg) { return deg == 0 ? 1 : (deg == 1 ? 3 : 6); }
__host__ __device__ constexpr int moment_terms(int deg) { return deg == 0 ? 1 : (deg == 1 ? 6 : 15); }

// Float64 matrix-core fit (Gaussian or inverse-distance weight).  Returns a
// hipError_t.  With the inverse-distance weight, launch_hits must follow.
// With a.gtab (f64_table_bytes of scratch) the Gaussian factors of every
// grid column and row are tabulated first and copied by the tiles.
hipError_t launch_fit_f64(const FitArgs& a, hipStream_t stream);
// Float64 Gaussian factor tables: points padded to the chunk, columns and
// rows padded to the tile; 0 bytes when the tables would pass the cap (the
// kernel then generates the factors per tile).
constexpr size_t kF64TableCap = (size_t)512 << 20;
int64_t f64_table_points(int64_t n);
int f64_table_rows(int cells);
size_t f64_table_bytes(int64_t n, int32_t W, int32_t H);

// Cell-ordered payload for compactly supported weights (from launch_cells).
struct CellGeom;
struct LPCells;

// 16-bit matrix-core fit (bf16 or fp16 feature terms, float32
// accumulation).  vals_t/shift/scale come from launch_stage; the Wendland
// weight needs `cells`.
hipError_t launch_fit_lp(const FitArgs& a, const float* vals_t, const float* shift,
                         const float* scale, bool fp16, int terms, const LPCells* cells,
                         hipStream_t stream);
// Attribute slabs of the 16-bit kernel: `forced_ds` attributes per slab
// (0 = the cost model's choice); NTS feature tiles of 16 per slab.
void lp_slab_plan(int degree, int D, int forced_ds, int* nts, int* ds, int* nslab);
// The checks of mls_fit / mls_fit_grad and the fit's arguments (no device
// work enqueued); `terms` receives the 16-bit terms per feature.  The
// caller passes the library's public types through void pointers to keep
// this header free of them.
mls_status_t fit_prepare_c(void* ctx, const float* d_points, const float* d_values, int64_t n,
                           int32_t d, int32_t basis, const void* weight, const void* grid,
                           int32_t precision, const void* opts, float* d_fields, float* d_grad,
                           uint8_t* d_degree, FitArgs* out, int* terms);

// A context's fit scratch (reserved with mls_context_reserve): pointer and
// size.  The served batches stage their requests there.
void* context_scratch(void* ctx, size_t* bytes);

// Served batches of one-pass 16-bit fits with the Gaussian weight: requests
// of one class (degree, feature tiles per slab, terms, float16 or bfloat16)
// share a persistent kernel that takes (request, block) items from a device
// counter (mls_server.cpp).
struct LPBatchClass {
  int deg, nts, terms;
  bool fp16;
  int64_t blocks;        // work items of this request (tiles x slabs)
};
// False if the request does not run the one-pass Gaussian kernel with its
// format's default term count (3 bfloat16, 2 float16 terms).
bool lp_batch_class(const FitArgs& a, bool fp16, int terms, LPBatchClass* cls);
// The kernel parameters of one request (lp_params_bytes() bytes, opaque).
size_t lp_params_bytes();
void lp_params_write(const FitArgs& a, const float* vals_t, const float* shift,
                     const float* scale, void* out);
// d_items: n_items (request, block) pairs of uint32; d_total[n_req] items
// per request; d_head (one word), d_done[n_req] and d_skipped[n_req] zero
// at launch; h_complete (set to 1, or 2 if items were skipped) and h_cancel
// host-visible flags per request.  grid: at most this many workgroups (0:
// one per resident slot of the device).
hipError_t launch_fit_lp_batch(const LPBatchClass& c, const void* d_params, const uint32_t* d_items,
                               int n_items, const uint32_t* d_total, uint32_t* d_head,
                               uint32_t* d_done, uint32_t* d_skipped, uint32_t* h_complete,
                               const uint32_t* h_cancel, int grid, hipStream_t s);

// Whether the 16-bit fit runs in the two-pass (shape-function) form.
bool lp_use_shape_form(int degree, int D, bool fp16, int wkind, bool grads, int terms,
                       int forced_ds, int form);
// Largest attributes per slab the kernel supports for a degree.
int lp_max_slab(int degree);
// Largest node offset across a 16 x 16 node tile, in units of h.
double lp_tile_extent(double dx, double dy, double h);

// Attribute staging: partial ranges (stage_partial_blocks(n) x D floats in
// pmin and pmax), shift/scale [D], attribute-major normalised copy [D][n].
int64_t stage_partial_blocks(int64_t n);
hipError_t launch_stage(const float* vals, int64_t n, int D, float* pmin, float* pmax,
                        float* shift, float* scale, float* vals_t, hipStream_t s);

// Geometry shared by the cell list and the kernels that walk it: square
// cells of side `cell` from (ox, oy); node tiles of kTileCols x kTileRows
// nodes of the grid (x0 + c dx, y0 + r dy); support radius h.
constexpr int kTileCols = 16;
constexpr int kTileRows = 16;
struct CellGeom {
  double ox, oy, cell;
  double x0, y0, dx, dy;
  double h;
};

// Cell columns [cx0, cx1] and rows [cy0, cy1] that can hold points within h
// of some node of tile (tc, tr).
__host__ __device__ inline void tile_cell_range(const CellGeom& g, int tc, int tr, int ncx,
                                                int ncy, int* cx0, int* cx1, int* cy0,
                                                int* cy1) {
  const double xa = g.x0 + (double)(tc * kTileCols) * g.dx;
  const double xb = g.x0 + (double)(tc * kTileCols + kTileCols - 1) * g.dx;
  const double ya = g.y0 + (double)(tr * kTileRows) * g.dy;
  const double yb = g.y0 + (double)(tr * kTileRows + kTileRows - 1) * g.dy;
  const double xlo = (xa < xb ? xa : xb) - g.h, xhi = (xa < xb ? xb : xa) + g.h;
  const double ylo = (ya < yb ? ya : yb) - g.h, yhi = (ya < yb ? yb : ya) + g.h;
  double fx0 = floor((xlo - g.ox) / g.cell), fx1 = floor((xhi - g.ox) / g.cell);
  double fy0 = floor((ylo - g.oy) / g.cell), fy1 = floor((yhi - g.oy) / g.cell);
  fx0 = fx0 < 0 ? 0 : fx0;
  fy0 = fy0 < 0 ? 0 : fy0;
  fx1 = fx1 > ncx - 1 ? ncx - 1 : fx1;
  fy1 = fy1 > ncy - 1 ? ncy - 1 : fy1;
  *cx0 = (int)fx0;
  *cx1 = (int)fx1;
  *cy0 = (int)fy0;
  *cy1 = (int)fy1;
}

struct CellArgs {
  const float* pts;        // [n][2]
  const float* vals_t;     // [D][n] staged attributes
  int64_t n;
  int D;
  CellGeom geom;
  int ncx, ncy;
  int tiles_x, tiles;
  // outputs
  uint32_t* cell_start;    // [ncx * ncy + 1]
  uint32_t* perm;          // [n] input index of each sorted point
  float* pts_s;            // [n][2] in cell order
  float* vals_ts;          // [D][n] in cell order
  uint32_t* torder;        // [tile_order_slots] node tile of each workgroup slot
  // per-tile point lists: the cell-ordered indices of the points within h
  // of some node of the tile (in cell order), tile t's entries at
  // [tile_start[t], tile_start[t + 1]) of tile_list
  uint32_t* tile_start;    // [tiles + 1]
  uint32_t* tile_list;     // [list_cap]
  int64_t list_cap;
  // scratch
  uint32_t* keys;          // [n]
  uint32_t* keys2;         // [n]
  uint32_t* perm2;         // [n]
  uint32_t* hist;          // [256 * radix_blocks(n)]
  uint32_t* tkeys;         // [tiles]
  uint32_t* tkeys2;        // [tiles]
  uint32_t* torder2;       // [tiles]
  uint32_t* thist;         // [256 * radix_blocks(tiles)]
  uint32_t* sorder;        // [tiles] supertiles by descending work
  uint32_t* ssum;          // [scan_sums_words(largest scan)] scan block sums
};
int64_t radix_blocks(int64_t n);
// Stable LSD radix sort of (key, value) pairs on the low `bits` bits; the
// result ends in (k0, v0); (k1, v1), hist[256 * radix_blocks(n)] and
// sums[scan_sums_words(256 * radix_blocks(n))] are scratch.
hipError_t radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n,
                            int bits, uint32_t* hist, uint32_t* sums, hipStream_t s);
// Exclusive scan of `count` uint32 values in place (block sums in `sums`,
// scan_sums_words(count) words).
int64_t scan_sums_words(int64_t count);
hipError_t scan_u32(uint32_t* v, int64_t count, uint32_t* sums, hipStream_t s);

// Exact hits of the inverse-distance weight: nodes on data points take the
// mean of those points' values and degree code 254.
struct HitArgs {
  const float* pts;        // [n][2]
  const float* vals;       // [n][D]
  int64_t n;
  int32_t D;
  double x0, y0, dx, dy;   // dx, dy nonzero
  int32_t W, H;
  float* fields;           // [D][H][W]
  uint8_t* deg_out;        // [H][W] or null
  float* grads;            // [D][2][H][W] or null (NaN at hit nodes)
  uint32_t *keys, *keys2, *idx, *idx2, *hist;   // scratch (n, n, n, n, 256 radix_blocks(n))
  uint32_t* ssum;                               // scratch (scan block sums)
};
hipError_t launch_hits(const HitArgs& a, hipStream_t s);
hipError_t launch_cells(const CellArgs& a, hipStream_t stream);

// Scratch layout of one mls_fit call (byte offsets into one buffer).
struct FitPlan {
  size_t o_pmin, o_pmax, o_shift, o_scale, o_vals;
  size_t o_keys, o_keys2, o_perm, o_perm2, o_hist, o_cs, o_pts, o_vals_s;
  size_t o_tk, o_tk2, o_to, o_to2, o_th;
  size_t o_ts, o_tl, o_so, o_ssum;
  size_t o_gtab, gtab_bytes;   // float64 Gaussian factor tables (gtab_bytes 0: none)
  int64_t order_slots;
  int64_t list_cap;       // entries of the per-tile point lists, at most
  size_t total;
  int ncx, ncy, tiles_x, tiles;
  CellGeom geom;
};
FitPlan make_fit_plan(int64_t n, int32_t d, int32_t precision, int32_t wkind, double h,
                      double x0, double y0, double dx, double dy, int32_t W, int32_t H);
size_t fit_scratch_bytes(int64_t n, int32_t d, int32_t precision, int32_t wkind, double h,
                         double x0, double y0, double dx, double dy, int32_t W, int32_t H);

struct LPCells {
  const float* pts_s;
  const float* vals_ts;
  const uint32_t* cell_start;
  const uint32_t* torder;
  const uint32_t* tile_start;
  const uint32_t* tile_list;
  int ncx, ncy;
  CellGeom geom;
};

// Workgroup slots of the compact-support fit's tile order: node tiles are
// grouped into 4 x 4 supertiles, and the supertiles (heaviest first) are
// dealt to the eight XCDs in turn, each supertile's 16 tiles on 16
// consecutive slots of one XCD, so that tiles sharing points share an L2.
// Slots without a tile hold 0xFFFFFFFF.
constexpr int kSuperTile = 4;
inline int64_t tile_order_slots(int tiles_x, int tiles_y) {
  const int64_t sx = (tiles_x + kSuperTile - 1) / kSuperTile;
  const int64_t sy = (tiles_y + kSuperTile - 1) / kSuperTile;
  return 8 * kSuperTile * kSuperTile * ((sx * sy + 7) / 8);
}

// Upper bound of the per-tile point list entries: a point lies within h of
// the node rectangles of at most this many tiles.
int64_t tile_list_bound(int64_t n, double h, double dx, double dy, int tiles_x, int tiles_y);

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
  // scratch (library-owned): contour_scratch_entries() int32 counts, which
  // the scan turns into int32 offsets in place; contour_scan_tiles() int64
  // tile sums; one int64 total
  int32_t* counts;
  int32_t* offsets;
  int64_t* tile_sums;
  int64_t* total;
};
int64_t contour_scratch_entries(int32_t D, int32_t n_iso, int32_t W, int32_t H);
int64_t contour_scan_tiles(int64_t entries);
hipError_t launch_contour(const ContourArgs& a, hipStream_t stream);

// The contour passes' fixed device scratch (for callers that cannot
// allocate): resolve its address on `device` (made current by the caller;
// once per device, later calls return the cached address), and read it back.
hipError_t contour_static_scratch_resolve(int device);
void* contour_static_scratch(int device);

// Space mappings (discrete colour bands, adaptive contour lines) of D
// fields of P nodes each.
struct MapBandsArgs {
  const float* fields;      // [D][P]
  const float* iso;         // [D][n_iso]
  const uint32_t* colormap; // [D][n_iso + 1] or null
  int32_t D, n_iso;
  int64_t P;
  uint8_t* bands;           // [D][P] or null
  uint32_t* rgba;           // [D][P] or null (needs colormap)
};
hipError_t launch_map_bands(const MapBandsArgs& a, hipStream_t s);

struct MapAdaptiveArgs {
  const float* fields;      // [D][P]
  const float* grads;       // [D][2][P]
  const float* levels;      // [D][2] origin, spacing
  int32_t D, n_levels;
  int64_t P;
  double dx, dy, halfwidth, fade_lo, fade_hi;
  float* out;               // [D][P]
};
hipError_t launch_map_adaptive(const MapAdaptiveArgs& a, hipStream_t s);

// Planarity-preserving layout iterations (float64 state in buf0/buf1,
// each [n][2]); pos holds the float32 positions in and out.
struct LayoutArgs {
  float* pos;
  int64_t n;
  const int32_t *adj_start, *adj, *fan_start, *fan;
  int64_t n_adj, n_fan;
  double C, D, eta, t0, lambda;
  int32_t iterations;
  double *buf0, *buf1;
};
hipError_t launch_layout(const LayoutArgs& a, hipStream_t s);

}  // namespace mls
