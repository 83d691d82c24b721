/*
 * mls.h -- C ABI of the MI355X (gfx950) moving-least-squares field library.
 *
 * The library evaluates the moving-least-squares (MLS) interpolation of
 * Muelder et al., "A Moving Least Squares Based Approach for Contour
 * Visualization of Multi-Dimensional Data" (Sec. 3.3), on every node of a
 * 2-D grid laid over N scattered points that each carry D attribute values,
 * and extracts contour lines of the resulting fields (Sec. 3.4).
 *
 * Per grid node p, with data points x_i and values f_i in R^D:
 *   weights   w_i = w(|x_i - p|)         Gaussian exp(-r^2/h^2),
 *                                         Wendland C2 (1-r/h)^4 (4r/h+1), r<h,
 *                                         or inverse distance (r/h)^(-2 alpha)
 *                                         (Eq. 4)
 *   basis     b(u) = [1, u_x, u_y, u_x^2, u_x u_y, u_y^2]   (m = 1, 3, 6
 *             terms for constant / linear / quadratic), u = (x_i - p) / h
 *   normal equations   M c = R,  M = sum w_i b_i b_i^T,  R = sum w_i b_i f_i^T
 *   value     field_d(p) = c_{0,d}
 * The linear basis is the affine MLS of Eq. 6-8; the constant basis is the
 * weighted mean of Eq. 5.  Where sum_i w_i < weight_floor the node is
 * undetermined (NaN, degree code 255).  Otherwise a degree ladder runs: the
 * requested degree is accepted if the equilibrated Cholesky factorisation of
 * its normal matrix has every pivot >= pivot_tol, else the next lower degree
 * is tried; degree 0 always succeeds.
 *
 * Conventions for every call:
 *  - Pointers named d_* are device pointers (hipMalloc / torch CUDA tensors)
 *    on the context's device; h_* are host pointers.  The caller owns every
 *    buffer; the library never frees caller memory.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *    enqueued asynchronously; results are valid after the stream syncs.
 *  - Argument errors are detected before any device work is enqueued and
 *    returned synchronously; nothing is written to outputs in that case.
 *    A device failure during enqueue returns MLS_ERR_DEVICE.  The detail of
 *    the last error of the calling thread is available from mls_last_error().
 *  - A context is used by one host thread at a time.  Its scratch memory
 *    is shared by all its calls: a call enqueued on a different stream
 *    from the previous scratch-using call first makes its stream wait for
 *    that call's work (an event the context records), so calls on several
 *    streams are correct but run one after the other.  Use one context per
 *    stream for concurrency.
 */
#ifndef MLS_H_
#define MLS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MLS_OK = 0,
  MLS_ERR_INVALID_ARG = -1,   /* bad size, pointer, enum or parameter */
  MLS_ERR_OUT_OF_MEMORY = -2, /* a library scratch allocation failed */
  MLS_ERR_CAPACITY = -3,      /* output buffer too small (contour) */
  MLS_ERR_DEVICE = -4,        /* HIP runtime error, wrong device */
  MLS_ERR_OVER_BUDGET = -5,   /* (server) request or point set exceeds the budget */
  MLS_ERR_CANCELLED = -6,     /* (server) request cancelled or past its timeout */
  MLS_ERR_UNSUPPORTED = -7,   /* valid request the library does not run */
  MLS_PENDING = 1             /* (server) request not finished yet */
} mls_status;

typedef enum {
  MLS_BASIS_CONSTANT = 0,  /* m = 1: weighted mean (Eq. 5) */
  MLS_BASIS_LINEAR = 1,    /* m = 3: affine MLS (Eq. 6-8) */
  MLS_BASIS_QUADRATIC = 2, /* m = 6 */
  MLS_BASIS_RIGID = 3       /* rigid MLS of 2-vector values (Eq. 9-10): d = 2,
                               fields[0..1] are the mapped coordinates; the
                               rotation-and-translation fit comes from the
                               linear-basis moments; MLS_PREC_F64 only, no
                               gradients */
} mls_basis;

typedef enum {
  MLS_W_GAUSSIAN = 0,    /* exp(-r^2/h^2) */
  MLS_W_WENDLAND_C2 = 1, /* (1 - r/h)^4 (4 r/h + 1) for r < h, else 0 */
  MLS_W_INVPOW = 2       /* (r/h)^(-2 alpha), Eq. 4 */
} mls_weight_kind;

/*
 * Arithmetic of the weight x feature contraction (inputs and outputs are
 * always float32; the per-node solve is always float64).
 *  MLS_PREC_F64:  float64 contraction on the matrix cores.  This is the
 *                 accurate plain path: the normal equations lose about
 *                 log10(condition) digits, which float32 sums cannot spare.
 *  MLS_PREC_BF16: bfloat16 matrix-core contraction with float32
 *                 accumulation.  Attributes are normalised to [-1, 1], each
 *                 feature is carried as `lp_terms` bfloat16 terms (default
 *                 3, about 24 significant bits) and the weight as a hi + lo
 *                 pair; the lo part multiplies every feature term but the
 *                 last, so all features of a (node, point) pair see the
 *                 same weight to about 24 bits (5 products per feature).
 *  MLS_PREC_FP16: the same with float16 terms (default 2 terms, about 22
 *                 bits; 3 products per feature).  Weights are scaled by
 *                 2^15 internally to stay above float16's subnormals.
 */
typedef enum {
  MLS_PREC_F64 = 0,
  MLS_PREC_BF16 = 1,
  MLS_PREC_FP16 = 2
} mls_precision;

typedef struct {
  int32_t kind;  /* mls_weight_kind */
  double h;      /* bandwidth (Gaussian), support radius (Wendland), or length
                    unit (inverse distance); finite and > 0 */
  double alpha;  /* inverse-distance exponent (Eq. 4); ignored otherwise */
} mls_weight;

/* Node (r, c) sits at (x0 + c*dx, y0 + r*dy), 0 <= r < height,
 * 0 <= c < width.  Fields are stored row-major [D][height][width]. */
typedef struct {
  double x0, y0, dx, dy;
  int32_t width, height;
} mls_grid;

typedef struct {
  double pivot_tol;     /* tau: smallest accepted equilibrated pivot; 1e-8 */
  double weight_floor;  /* nodes with sum of weights below this are NaN; 1e-6 */
  int32_t lp_terms;     /* 16-bit terms per feature for MLS_PREC_BF16/FP16:
                           1, 2 or 3; 0 selects the default (3 for
                           bfloat16, 2 for float16) */
  int32_t lp_slab;      /* MLS_PREC_BF16/FP16: attributes per workgroup
                           slab, 0 = the library's plan, else 1 ..
                           MLS_LP_MAX_SLAB_<basis>.  A tuning knob only:
                           results are bitwise the same for every value */
  int32_t lp_form;      /* MLS_PREC_BF16 with the Gaussian weight, linear or
                           quadratic basis, no gradients: 0 = the library's
                           choice, 1 = one pass (moments and right-hand
                           sides together, F = n_mom + m D columns),
                           2 = two passes (shape-function form: the moments
                           and each node's ladder first, then the effective
                           weights w (y^T b) against the attributes, F =
                           n_mom + D columns).  Ignored elsewhere */
} mls_solve_opts;

typedef struct mls_context mls_context;

/* Degree codes written to d_degree. */
#define MLS_DEGREE_UNDETERMINED 255
#define MLS_DEGREE_POINT_HIT 254

/* Largest attribute count D accepted by mls_fit with MLS_PREC_F64 for each
 * basis, and with the 16-bit precisions (any basis). */
#define MLS_MAX_D_CONSTANT 255
#define MLS_MAX_D_LINEAR 83
#define MLS_MAX_D_QUADRATIC 40
#define MLS_MAX_D_LP 1024
/* Largest point count. */
#define MLS_MAX_N ((int64_t)1 << 31)
/* 16-bit precisions: largest span of a 16 x 16 node tile, 15 max(|dx|, |dy|)
 * / h, per basis (the constant basis has no limit).  The tile shares one
 * moment frame; moving the float32 moments to a node that far from it
 * cancels digits (the quadratic basis more, through fourth powers). */
#define MLS_LP_MAX_SLAB_CONSTANT 40
#define MLS_LP_MAX_SLAB_LINEAR 40
#define MLS_LP_MAX_SLAB_QUADRATIC 18
#define MLS_LP_MAX_TILE_SPAN_LINEAR 4.0
#define MLS_LP_MAX_TILE_SPAN_QUADRATIC 2.5

/* Status name ("MLS_OK", ...); never NULL. */
const char* mls_status_string(mls_status s);

/* Detail of the calling thread's last failed call ("" if none). */
const char* mls_last_error(void);

/* Create a context on HIP device `device` (must be a gfx950 device).
 * Returns MLS_ERR_DEVICE if the device cannot be used. */
mls_status mls_context_create(int32_t device, mls_context** out);

/* Release a context and its scratch memory.  NULL is a no-op. */
void mls_context_destroy(mls_context* ctx);

/*
 * Evaluate D MLS fields on a grid (Sec. 3.3, Eq. 4-8; see top of file).
 *  d_points  float32 [n][2] (x, y), row-major, device
 *  d_values  float32 [n][d], row-major, device
 *  n >= 1 points (at most MLS_MAX_N), 1 <= d attributes (at most
 *            MLS_MAX_D_<basis> for MLS_PREC_F64, MLS_MAX_D_LP otherwise);
 *            coordinates and values must be finite
 *  basis     mls_basis
 *  weight    weight kind and parameters (host struct)
 *  grid      grid description (host struct), width >= 1, height >= 1,
 *            finite x0, y0, dx, dy
 *  precision mls_precision of the contraction
 *  opts      solve options (host struct) or NULL for the defaults
 *  d_fields  float32 [d][height][width] output, device
 *  d_degree  uint8 [height][width] output (accepted degree, 255 for
 *            undetermined), device, or NULL
 * Supported: the Gaussian weight with all three bases and all
 * precisions; the Wendland C2 weight with the 16-bit precisions (through a
 * device cell list); the inverse-distance weight with MLS_PREC_F64 on grids
 * with nonzero dx and dy (a node that coincides exactly with data points
 * takes the mean of their values, degree code 254; library scratch of about
 * 16 n bytes; the Gaussian on MLS_PREC_F64 uses scratch for its factor
 * tables, see mls_fit_scratch_bytes).  Other combinations return
 * MLS_ERR_UNSUPPORTED.  The 16-bit precisions
 * also return MLS_ERR_UNSUPPORTED when a node tile spans more than
 * MLS_LP_MAX_TILE_SPAN_<basis> (linear, quadratic), and MLS_PREC_FP16 when
 * tile-frame features would leave the float16 range; MLS_PREC_F64 serves
 * such coarse grids.
 * The 16-bit precisions use library scratch of about 4 n d bytes (plus the
 * cell list for Wendland); mls_fit_scratch_bytes gives the exact figure.
 */
mls_status mls_fit(mls_context* ctx, const float* d_points, const float* d_values,
                   int64_t n, int32_t d, int32_t basis, const mls_weight* weight,
                   const mls_grid* grid, int32_t precision,
                   const mls_solve_opts* opts, float* d_fields, uint8_t* d_degree,
                   void* stream);

/*
 * mls_fit plus the slope of each node's local fit (the gradient that the
 * adaptive contour-line mapping of Sec. 3.4 follows): for the basis centred
 * on the node and scaled by h, d f_d / dx = c_1 / h and d f_d / dy = c_2 / h.
 *  d_grad  float32 [d][2][height][width] output, device, not NULL: plane
 *          2 d holds d f_d / dx, plane 2 d + 1 holds d f_d / dy.  Zero where
 *          the ladder accepts the constant basis; NaN where the field is
 *          NaN and at exact hits of the inverse-distance weight (the field
 *          jumps to the points' value there).
 * Other arguments, errors and scratch as mls_fit.  The float64 path runs a
 * separate kernel variant (one workgroup per CU instead of two).
 */
mls_status mls_fit_grad(mls_context* ctx, const float* d_points, const float* d_values,
                        int64_t n, int32_t d, int32_t basis, const mls_weight* weight,
                        const mls_grid* grid, int32_t precision,
                        const mls_solve_opts* opts, float* d_fields, float* d_grad,
                        uint8_t* d_degree, void* stream);

/* Parameters of the planarity-preserving layout (Sec. 3.2, Eq. 1-3). */
typedef struct {
  double C;       /* repulsion scale (Eq. 1 and 3), >= 0 */
  double D;       /* desired edge length (Eq. 2), > 0 */
  double eta;     /* softening of Eq. 1-3, and the margin every node keeps
                     from every limiting line, > 0 */
  double t0;      /* temperature of the first iteration: the longest move */
  double lambda;  /* temperature decay, t_k = t0 lambda^k, 0 < lambda <= 1 */
} mls_layout_params;

/*
 * Planarity-preserving force-directed layout of a triangulated point set
 * (Sec. 3.2, Eq. 1-3, with the limiting-line constraint): `iterations`
 * iterations; in each, every node moves by the sum of the repulsion from
 * every other node, the springs along its mesh edges and the repulsion from
 * the opposite edge of each of its triangles, shortened to the
 * temperature, then scaled down so that it crosses none of the three
 * limiting lines (through the midpoints of two edges) of any of its
 * triangles, keeping eta clear.  No triangle of the mesh can flip.
 *  d_pos        float32 [n][2] positions, device; read, then overwritten
 *               with the result
 *  d_adj_start  int32 [n + 1] CSR starts of the neighbour lists, device
 *  d_adj        int32 [n_adj] neighbour indices, device (NULL if n_adj = 0)
 *  d_fan_start  int32 [n + 1] starts of the triangle fans, device
 *  d_fan        int32 [n_fan][2] the other two vertices of each triangle
 *               around the node, device (NULL if n_fan = 0)
 * Entries outside [0, n) and list ranges outside the arrays are ignored,
 * not read.  The state is float64 in library scratch (32 n bytes).  Runs on
 * the stream; returns after enqueueing.
 */
mls_status mls_layout(mls_context* ctx, float* d_pos, int64_t n, const int32_t* d_adj_start,
                      const int32_t* d_adj, int64_t n_adj, const int32_t* d_fan_start,
                      const int32_t* d_fan, int64_t n_fan, const mls_layout_params* params,
                      int32_t iterations, void* stream);

/*
 * Per-stage timing of a context's calls (the paper reports per-stage times,
 * Table 1).  With tracing on, every mls_fit, mls_fit_grad, mls_contour and
 * mls_layout call records timing events on its stream around its stages:
 *   fit:     "stage" (16-bit staging), "cells" (compact-support cell list
 *            and tile lists), "contract" (the weight x feature contraction
 *            and the per-node solve), "hits" (inverse-distance exact hits)
 *   contour: "passes";  layout: "iterations"
 * Recording adds events only; nothing waits for them until a record is read
 * back.  When jsonl_path is given (may be NULL), each call appends one JSON
 * line {"call", the request's sizes, "stages_ms": {...}, "total_ms"} to it
 * once its events complete (read back lazily, at most 64 calls pending).
 * Turning tracing off (or on again) first reads back every pending call.
 */
#define MLS_TRACE_MAX_STAGES 4
typedef struct {
  char call[16];                     /* "fit", "fit_grad", "contour", "layout" */
  int32_t form;                      /* fits: 0 float64 contraction, 1 16-bit one
                                        pass, 2 16-bit two passes; -1 otherwise */
  int32_t n_stages;
  char stage[MLS_TRACE_MAX_STAGES][16];
  double ms[MLS_TRACE_MAX_STAGES];   /* per stage, in stream order */
  double total_ms;
} mls_trace_record;

mls_status mls_context_trace(mls_context* ctx, int32_t enable, const char* jsonl_path);

/* Wait for the context's traced calls and return the last one's stage
 * times.  MLS_ERR_INVALID_ARG if no call has been traced. */
mls_status mls_context_trace_last(mls_context* ctx, mls_trace_record* out);

/*
 * Device scratch bytes mls_fit needs for this request; 0 also for invalid
 * arguments.  MLS_PREC_F64 with the Gaussian weight tabulates the weight
 * factors of every grid column and row once per call, 8 x (n rounded up to
 * 64) x (width and height each rounded up to 16) bytes, when that is at most
 * 512 MiB (beyond, the factors are generated per tile and no scratch is
 * needed); the inverse-distance weight needs about 16 n bytes.
 */
size_t mls_fit_scratch_bytes(int64_t n, int32_t d, int32_t precision,
                             const mls_weight* weight, const mls_grid* grid);

/*
 * Allocate `bytes` of fit scratch in the context now, so that later mls_fit
 * calls that need at most that much allocate nothing.  (mls_fit grows the
 * scratch when it needs more; growing frees the old buffer, which waits for
 * the device.)
 */
mls_status mls_context_reserve(mls_context* ctx, size_t bytes);

/*
 * Marching-squares contour lines of fields on a grid (Sec. 3.4, contour
 * lines of the MLS output; Fig. 5a).
 *  d_fields   float32 [d][height][width], device (e.g. mls_fit output)
 *  d          number of fields, >= 1
 *  grid       node positions as for mls_fit; width, height >= 2
 *  d_iso      float32 [d][n_iso] isovalues per field, device
 *  n_iso      isovalues per field, >= 1
 *  d_cases    uint8 [d][n_iso][height-1][width-1] output, device, or NULL:
 *             per cell, bit k = (corner k >= iso) with corners
 *             v0 = f[i][j], v1 = f[i][j+1], v2 = f[i+1][j+1], v3 = f[i+1][j];
 *             255 where a corner is NaN (no segment)
 *  d_segments float32 [capacity][4] output (x_from, y_from, x_to, y_to) in
 *             grid coordinates, device, 16-byte aligned; may be NULL when
 *             capacity == 0
 *  d_seg_ids  int32 [capacity][3] output (field, iso index, cell index
 *             i*(width-1)+j), device, or NULL
 *  capacity   number of segment slots (>= 0)
 *  h_count    host output: the number of segments the call produces
 * Rules: saddle cells (cases 5, 10) join the corners >= iso when the centre
 * value ((v0+v1)+(v2+v3))/4 >= iso; a crossing is interpolated from the
 * edge endpoint with the smaller (row, col), so shared edges give identical
 * points; segments keep the >= iso side on their left; segments are ordered
 * by (field, iso, cell, segment).  The call waits for the stream to deliver
 * the count.  If the count exceeds capacity it returns MLS_ERR_CAPACITY
 * (*h_count still written, d_cases complete, segment contents unspecified);
 * call again with a larger buffer.
 */
mls_status mls_contour(mls_context* ctx, const float* d_fields, int32_t d,
                       const mls_grid* grid, const float* d_iso, int32_t n_iso,
                       uint8_t* d_cases, float* d_segments, int32_t* d_seg_ids,
                       int64_t capacity, int64_t* h_count, void* stream);

/*
 * Allocation-free variant of mls_contour, for callers that cannot allocate
 * device or pinned memory during the call (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same segments,
 * ids and cases as mls_contour, bit for bit, with three differences:
 *  - the scratch is a fixed device array of MLS_CONTOUR_STATIC_SCRATCH_BYTES
 *    per GPU, held from the first context created on the GPU until the
 *    process ends; a call needs 4 (d n_iso chunks) + 8 tiles + 256 bytes of
 *    it, where chunks = ceil((height-1)(width-1) / 256) and tiles =
 *    ceil(d n_iso chunks / 1024), and returns MLS_ERR_INVALID_ARG for
 *    larger calls before enqueueing anything;
 *  - the required segment count goes to d_count, an int64 in device
 *    memory, written by the stream; the call does not wait for the stream;
 *  - when the count exceeds capacity, the first `capacity` segments (and
 *    ids) are still written, in order.
 * Every call on one GPU shares that GPU's array and overwrites what the
 * last call left there: calls that overlap on one GPU (other streams,
 * other threads, other contexts) race and must be ordered by the caller.
 * Nothing needs clearing between calls.  The context only names the device
 * (its own scratch is not used).
 */
#define MLS_CONTOUR_STATIC_SCRATCH_BYTES ((size_t)16 << 20)
mls_status mls_contour_static(mls_context* ctx, const float* d_fields, int32_t d,
                              const mls_grid* grid, const float* d_iso, int32_t n_iso,
                              uint8_t* d_cases, float* d_segments, int32_t* d_seg_ids,
                              int64_t capacity, int64_t* d_count, void* stream);

/*
 * Discrete colours (Sec. 3.4, Fig. 5b): per node, the band of its value --
 * the number of isovalues at or below it, the same tie rule as the contour
 * cases -- and optionally the band's colour.
 *  d_fields   float32 [d][height][width], device
 *  d_iso      float32 [d][n_iso], device (any order), 1 <= n_iso <= 254
 *  d_colormap uint32 [d][n_iso + 1] RGBA8 colour of each band, device, or
 *             NULL when d_rgba is NULL
 *  d_bands    uint8 [d][height][width] output (255 where the value is
 *             NaN), device, or NULL
 *  d_rgba     uint32 [d][height][width] output (0 where NaN), device, or
 *             NULL; at least one of d_bands, d_rgba
 * Enqueued on the stream; no scratch.
 */
mls_status mls_map_bands(mls_context* ctx, const float* d_fields, int32_t d,
                         const mls_grid* grid, const float* d_iso, int32_t n_iso,
                         const uint32_t* d_colormap, uint8_t* d_bands, uint32_t* d_rgba,
                         void* stream);

/* Adaptive contour lines (Sec. 3.4, Fig. 5d): lines fade in where space is
 * expanded (the field changes slowly per pixel) and out where it is
 * compressed.  Level j = 0 .. levels-1 has lines at origin + k spacing/2^j;
 * at a node with gradient g the field changes by r = |(g_x dx, g_y dy)|
 * per pixel, so level j's lines are s_j = (spacing / 2^j) / r pixels
 * apart.  Level 0 is always drawn; level j >= 1 with opacity
 * clamp((s_j - fade_lo) / (fade_hi - fade_lo), 0, 1).  The intensity is the
 * largest opacity x max(0, 1 - e_j / halfwidth) over the levels, e_j the
 * pixel distance to the nearest level-j line: in [0, 1], NaN where the
 * value is NaN, 0 where r is 0 or not finite. */
typedef struct {
  int32_t levels;     /* 1 .. 30 */
  double halfwidth;   /* line half-width in pixels, finite, > 0 */
  double fade_lo;     /* finite, fade_lo < fade_hi */
  double fade_hi;
} mls_adaptive_params;

/*
 *  d_fields    float32 [d][height][width], device
 *  d_grad      float32 [d][2][height][width] (d/dx, d/dy, as mls_fit_grad
 *              writes them), device
 *  d_levels    float32 [d][2] (origin, spacing of the level-0 lines),
 *              device
 *  d_intensity float32 [d][height][width] output, device
 * Enqueued on the stream; no scratch.
 */
mls_status mls_map_adaptive(mls_context* ctx, const float* d_fields, const float* d_grad,
                            int32_t d, const mls_grid* grid, const float* d_levels,
                            const mls_adaptive_params* params, float* d_intensity,
                            void* stream);

/* ------------------------------------------------------------------------ */
/* Served form: resident point sets and continuously batched fit requests    */
/* ------------------------------------------------------------------------ */
/*
 * The paper re-evaluates the MLS field on every interaction (Sec. 3.5,
 * Sec. 4.5).  A server keeps point sets resident on one device and runs fit
 * requests as they arrive, on `slots` execution slots (a stream and a
 * context with reserved scratch each).  Whenever a slot is free, a
 * scheduler thread gives it the request at the head of the queue together
 * with the later queued requests of the same kernel class (16-bit one-pass
 * fits with the Gaussian weight, no gradients and the format's default
 * lp_terms, of one degree, feature tiles per workgroup and format), in
 * arrival order, while their
 * staging fits the slot's scratch.  Such a batch runs as one persistent
 * kernel whose workgroups take (request, tile) work items from a device
 * counter; each request's completion flag lives in pinned host memory and
 * is set by the workgroup that finishes the request's last item, so
 * requests retire one by one while the batch runs on, and a request that
 * arrives meanwhile joins the next batch a slot takes.  Other requests
 * (MLS_PREC_F64, the Wendland weight, the two-pass bfloat16 form) run
 * alone on a slot.  Memory: resident point sets + slots x slot_scratch_bytes
 * (+ the tuner's reservation) <= hbm_budget_bytes; admitted requests
 * allocate nothing.  All server calls are thread-safe.  Results of a request
 * are bit-identical to mls_fit's with the same arguments, alone or among
 * others.  Timestamps are seconds since server creation (steady clock).
 */
typedef struct mls_server mls_server;

typedef struct {
  uint64_t pointset;      /* id from mls_server_put_points */
  int32_t basis;          /* mls_basis */
  mls_weight weight;
  mls_grid grid;
  int32_t precision;      /* mls_precision */
  mls_solve_opts opts;    /* zeros select nothing useful: set tau, floor */
  float* d_fields;        /* [d][height][width] output, caller-owned device */
  uint8_t* d_degree;      /* [height][width] output or NULL */
  double timeout_s;       /* > 0: cancel the request this many seconds after
                           * submit if it has not finished; 0: no timeout */
} mls_request;

typedef struct {
  int32_t status;         /* MLS_PENDING, MLS_OK, MLS_ERR_CANCELLED, or the
                           * fit's error status */
  double t_submit, t_admit, t_start, t_end;
  char detail[128];       /* error detail */
} mls_result;

/* Create a server on `device` with `slots` execution slots (1..64) of
 * `slot_scratch_bytes` reserved scratch each (see mls_fit_scratch_bytes;
 * a batch stages all its requests in one slot's scratch). */
mls_status mls_server_create(int32_t device, size_t hbm_budget_bytes, int32_t slots,
                             size_t slot_scratch_bytes, mls_server** out);
/* Wait for all submitted requests, then free everything. */
void mls_server_destroy(mls_server* srv);
/* Copy a point set (device or host pointers) into server memory; returns
 * once the copy is complete.  The source buffers must already hold their
 * values when the call is made: synchronise the stream that produced them
 * first (the server's streams are not ordered with the caller's). */
mls_status mls_server_put_points(mls_server* srv, const float* points, const float* values,
                                 int64_t n, int32_t d, uint64_t* pointset);
/* Drop a point set once no queued or running request (or tuning run) uses
 * it. */
mls_status mls_server_release_points(mls_server* srv, uint64_t pointset);
/* Queue a request (returns at once).  Every check of mls_fit is made here:
 * a request that mls_fit would refuse is refused with the same status.
 * MLS_ERR_OVER_BUDGET if its scratch exceeds a slot's.  The request's
 * output buffers are written from a server stream that is not ordered with
 * the caller's streams: work the caller queued on them must be complete at
 * submit, and they must not be read before the request has finished. */
mls_status mls_server_submit(mls_server* srv, const mls_request* req, uint64_t* ticket);
/* Cancel a queued or running request.  A queued request is dropped at once;
 * a batched request's remaining work items are skipped (items already
 * started finish), so its outputs are left partly written; a request
 * running alone on a slot completes.  Its result status is
 * MLS_ERR_CANCELLED, unless it had finished before the cancellation took
 * effect (then MLS_OK).  MLS_ERR_INVALID_ARG for an unknown or finished
 * ticket.  A request's timeout_s acts the same way. */
mls_status mls_server_cancel(mls_server* srv, uint64_t ticket);
/* MLS_PENDING while the request runs; MLS_OK once finished (the result is
 * written, the ticket retired; result.status holds the fit's status). */
mls_status mls_server_poll(mls_server* srv, uint64_t ticket, mls_result* out);
/* Block until the request finishes, then as mls_server_poll. */
mls_status mls_server_wait(mls_server* srv, uint64_t ticket, mls_result* out);
/* Detail of the calling thread's last failed server call. */
const char* mls_server_last_error(void);

/*
 * Autotuner of the served 16-bit fits (callers that serve many requests of
 * recurring shapes).  The node tile is fixed at 16 x 16 by the matrix
 * instruction; the tuned tile dimension is the feature axis: the attributes
 * per slab, which set the feature tiles of 16 columns a workgroup computes.
 * enable = 1: the first request of each shape class (precision, basis,
 * weight kind, D rounded up to a power of two, node count rounded up to a
 * power of four) is queued to a tuner thread, which times the candidate
 * widths (three interleaved rounds, the fastest time of each) on its own
 * stream, context and output buffer while the scheduler serves the class
 * with the library's plan; later requests of the class take the fastest
 * width if it beats the library's plan by at least 5%, else the plan.  The tuner's memory (2 x slot_scratch_bytes) is
 * reserved from the budget when tuning is first enabled
 * (MLS_ERR_OVER_BUDGET if it does not fit) and kept until the server is
 * destroyed; a request whose output does not fit it leaves its class on
 * the library's plan.  Requests that set opts.lp_slab themselves are not
 * tuned.  cache_path (may be NULL): a text file of "class = width" lines,
 * read now and rewritten whenever a class is added.  Tuning never changes a
 * result bit.
 */
mls_status mls_server_tuning(mls_server* srv, int32_t enable, const char* cache_path);

/* Number of shape classes the tuner holds. */
int64_t mls_server_tuned_classes(mls_server* srv);
/* Number of shape classes queued to or being timed by the tuner thread. */
int64_t mls_server_tuning_pending(mls_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* MLS_H_ */
