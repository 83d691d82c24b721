// Host side of the C ABI (include/mls.h): argument validation, contexts,
// dispatch to the kernels.  Every argument is checked before any HIP call,
// so a rejected call has no side effect on the device.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <new>
#include <string>
#include <vector>

#include "../../include/mls.h"
#include "mls_internal.h"

struct Scratch {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// One traced call: its stages' end events (after a start event) and what
// the JSON line reports about the call.
struct TraceCall {
  std::string call;
  int form = -1;
  std::string meta;                 // JSON members describing the request
  std::vector<hipEvent_t> ev;       // ev[0] start, ev[k] end of stage k
  std::vector<std::string> stages;  // stage k's name at stages[k - 1]
};

struct Tracing {
  bool on = false;
  std::string path;                 // JSON-lines file, or empty
  std::deque<TraceCall> pending;    // recorded, not yet read back
  mls_trace_record last{};
  bool have_last = false;
};

struct mls_context {
  int device;
  Tracing trace;
  // device scratch, grown on demand: contour counts, offsets, tile sums
  Scratch scratch;
  // fit staging: attribute ranges, shift/scale, normalised values
  Scratch fit_scratch;

  // pinned host word for counts read back by mls_contour
  int64_t* pinned = nullptr;

  // Both scratch buffers are shared by every call on the context, whatever
  // its stream: `last_use` is recorded after the last enqueued work that
  // touched them, on `last_stream`, and a call on another stream waits for
  // it before its own kernels run.
  hipEvent_t last_use = nullptr;
  hipStream_t last_stream = nullptr;
  bool used = false;
};

namespace {

thread_local char g_last_error[512] = "";

mls_status fail(mls_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return s;
}

mls_status device_fail(hipError_t e, const char* where) {
  return fail(MLS_ERR_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

bool is_finite(double v) { return std::isfinite(v); }

int max_d_for(int32_t basis) {
  switch (basis) {
    case MLS_BASIS_CONSTANT: return MLS_MAX_D_CONSTANT;
    case MLS_BASIS_LINEAR: return MLS_MAX_D_LINEAR;
    case MLS_BASIS_RIGID: return 2;
    default: return MLS_MAX_D_QUADRATIC;
  }
}

// Device pointers must belong to the context's device (or be managed).
mls_status check_device_ptr(const mls_context* ctx, const void* ptr, const char* name) {
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(MLS_ERR_INVALID_ARG, "%s is not a device pointer", name);
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    return fail(MLS_ERR_INVALID_ARG, "%s is not device memory", name);
  if (attr.type == hipMemoryTypeDevice && attr.device != ctx->device)
    return fail(MLS_ERR_INVALID_ARG, "%s lives on device %d, context is on %d", name,
                attr.device, ctx->device);
  return MLS_OK;
}

// Make sure `sc` holds at least `bytes`.
mls_status ensure_scratch(Scratch& sc, size_t bytes) {
  if (sc.bytes >= bytes) return MLS_OK;
  if (sc.ptr) {
    hipError_t e = hipFree(sc.ptr);  // synchronises with queued work
    sc.ptr = nullptr;
    sc.bytes = 0;
    if (e != hipSuccess) return device_fail(e, "hipFree");
  }
  size_t want = bytes < ((size_t)1 << 20) ? ((size_t)1 << 20) : bytes;
  hipError_t e = hipMalloc(&sc.ptr, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    sc.ptr = nullptr;
    return fail(MLS_ERR_OUT_OF_MEMORY, "scratch allocation of %zu bytes failed", want);
  }
  sc.bytes = want;
  return MLS_OK;
}

// Order this call's scratch use after the previous call's, when the two run
// on different streams.
mls_status scratch_acquire(mls_context* ctx, hipStream_t s) {
  if (ctx->used && ctx->last_stream != s) {
    hipError_t e = hipStreamWaitEvent(s, ctx->last_use, 0);
    if (e != hipSuccess) return device_fail(e, "hipStreamWaitEvent");
  }
  return MLS_OK;
}

mls_status scratch_release(mls_context* ctx, hipStream_t s) {
  hipError_t e = hipEventRecord(ctx->last_use, s);
  if (e != hipSuccess) return device_fail(e, "hipEventRecord");
  ctx->last_stream = s;
  ctx->used = true;
  return MLS_OK;
}

// ---- tracing: per-stage hipEvent timing behind mls_context_trace ----

void trace_destroy(TraceCall& c) {
  for (hipEvent_t e : c.ev) (void)hipEventDestroy(e);
  c.ev.clear();
}

// Wait for a traced call, turn its events into stage times, append its JSON
// line and keep it as the context's last record.
void trace_finalize(mls_context* ctx, TraceCall& c) {
  mls_trace_record r{};
  std::snprintf(r.call, sizeof(r.call), "%s", c.call.c_str());
  r.form = c.form;
  bool ok = !c.ev.empty() && hipEventSynchronize(c.ev.back()) == hipSuccess;
  double total = 0.0;
  const int ns = (int)c.stages.size() < MLS_TRACE_MAX_STAGES ? (int)c.stages.size()
                                                             : MLS_TRACE_MAX_STAGES;
  for (int k = 0; ok && k < ns; ++k) {
    float ms = 0.0f;
    ok = hipEventElapsedTime(&ms, c.ev[k], c.ev[k + 1]) == hipSuccess;
    std::snprintf(r.stage[k], sizeof(r.stage[k]), "%s", c.stages[k].c_str());
    r.ms[k] = ms;
    total += ms;
  }
  (void)hipGetLastError();
  trace_destroy(c);
  if (!ok) return;
  r.n_stages = ns;
  r.total_ms = total;
  ctx->trace.last = r;
  ctx->trace.have_last = true;
  if (ctx->trace.path.empty()) return;
  if (FILE* f = std::fopen(ctx->trace.path.c_str(), "a")) {
    std::fprintf(f, "{\"call\": \"%s\", \"form\": %d, %s\"stages_ms\": {", r.call, r.form,
                 c.meta.c_str());
    for (int k = 0; k < ns; ++k)
      std::fprintf(f, "%s\"%s\": %.6f", k ? ", " : "", r.stage[k], r.ms[k]);
    std::fprintf(f, "}, \"total_ms\": %.6f}\n", total);
    std::fclose(f);
  }
}

// Read back the pending calls whose last event has completed (all of them
// when `all`), oldest first.
void trace_drain(mls_context* ctx, bool all) {
  while (!ctx->trace.pending.empty()) {
    TraceCall& c = ctx->trace.pending.front();
    if (!all && hipEventQuery(c.ev.back()) != hipSuccess) {
      (void)hipGetLastError();
      if (ctx->trace.pending.size() < 64) break;   // keep at most 64 calls in flight
    }
    TraceCall done = std::move(c);
    ctx->trace.pending.pop_front();
    trace_finalize(ctx, done);
  }
}

// Records the stages of one call on its stream when the context traces.
class Tracer {
 public:
  Tracer(mls_context* ctx, hipStream_t s, const char* call, std::string meta)
      : ctx_(ctx), s_(s), on_(ctx->trace.on) {
    if (!on_) return;
    c_.call = call;
    c_.meta = std::move(meta);
    on_ = record();
  }
  ~Tracer() {
    if (on_) trace_destroy(c_);
  }
  // End of a stage that began at the previous mark.
  void mark(const char* stage) {
    if (!on_) return;
    c_.stages.emplace_back(stage);
    on_ = record();
    if (!on_) trace_destroy(c_);
  }
  void set_form(int form) { c_.form = form; }
  void finish() {
    if (!on_ || c_.stages.empty()) return;
    ctx_->trace.pending.push_back(std::move(c_));
    c_ = TraceCall();
    on_ = false;
    trace_drain(ctx_, false);
  }

 private:
  bool record() {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    c_.ev.push_back(e);
    if (hipEventRecord(e, s_) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    return true;
  }
  mls_context* ctx_;
  hipStream_t s_;
  bool on_;
  TraceCall c_;
};

std::string fit_meta(int64_t n, int32_t d, int32_t basis, int32_t wkind, const mls_grid* g,
                     int32_t precision) {
  char buf[256];
  std::snprintf(buf, sizeof(buf),
                "\"n\": %lld, \"d\": %d, \"basis\": %d, \"weight\": %d, \"width\": %d, "
                "\"height\": %d, \"precision\": %d, ",
                (long long)n, d, basis, wkind, g->width, g->height, precision);
  return buf;
}

}  // namespace

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

namespace mls {

// Device scratch layout of one mls_fit call (none for the float64 path).
FitPlan make_fit_plan(int64_t n, int32_t d, int32_t precision, int32_t wkind, double h,
                      double x0, double y0, double dx, double dy, int32_t W, int32_t H) {
  FitPlan p{};
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes, 256);
    return o;
  };
  if (precision == MLS_PREC_F64) {
    // the Gaussian's factor tables, when they fit the cap
    if (wkind == MLS_W_GAUSSIAN) {
      p.gtab_bytes = f64_table_bytes(n, W, H);
      if (p.gtab_bytes) p.o_gtab = carve(p.gtab_bytes);
    }
    // the inverse-distance weight's exact-hit pass sorts (node, point) keys
    if (wkind == MLS_W_INVPOW) {
      p.o_keys = carve(4 * (size_t)n);
      p.o_keys2 = carve(4 * (size_t)n);
      p.o_perm = carve(4 * (size_t)n);
      p.o_perm2 = carve(4 * (size_t)n);
      p.o_hist = carve(4 * 256 * (size_t)radix_blocks(n));
      p.o_ssum = carve(4 * (size_t)scan_sums_words(256 * radix_blocks(n)));
    }
    p.total = off;
    return p;
  }
  const int64_t nblk = stage_partial_blocks(n);
  p.o_pmin = carve(sizeof(float) * (size_t)(nblk * d));
  p.o_pmax = carve(sizeof(float) * (size_t)(nblk * d));
  p.o_shift = carve(sizeof(float) * (size_t)d);
  p.o_scale = carve(sizeof(float) * (size_t)d);
  p.o_vals = carve(sizeof(float) * (size_t)n * (size_t)d);
  if (wkind == MLS_W_WENDLAND_C2) {
    // cells of side >= h over the grid extent grown by h (points outside it
    // fall into the border cells, which is still exact: the weight decides,
    // the cells only bound the search)
    const double xa = x0, xb = x0 + (double)(W - 1) * dx;
    const double ya = y0, yb = y0 + (double)(H - 1) * dy;
    const double xmin = std::fmin(xa, xb), xmax = std::fmax(xa, xb);
    const double ymin = std::fmin(ya, yb), ymax = std::fmax(ya, yb);
    const double wx = (xmax - xmin) + 2.0 * h, wy = (ymax - ymin) + 2.0 * h;
    p.geom.cell = std::fmax(h, std::fmax(wx, wy) / 2048.0);
    p.geom.ox = xmin - h;
    p.geom.oy = ymin - h;
    p.geom.x0 = x0;
    p.geom.y0 = y0;
    p.geom.dx = dx;
    p.geom.dy = dy;
    p.geom.h = h;
    p.ncx = (int)std::floor(wx / p.geom.cell) + 1;
    p.ncy = (int)std::floor(wy / p.geom.cell) + 1;
    p.tiles_x = (W + kTileCols - 1) / kTileCols;
    p.tiles = p.tiles_x * ((H + kTileRows - 1) / kTileRows);
    const int64_t ncells = (int64_t)p.ncx * p.ncy;
    const int64_t nrb = radix_blocks(n), trb = radix_blocks(p.tiles);
    p.o_keys = carve(4 * (size_t)n);
    p.o_keys2 = carve(4 * (size_t)n);
    p.o_perm = carve(4 * (size_t)n);
    p.o_perm2 = carve(4 * (size_t)n);
    p.o_hist = carve(4 * 256 * (size_t)nrb);
    p.o_cs = carve(4 * (size_t)(ncells + 1));
    p.o_pts = carve(8 * (size_t)n);
    p.o_vals_s = carve(4 * (size_t)n * (size_t)d);
    p.o_tk = carve(4 * (size_t)p.tiles);
    p.o_tk2 = carve(4 * (size_t)p.tiles);
    p.order_slots = tile_order_slots(p.tiles_x, p.tiles / p.tiles_x);
    p.o_to = carve(4 * (size_t)p.order_slots);
    p.o_so = carve(4 * (size_t)p.tiles);
    int64_t scan_max = 256 * nrb;
    if (ncells + 1 > scan_max) scan_max = ncells + 1;
    if (p.tiles + 1 > scan_max) scan_max = p.tiles + 1;
    if (256 * trb > scan_max) scan_max = 256 * trb;
    p.o_ssum = carve(4 * (size_t)scan_sums_words(scan_max));
    p.o_to2 = carve(4 * (size_t)p.tiles);
    p.o_th = carve(4 * 256 * (size_t)trb);
    p.o_ts = carve(4 * (size_t)(p.tiles + 1));
    p.list_cap = tile_list_bound(n, h, dx, dy, p.tiles_x, p.tiles / p.tiles_x);
    p.o_tl = carve(4 * (size_t)p.list_cap);
  }
  p.total = off;
  return p;
}

size_t fit_scratch_bytes(int64_t n, int32_t d, int32_t precision, int32_t wkind, double h,
                         double x0, double y0, double dx, double dy, int32_t W, int32_t H) {
  return make_fit_plan(n, d, precision, wkind, h, x0, y0, dx, dy, W, H).total;
}

}  // namespace mls

extern "C" {

const char* mls_status_string(mls_status s) {
  switch (s) {
    case MLS_OK: return "MLS_OK";
    case MLS_ERR_INVALID_ARG: return "MLS_ERR_INVALID_ARG";
    case MLS_ERR_OUT_OF_MEMORY: return "MLS_ERR_OUT_OF_MEMORY";
    case MLS_ERR_CAPACITY: return "MLS_ERR_CAPACITY";
    case MLS_ERR_DEVICE: return "MLS_ERR_DEVICE";
    case MLS_ERR_OVER_BUDGET: return "MLS_ERR_OVER_BUDGET";
    case MLS_ERR_CANCELLED: return "MLS_ERR_CANCELLED";
    case MLS_ERR_UNSUPPORTED: return "MLS_ERR_UNSUPPORTED";
    case MLS_PENDING: return "MLS_PENDING";
  }
  return "MLS_UNKNOWN_STATUS";
}

const char* mls_last_error(void) { return g_last_error; }

mls_status mls_context_create(int32_t device, mls_context** out) {
  g_last_error[0] = '\0';
  if (!out) return fail(MLS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return device_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= count)
    return fail(MLS_ERR_DEVICE, "device %d out of range (%d devices)", device, count);
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return device_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(MLS_ERR_DEVICE, "device %d is %s; this library is built for gfx950", device,
                prop.gcnArchName);
  e = hipSetDevice(device);
  if (e != hipSuccess) return device_fail(e, "hipSetDevice");
  mls_context* ctx = new (std::nothrow) mls_context;
  if (!ctx) return fail(MLS_ERR_OUT_OF_MEMORY, "host allocation failed");
  ctx->device = device;
  e = hipEventCreateWithFlags(&ctx->last_use, hipEventDisableTiming);
  if (e != hipSuccess) {
    delete ctx;
    return device_fail(e, "hipEventCreateWithFlags");
  }
  // the fixed scratch of mls_contour_static: its address on this device
  e = mls::contour_static_scratch_resolve(device);
  if (e != hipSuccess) {
    (void)hipEventDestroy(ctx->last_use);
    delete ctx;
    return device_fail(e, "hipGetSymbolAddress (contour scratch)");
  }
  *out = ctx;
  return MLS_OK;
}

void mls_context_destroy(mls_context* ctx) {
  if (!ctx) return;
  if (hipSetDevice(ctx->device) == hipSuccess) {
    for (TraceCall& c : ctx->trace.pending) trace_destroy(c);
    if (ctx->scratch.ptr) (void)hipFree(ctx->scratch.ptr);
    if (ctx->fit_scratch.ptr) (void)hipFree(ctx->fit_scratch.ptr);

    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->last_use) (void)hipEventDestroy(ctx->last_use);
  }
  delete ctx;
}

}  // extern "C"

namespace mls {

// Every check of mls_fit / mls_fit_grad (arguments, then the device
// pointers), and the fit's arguments, without enqueueing anything.
mls_status fit_prepare(mls_context* ctx, const float* d_points, const float* d_values, int64_t n,
                       int32_t d, int32_t basis, const mls_weight* weight, const mls_grid* grid,
                       int32_t precision, const mls_solve_opts* opts, float* d_fields,
                       float* d_grad, uint8_t* d_degree, FitArgs* out, int* terms_out) {
  // ---- arguments, checked without touching the device ----
  if (basis < MLS_BASIS_CONSTANT || basis > MLS_BASIS_RIGID)
    return fail(MLS_ERR_INVALID_ARG, "basis %d is not an mls_basis", basis);
  if (basis == MLS_BASIS_RIGID && d != 2)
    return fail(MLS_ERR_INVALID_ARG, "d = %d; the rigid map takes 2-vector values", d);
  if (n < 1) return fail(MLS_ERR_INVALID_ARG, "n = %lld; need at least one point", (long long)n);
  if (n > MLS_MAX_N) return fail(MLS_ERR_INVALID_ARG, "n = %lld is too large", (long long)n);
  if (precision < MLS_PREC_F64 || precision > MLS_PREC_FP16)
    return fail(MLS_ERR_INVALID_ARG, "precision %d is not an mls_precision", precision);
  const int dmax = precision == MLS_PREC_F64 ? max_d_for(basis) : MLS_MAX_D_LP;
  if (d < 1 || d > dmax)
    return fail(MLS_ERR_INVALID_ARG, "d = %d; basis %d with precision %d accepts 1..%d attributes",
                d, basis, precision, dmax);
  if (!weight) return fail(MLS_ERR_INVALID_ARG, "weight is NULL");
  if (weight->kind < MLS_W_GAUSSIAN || weight->kind > MLS_W_INVPOW)
    return fail(MLS_ERR_INVALID_ARG, "weight kind %d is not an mls_weight_kind", weight->kind);
  if (!is_finite(weight->h) || !(weight->h > 0.0))
    return fail(MLS_ERR_INVALID_ARG, "h = %g; need a finite h > 0", weight->h);
  if (weight->kind == MLS_W_INVPOW && (!is_finite(weight->alpha) || !(weight->alpha > 0.0)))
    return fail(MLS_ERR_INVALID_ARG, "alpha = %g; need a finite alpha > 0", weight->alpha);
  if (!grid) return fail(MLS_ERR_INVALID_ARG, "grid is NULL");
  if (grid->width < 1 || grid->height < 1)
    return fail(MLS_ERR_INVALID_ARG, "grid %d x %d; need width, height >= 1", grid->width,
                grid->height);
  if ((int64_t)grid->width * grid->height > ((int64_t)1 << 31))
    return fail(MLS_ERR_INVALID_ARG, "grid %d x %d has more than 2^31 nodes", grid->width,
                grid->height);
  if (!is_finite(grid->x0) || !is_finite(grid->y0) || !is_finite(grid->dx) || !is_finite(grid->dy))
    return fail(MLS_ERR_INVALID_ARG, "grid origin and spacing must be finite");
  double tau = 1e-8, floor_w = 1e-6;
  int terms = precision == MLS_PREC_FP16 ? 2 : 3;
  int slab = 0, form = 0;
  if (opts) {
    tau = opts->pivot_tol;
    floor_w = opts->weight_floor;
    if (opts->lp_terms < 0 || opts->lp_terms > 3)
      return fail(MLS_ERR_INVALID_ARG, "lp_terms = %d; need 0..3", opts->lp_terms);
    if (opts->lp_terms > 0) terms = opts->lp_terms;
    const int max_slab = basis == MLS_BASIS_QUADRATIC ? MLS_LP_MAX_SLAB_QUADRATIC
                         : basis == MLS_BASIS_LINEAR  ? MLS_LP_MAX_SLAB_LINEAR
                                                      : MLS_LP_MAX_SLAB_CONSTANT;
    if (opts->lp_slab < 0 || opts->lp_slab > max_slab)
      return fail(MLS_ERR_INVALID_ARG, "lp_slab = %d; need 0..%d for this basis", opts->lp_slab,
                  max_slab);
    slab = opts->lp_slab;
    if (opts->lp_form < 0 || opts->lp_form > 2)
      return fail(MLS_ERR_INVALID_ARG, "lp_form = %d; need 0..2", opts->lp_form);
    form = opts->lp_form;
    if (!is_finite(tau) || !(tau > 0.0) || !(tau <= 1.0))
      return fail(MLS_ERR_INVALID_ARG, "pivot_tol = %g; need 0 < tau <= 1", tau);
    if (!is_finite(floor_w) || floor_w < 0.0)
      return fail(MLS_ERR_INVALID_ARG, "weight_floor = %g; need a finite value >= 0", floor_w);
  }
  if (!d_points) return fail(MLS_ERR_INVALID_ARG, "d_points is NULL");
  if (!d_values) return fail(MLS_ERR_INVALID_ARG, "d_values is NULL");
  if (!d_fields) return fail(MLS_ERR_INVALID_ARG, "d_fields is NULL");
  if (!ctx) return fail(MLS_ERR_INVALID_ARG, "ctx is NULL");
  if ((weight->kind == MLS_W_INVPOW && precision != MLS_PREC_F64) ||
      (weight->kind == MLS_W_WENDLAND_C2 && precision == MLS_PREC_F64))
    return fail(MLS_ERR_UNSUPPORTED, "weight kind %d is not available with precision %d",
                weight->kind, precision);
  if (basis == MLS_BASIS_RIGID &&
      (precision != MLS_PREC_F64 || weight->kind == MLS_W_WENDLAND_C2 || d_grad))
    return fail(MLS_ERR_UNSUPPORTED, "the rigid map runs on MLS_PREC_F64 with the Gaussian or "
                "inverse-distance weight, without gradients");
  if (weight->kind == MLS_W_INVPOW && (grid->dx == 0.0 || grid->dy == 0.0))
    return fail(MLS_ERR_UNSUPPORTED, "the inverse-distance weight needs nonzero grid spacing "
                "(nodes on one position would share their exact hits)");

  if (precision != MLS_PREC_F64) {
    // The 16-bit contraction accumulates moments in a frame shared by a
    // 16 x 16 node tile; moving them to a node far from the frame's origin
    // cancels digits the float32 accumulator cannot spare (the constant basis
    // has no frame-dependent moments).  Grids that coarse against h are small:
    // the float64 path serves them.
    const double extent = mls::lp_tile_extent(grid->dx, grid->dy, weight->h);
    const double span_max = basis == MLS_BASIS_QUADRATIC ? MLS_LP_MAX_TILE_SPAN_QUADRATIC
                            : basis == MLS_BASIS_LINEAR  ? MLS_LP_MAX_TILE_SPAN_LINEAR
                                                         : HUGE_VAL;
    if (extent > span_max * (1.0 + 1e-12))
      return fail(MLS_ERR_UNSUPPORTED, "a 16 x 16 node tile spans %.2f h (> %.1f h for this "
                  "basis); use MLS_PREC_F64 for grids this coarse against h", extent, span_max);
    if (precision == MLS_PREC_FP16) {
      // tile-frame features reach |u| <= 8 + half the tile diagonal (in h);
      // the largest, u^4 times an attribute in [-1, 1], must stay finite
      const double sx = grid->dx / weight->h, sy = grid->dy / weight->h;
      const double reach = 8.0 + 0.5 * std::sqrt(256.0 * (sx * sx + sy * sy));
      const double big = basis == MLS_BASIS_QUADRATIC ? reach * reach * reach * reach
                         : (basis == MLS_BASIS_LINEAR ? reach * reach : 1.0);
      if (big > 6.0e4)
        return fail(MLS_ERR_UNSUPPORTED, "grid spacing %g x %g is too coarse against h = %g for "
                    "float16 features", grid->dx, grid->dy, weight->h);
    }
    if (weight->kind == MLS_W_WENDLAND_C2 &&
        mls::make_fit_plan(n, d, precision, weight->kind, weight->h, grid->x0, grid->y0, grid->dx,
                           grid->dy, grid->width, grid->height).list_cap > (int64_t)0xFFFFFFFFu)
      return fail(MLS_ERR_UNSUPPORTED, "the per-tile point lists of %lld points with h = %g on "
                  "this grid could exceed 2^32 entries", (long long)n, weight->h);
  }

  // ---- device ----
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return device_fail(e, "hipSetDevice");
  mls_status st;
  if ((st = check_device_ptr(ctx, d_points, "d_points")) != MLS_OK) return st;
  if ((st = check_device_ptr(ctx, d_values, "d_values")) != MLS_OK) return st;
  if ((st = check_device_ptr(ctx, d_fields, "d_fields")) != MLS_OK) return st;
  if (d_degree && (st = check_device_ptr(ctx, d_degree, "d_degree")) != MLS_OK) return st;
  if (d_grad && (st = check_device_ptr(ctx, d_grad, "d_grad")) != MLS_OK) return st;

  mls::FitArgs a;
  a.pts = d_points;
  a.vals = d_values;
  a.n = n;
  a.D = d;
  a.degree = basis == MLS_BASIS_RIGID ? MLS_BASIS_LINEAR : basis;
  a.rigid = basis == MLS_BASIS_RIGID;
  a.wkind = weight->kind;
  a.h = weight->h;
  a.alpha = weight->alpha;
  a.x0 = grid->x0;
  a.y0 = grid->y0;
  a.dx = grid->dx;
  a.dy = grid->dy;
  a.W = grid->width;
  a.H = grid->height;
  a.tau = tau;
  a.floor_w = floor_w;
  a.lp_slab = slab;
  a.fields = d_fields;
  a.deg_out = d_degree;
  a.grads = d_grad;
  a.lp_form = form;
  a.gtab = nullptr;
  *out = a;
  *terms_out = terms;
  return MLS_OK;
}

void* context_scratch(void* ctx, size_t* bytes) {
  mls_context* c = (mls_context*)ctx;
  *bytes = c->fit_scratch.bytes;
  return c->fit_scratch.ptr;
}

mls_status_t fit_prepare_c(void* ctx, const float* d_points, const float* d_values, int64_t n,
                           int32_t d, int32_t basis, const void* weight, const void* grid,
                           int32_t precision, const void* opts, float* d_fields, float* d_grad,
                           uint8_t* d_degree, FitArgs* out, int* terms) {
  g_last_error[0] = '\0';
  return fit_prepare((mls_context*)ctx, d_points, d_values, n, d, basis,
                     (const mls_weight*)weight, (const mls_grid*)grid, precision,
                     (const mls_solve_opts*)opts, d_fields, d_grad, d_degree, out, terms);
}

}  // namespace mls

extern "C" {

// mls_fit and mls_fit_grad: d_grad (slopes of the local fits) may be NULL.
static mls_status fit_impl(mls_context* ctx, const float* d_points, const float* d_values,
                           int64_t n, int32_t d, int32_t basis, const mls_weight* weight,
                           const mls_grid* grid, int32_t precision,
                           const mls_solve_opts* opts, float* d_fields, float* d_grad,
                           uint8_t* d_degree, void* stream) {
  mls::FitArgs a;
  int terms = 0;
  mls_status st = mls::fit_prepare(ctx, d_points, d_values, n, d, basis, weight, grid, precision,
                                   opts, d_fields, d_grad, d_degree, &a, &terms);
  if (st != MLS_OK) return st;
  const int form = a.lp_form;
  hipError_t e;
  hipStream_t s = (hipStream_t)stream;
  Tracer tr(ctx, s, d_grad ? "fit_grad" : "fit",
            fit_meta(n, d, basis, weight->kind, grid, precision));
  if (precision == MLS_PREC_F64) {
    const mls::FitPlan plan = mls::make_fit_plan(n, d, precision, weight->kind, weight->h,
                                                 grid->x0, grid->y0, grid->dx, grid->dy,
                                                 grid->width, grid->height);
    if (plan.total > 0) {
      if ((st = ensure_scratch(ctx->fit_scratch, plan.total)) != MLS_OK) return st;
      if ((st = scratch_acquire(ctx, s)) != MLS_OK) return st;
      if (plan.gtab_bytes) a.gtab = (double*)((char*)ctx->fit_scratch.ptr + plan.o_gtab);
    }
    e = mls::launch_fit_f64(a, s);
    if (e != hipSuccess) return device_fail(e, "fit kernel launch");
    tr.set_form(0);
    tr.mark("contract");
    if (weight->kind == MLS_W_INVPOW) {
      char* base = (char*)ctx->fit_scratch.ptr;
      mls::HitArgs hta;
      hta.pts = d_points;
      hta.vals = d_values;
      hta.n = n;
      hta.D = d;
      hta.x0 = grid->x0;
      hta.y0 = grid->y0;
      hta.dx = grid->dx;
      hta.dy = grid->dy;
      hta.W = grid->width;
      hta.H = grid->height;
      hta.fields = d_fields;
      hta.deg_out = d_degree;
      hta.grads = d_grad;
      hta.keys = (uint32_t*)(base + plan.o_keys);
      hta.keys2 = (uint32_t*)(base + plan.o_keys2);
      hta.idx = (uint32_t*)(base + plan.o_perm);
      hta.idx2 = (uint32_t*)(base + plan.o_perm2);
      hta.hist = (uint32_t*)(base + plan.o_hist);
      hta.ssum = (uint32_t*)(base + plan.o_ssum);
      e = mls::launch_hits(hta, s);
      if (e != hipSuccess) return device_fail(e, "exact-hit pass launch");
      tr.mark("hits");
      tr.finish();
      return scratch_release(ctx, s);
    }
    tr.finish();
    return plan.total > 0 ? scratch_release(ctx, s) : MLS_OK;
  }
  const bool fp16 = precision == MLS_PREC_FP16;
  const mls::FitPlan plan = mls::make_fit_plan(n, d, precision, weight->kind, weight->h,
                                               grid->x0, grid->y0, grid->dx, grid->dy,
                                               grid->width, grid->height);
  if ((st = ensure_scratch(ctx->fit_scratch, plan.total)) != MLS_OK) return st;
  if ((st = scratch_acquire(ctx, s)) != MLS_OK) return st;
  char* base = (char*)ctx->fit_scratch.ptr;
  float* pmin = (float*)(base + plan.o_pmin);
  float* pmax = (float*)(base + plan.o_pmax);
  float* shift = (float*)(base + plan.o_shift);
  float* scale = (float*)(base + plan.o_scale);
  float* vals_t = (float*)(base + plan.o_vals);
  e = mls::launch_stage(d_values, n, d, pmin, pmax, shift, scale, vals_t, s);
  if (e != hipSuccess) return device_fail(e, "staging kernel launch");
  tr.mark("stage");
  tr.set_form(mls::lp_use_shape_form(a.degree, d, fp16, weight->kind, d_grad != nullptr, terms,
                                     0, form) ? 2 : 1);
  if (weight->kind != MLS_W_WENDLAND_C2) {
    e = mls::launch_fit_lp(a, vals_t, shift, scale, fp16, terms, nullptr, s);
    if (e != hipSuccess) return device_fail(e, "fit kernel launch");
    tr.mark("contract");
    tr.finish();
    return scratch_release(ctx, s);
  }
  mls::CellArgs ca;
  ca.pts = d_points;
  ca.vals_t = vals_t;
  ca.n = n;
  ca.D = d;
  ca.geom = plan.geom;
  ca.ncx = plan.ncx;
  ca.ncy = plan.ncy;
  ca.tiles_x = plan.tiles_x;
  ca.tiles = plan.tiles;
  ca.cell_start = (uint32_t*)(base + plan.o_cs);
  ca.perm = (uint32_t*)(base + plan.o_perm);
  ca.pts_s = (float*)(base + plan.o_pts);
  ca.vals_ts = (float*)(base + plan.o_vals_s);
  ca.torder = (uint32_t*)(base + plan.o_to);
  ca.keys = (uint32_t*)(base + plan.o_keys);
  ca.keys2 = (uint32_t*)(base + plan.o_keys2);
  ca.perm2 = (uint32_t*)(base + plan.o_perm2);
  ca.hist = (uint32_t*)(base + plan.o_hist);
  ca.tkeys = (uint32_t*)(base + plan.o_tk);
  ca.tkeys2 = (uint32_t*)(base + plan.o_tk2);
  ca.torder2 = (uint32_t*)(base + plan.o_to2);
  ca.thist = (uint32_t*)(base + plan.o_th);
  ca.sorder = (uint32_t*)(base + plan.o_so);
  ca.ssum = (uint32_t*)(base + plan.o_ssum);
  ca.tile_start = (uint32_t*)(base + plan.o_ts);
  ca.tile_list = (uint32_t*)(base + plan.o_tl);
  ca.list_cap = plan.list_cap;
  e = mls::launch_cells(ca, s);
  if (e != hipSuccess) return device_fail(e, "cell list kernels");
  tr.mark("cells");
  mls::LPCells cl;
  cl.pts_s = ca.pts_s;
  cl.vals_ts = ca.vals_ts;
  cl.cell_start = ca.cell_start;
  cl.torder = ca.torder;
  cl.tile_start = ca.tile_start;
  cl.tile_list = ca.tile_list;
  cl.ncx = plan.ncx;
  cl.ncy = plan.ncy;
  cl.geom = plan.geom;
  e = mls::launch_fit_lp(a, vals_t, shift, scale, fp16, terms, &cl, s);
  if (e != hipSuccess) return device_fail(e, "fit kernel launch");
  tr.mark("contract");
  tr.finish();
  return scratch_release(ctx, s);
}

mls_status mls_layout(mls_context* ctx, float* d_pos, int64_t n, const int32_t* d_adj_start,
                      const int32_t* d_adj, int64_t n_adj, const int32_t* d_fan_start,
                      const int32_t* d_fan, int64_t n_fan, const mls_layout_params* params,
                      int32_t iterations, void* stream) {
  g_last_error[0] = '\0';
  if (n < 1 || n > ((int64_t)1 << 30))
    return fail(MLS_ERR_INVALID_ARG, "n = %lld; need 1 .. 2^30 nodes", (long long)n);
  if (n_adj < 0 || n_fan < 0 || n_adj > ((int64_t)1 << 31) || n_fan > ((int64_t)1 << 30))
    return fail(MLS_ERR_INVALID_ARG, "n_adj = %lld, n_fan = %lld", (long long)n_adj,
                (long long)n_fan);
  if (iterations < 0) return fail(MLS_ERR_INVALID_ARG, "iterations = %d", iterations);
  if (!params) return fail(MLS_ERR_INVALID_ARG, "params is NULL");
  const mls_layout_params& q = *params;
  if (!is_finite(q.C) || !(q.C >= 0.0) || !is_finite(q.D) || !(q.D > 0.0) ||
      !is_finite(q.eta) || !(q.eta > 0.0) || !is_finite(q.t0) || !(q.t0 >= 0.0) ||
      !is_finite(q.lambda) || !(q.lambda > 0.0) || !(q.lambda <= 1.0))
    return fail(MLS_ERR_INVALID_ARG, "layout parameters: need C >= 0, D > 0, eta > 0, t0 >= 0, "
                "0 < lambda <= 1, all finite");
  if (!d_pos || !d_adj_start || !d_fan_start || (n_adj > 0 && !d_adj) || (n_fan > 0 && !d_fan))
    return fail(MLS_ERR_INVALID_ARG, "a required device array is NULL");
  if (!ctx) return fail(MLS_ERR_INVALID_ARG, "ctx is NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return device_fail(e, "hipSetDevice");
  mls_status st;
  if ((st = check_device_ptr(ctx, d_pos, "d_pos")) != MLS_OK) return st;
  if ((st = check_device_ptr(ctx, d_adj_start, "d_adj_start")) != MLS_OK) return st;
  if ((st = check_device_ptr(ctx, d_fan_start, "d_fan_start")) != MLS_OK) return st;
  if (n_adj > 0 && (st = check_device_ptr(ctx, d_adj, "d_adj")) != MLS_OK) return st;
  if (n_fan > 0 && (st = check_device_ptr(ctx, d_fan, "d_fan")) != MLS_OK) return st;
  const size_t half = align_up(sizeof(double) * 2 * (size_t)n, 256);
  if ((st = ensure_scratch(ctx->fit_scratch, 2 * half)) != MLS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = scratch_acquire(ctx, s)) != MLS_OK) return st;
  mls::LayoutArgs a;
  a.pos = d_pos;
  a.n = n;
  a.adj_start = d_adj_start;
  a.adj = d_adj;
  a.n_adj = n_adj;
  a.fan_start = d_fan_start;
  a.fan = d_fan;
  a.n_fan = n_fan;
  a.C = q.C;
  a.D = q.D;
  a.eta = q.eta;
  a.t0 = q.t0;
  a.lambda = q.lambda;
  a.iterations = iterations;
  a.buf0 = (double*)ctx->fit_scratch.ptr;
  a.buf1 = (double*)((char*)ctx->fit_scratch.ptr + half);
  char meta[96];
  std::snprintf(meta, sizeof(meta), "\"n\": %lld, \"iterations\": %d, ", (long long)n,
                iterations);
  Tracer tr(ctx, s, "layout", meta);
  e = mls::launch_layout(a, s);
  if (e != hipSuccess) return device_fail(e, "layout kernel launch");
  tr.mark("iterations");
  tr.finish();
  return scratch_release(ctx, s);
}

// Grid checks shared by the mappings.
static mls_status map_grid_check(const mls_grid* grid, int32_t d) {
  if (d < 1) return fail(MLS_ERR_INVALID_ARG, "d = %d; need at least one field", d);
  if (!grid) return fail(MLS_ERR_INVALID_ARG, "grid is NULL");
  if (grid->width < 1 || grid->height < 1)
    return fail(MLS_ERR_INVALID_ARG, "grid %d x %d; need width, height >= 1", grid->width,
                grid->height);
  if (!is_finite(grid->dx) || !is_finite(grid->dy))
    return fail(MLS_ERR_INVALID_ARG, "grid spacing must be finite");
  return MLS_OK;
}

mls_status mls_map_bands(mls_context* ctx, const float* d_fields, int32_t d,
                         const mls_grid* grid, const float* d_iso, int32_t n_iso,
                         const uint32_t* d_colormap, uint8_t* d_bands, uint32_t* d_rgba,
                         void* stream) {
  g_last_error[0] = '\0';
  mls_status st = map_grid_check(grid, d);
  if (st != MLS_OK) return st;
  if (n_iso < 1 || n_iso > 254)
    return fail(MLS_ERR_INVALID_ARG, "n_iso = %d; need 1 .. 254", n_iso);
  if (!d_fields) return fail(MLS_ERR_INVALID_ARG, "d_fields is NULL");
  if (!d_iso) return fail(MLS_ERR_INVALID_ARG, "d_iso is NULL");
  if (!d_bands && !d_rgba) return fail(MLS_ERR_INVALID_ARG, "d_bands and d_rgba are both NULL");
  if (d_rgba && !d_colormap) return fail(MLS_ERR_INVALID_ARG, "d_rgba needs d_colormap");
  if (!ctx) return fail(MLS_ERR_INVALID_ARG, "ctx is NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return device_fail(e, "hipSetDevice");
  if ((st = check_device_ptr(ctx, d_fields, "d_fields")) != MLS_OK) return st;
  if ((st = check_device_ptr(ctx, d_iso, "d_iso")) != MLS_OK) return st;
  if (d_colormap && (st = check_device_ptr(ctx, d_colormap, "d_colormap")) != MLS_OK) return st;
  if (d_bands && (st = check_device_ptr(ctx, d_bands, "d_bands")) != MLS_OK) return st;
  if (d_rgba && (st = check_device_ptr(ctx, d_rgba, "d_rgba")) != MLS_OK) return st;
  mls::MapBandsArgs a;
  a.fields = d_fields;
  a.iso = d_iso;
  a.colormap = d_colormap;
  a.D = d;
  a.n_iso = n_iso;
  a.P = (int64_t)grid->width * grid->height;
  a.bands = d_bands;
  a.rgba = d_rgba;
  hipStream_t s = (hipStream_t)stream;
  char meta[128];
  std::snprintf(meta, sizeof(meta), "\"d\": %d, \"n_iso\": %d, \"width\": %d, \"height\": %d, ",
                d, n_iso, grid->width, grid->height);
  Tracer tr(ctx, s, "map_bands", meta);
  e = mls::launch_map_bands(a, s);
  if (e != hipSuccess) return device_fail(e, "band kernel launch");
  tr.mark("bands");
  tr.finish();
  return MLS_OK;
}

mls_status mls_map_adaptive(mls_context* ctx, const float* d_fields, const float* d_grad,
                            int32_t d, const mls_grid* grid, const float* d_levels,
                            const mls_adaptive_params* params, float* d_intensity,
                            void* stream) {
  g_last_error[0] = '\0';
  mls_status st = map_grid_check(grid, d);
  if (st != MLS_OK) return st;
  if (!params) return fail(MLS_ERR_INVALID_ARG, "params is NULL");
  if (params->levels < 1 || params->levels > 30)
    return fail(MLS_ERR_INVALID_ARG, "levels = %d; need 1 .. 30", params->levels);
  if (!is_finite(params->halfwidth) || !(params->halfwidth > 0.0))
    return fail(MLS_ERR_INVALID_ARG, "halfwidth = %g; need a finite value > 0", params->halfwidth);
  if (!is_finite(params->fade_lo) || !is_finite(params->fade_hi) ||
      !(params->fade_hi > params->fade_lo))
    return fail(MLS_ERR_INVALID_ARG, "fade_lo = %g, fade_hi = %g; need finite fade_lo < fade_hi",
                params->fade_lo, params->fade_hi);
  if (!d_fields || !d_grad || !d_levels || !d_intensity)
    return fail(MLS_ERR_INVALID_ARG, "a required device array is NULL");
  if (!ctx) return fail(MLS_ERR_INVALID_ARG, "ctx is NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return device_fail(e, "hipSetDevice");
  if ((st = check_device_ptr(ctx, d_fields, "d_fields")) != MLS_OK) return st;
  if ((st = check_device_ptr(ctx, d_grad, "d_grad")) != MLS_OK) return st;
  if ((st = check_device_ptr(ctx, d_levels, "d_levels")) != MLS_OK) return st;
  if ((st = check_device_ptr(ctx, d_intensity, "d_intensity")) != MLS_OK) return st;
  mls::MapAdaptiveArgs a;
  a.fields = d_fields;
  a.grads = d_grad;
  a.levels = d_levels;
  a.D = d;
  a.n_levels = params->levels;
  a.P = (int64_t)grid->width * grid->height;
  a.dx = grid->dx;
  a.dy = grid->dy;
  a.halfwidth = params->halfwidth;
  a.fade_lo = params->fade_lo;
  a.fade_hi = params->fade_hi;
  a.out = d_intensity;
  hipStream_t s = (hipStream_t)stream;
  char meta[128];
  std::snprintf(meta, sizeof(meta), "\"d\": %d, \"levels\": %d, \"width\": %d, \"height\": %d, ",
                d, params->levels, grid->width, grid->height);
  Tracer tr(ctx, s, "map_adaptive", meta);
  e = mls::launch_map_adaptive(a, s);
  if (e != hipSuccess) return device_fail(e, "adaptive line kernel launch");
  tr.mark("lines");
  tr.finish();
  return MLS_OK;
}

mls_status mls_context_trace(mls_context* ctx, int32_t enable, const char* jsonl_path) {
  g_last_error[0] = '\0';
  if (!ctx) return fail(MLS_ERR_INVALID_ARG, "ctx is NULL");
  if (enable != 0 && enable != 1) return fail(MLS_ERR_INVALID_ARG, "enable = %d", enable);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return device_fail(e, "hipSetDevice");
  trace_drain(ctx, true);
  if (jsonl_path && jsonl_path[0]) {
    FILE* f = std::fopen(jsonl_path, "a");
    if (!f) return fail(MLS_ERR_INVALID_ARG, "cannot open %s for appending", jsonl_path);
    std::fclose(f);
  }
  ctx->trace.on = enable == 1;
  ctx->trace.path = jsonl_path ? jsonl_path : "";
  return MLS_OK;
}

mls_status mls_context_trace_last(mls_context* ctx, mls_trace_record* out) {
  g_last_error[0] = '\0';
  if (!ctx || !out) return fail(MLS_ERR_INVALID_ARG, "ctx or out is NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return device_fail(e, "hipSetDevice");
  trace_drain(ctx, true);
  if (!ctx->trace.have_last) return fail(MLS_ERR_INVALID_ARG, "no traced call on this context");
  *out = ctx->trace.last;
  return MLS_OK;
}

mls_status mls_context_reserve(mls_context* ctx, size_t bytes) {
  g_last_error[0] = '\0';
  if (!ctx) return fail(MLS_ERR_INVALID_ARG, "ctx is NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return device_fail(e, "hipSetDevice");
  return ensure_scratch(ctx->fit_scratch, bytes);
}

mls_status mls_fit(mls_context* ctx, const float* d_points, const float* d_values,
                   int64_t n, int32_t d, int32_t basis, const mls_weight* weight,
                   const mls_grid* grid, int32_t precision, const mls_solve_opts* opts,
                   float* d_fields, uint8_t* d_degree, void* stream) {
  g_last_error[0] = '\0';
  return fit_impl(ctx, d_points, d_values, n, d, basis, weight, grid, precision, opts, d_fields,
                  nullptr, d_degree, stream);
}

mls_status mls_fit_grad(mls_context* ctx, const float* d_points, const float* d_values,
                        int64_t n, int32_t d, int32_t basis, const mls_weight* weight,
                        const mls_grid* grid, int32_t precision, const mls_solve_opts* opts,
                        float* d_fields, float* d_grad, uint8_t* d_degree, void* stream) {
  g_last_error[0] = '\0';
  if (!d_grad) return fail(MLS_ERR_INVALID_ARG, "d_grad is NULL");
  return fit_impl(ctx, d_points, d_values, n, d, basis, weight, grid, precision, opts, d_fields,
                  d_grad, d_degree, stream);
}

size_t mls_fit_scratch_bytes(int64_t n, int32_t d, int32_t precision, const mls_weight* weight,
                             const mls_grid* grid) {
  if (!weight || !grid || n < 1 || d < 1) return 0;
  return mls::make_fit_plan(n, d, precision, weight->kind, weight->h, grid->x0, grid->y0,
                            grid->dx, grid->dy, grid->width, grid->height)
      .total;
}

// Arguments of mls_contour / mls_contour_static, checked before any device
// work; `count` is h_count or d_count.
static mls_status contour_check(mls_context* ctx, const float* d_fields, int32_t d,
                                const mls_grid* grid, const float* d_iso, int32_t n_iso,
                                uint8_t* d_cases, float* d_segments, int32_t* d_seg_ids,
                                int64_t capacity, const int64_t* count,
                                const char* count_name) {
  if (d < 1) return fail(MLS_ERR_INVALID_ARG, "d = %d; need at least one field", d);
  if (!grid) return fail(MLS_ERR_INVALID_ARG, "grid is NULL");
  if (grid->width < 2 || grid->height < 2)
    return fail(MLS_ERR_INVALID_ARG, "grid %d x %d; contours need width, height >= 2",
                grid->width, grid->height);
  if (!is_finite(grid->x0) || !is_finite(grid->y0) || !is_finite(grid->dx) || !is_finite(grid->dy))
    return fail(MLS_ERR_INVALID_ARG, "grid origin and spacing must be finite");
  if (n_iso < 1) return fail(MLS_ERR_INVALID_ARG, "n_iso = %d; need at least one", n_iso);
  if (capacity < 0) return fail(MLS_ERR_INVALID_ARG, "capacity = %lld", (long long)capacity);
  if (!count) return fail(MLS_ERR_INVALID_ARG, "%s is NULL", count_name);
  if (!d_fields) return fail(MLS_ERR_INVALID_ARG, "d_fields is NULL");
  if (!d_iso) return fail(MLS_ERR_INVALID_ARG, "d_iso is NULL");
  if (capacity > 0 && !d_segments)
    return fail(MLS_ERR_INVALID_ARG, "d_segments is NULL with capacity %lld", (long long)capacity);
  if (d_segments && ((uintptr_t)d_segments % 16) != 0)
    return fail(MLS_ERR_INVALID_ARG, "d_segments must be 16-byte aligned");
  const int64_t cells = (int64_t)(grid->width - 1) * (grid->height - 1);
  const int64_t blocks = (int64_t)d * ((cells + 255) / 256);
  if (blocks * 256 >= ((int64_t)1 << 32) || cells >= ((int64_t)1 << 31))
    return fail(MLS_ERR_INVALID_ARG, "%d fields of %d x %d nodes exceed one launch", d,
                grid->width, grid->height);
  if (!ctx) return fail(MLS_ERR_INVALID_ARG, "ctx is NULL");

  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return device_fail(e, "hipSetDevice");
  mls_status st;
  if ((st = check_device_ptr(ctx, d_fields, "d_fields")) != MLS_OK) return st;
  if ((st = check_device_ptr(ctx, d_iso, "d_iso")) != MLS_OK) return st;
  if (d_cases && (st = check_device_ptr(ctx, d_cases, "d_cases")) != MLS_OK) return st;
  if (d_segments && (st = check_device_ptr(ctx, d_segments, "d_segments")) != MLS_OK) return st;
  if (d_seg_ids && (st = check_device_ptr(ctx, d_seg_ids, "d_seg_ids")) != MLS_OK) return st;
  return MLS_OK;
}

// Byte offsets of one contour call's scratch: counts (scanned in place),
// tile sums, total.
struct ContourScratch {
  size_t off_tiles, off_total, need;
};

static ContourScratch contour_scratch_plan(int32_t d, int32_t n_iso, const mls_grid* grid) {
  const int64_t entries = mls::contour_scratch_entries(d, n_iso, grid->width, grid->height);
  const int64_t tiles = mls::contour_scan_tiles(entries);
  ContourScratch c;
  c.off_tiles = align_up(sizeof(int32_t) * (size_t)entries, 256);
  c.off_total = c.off_tiles + align_up(sizeof(int64_t) * (size_t)tiles, 256);
  c.need = c.off_total + 256;
  return c;
}

static mls::ContourArgs contour_args(const float* d_fields, int32_t d, const mls_grid* grid,
                                     const float* d_iso, int32_t n_iso, uint8_t* d_cases,
                                     float* d_segments, int32_t* d_seg_ids, int64_t capacity,
                                     char* base, const ContourScratch& cs, int64_t* total) {
  mls::ContourArgs a;
  a.fields = d_fields;
  a.iso = d_iso;
  a.D = d;
  a.n_iso = n_iso;
  a.W = grid->width;
  a.H = grid->height;
  a.x0 = grid->x0;
  a.y0 = grid->y0;
  a.dx = grid->dx;
  a.dy = grid->dy;
  a.cases = d_cases;
  a.segs = d_segments;
  a.ids = d_seg_ids;
  a.capacity = capacity;
  a.counts = (int32_t*)base;
  a.offsets = a.counts;   // scanned in place
  a.tile_sums = (int64_t*)(base + cs.off_tiles);
  a.total = total ? total : (int64_t*)(base + cs.off_total);
  return a;
}

mls_status mls_contour(mls_context* ctx, const float* d_fields, int32_t d,
                       const mls_grid* grid, const float* d_iso, int32_t n_iso,
                       uint8_t* d_cases, float* d_segments, int32_t* d_seg_ids,
                       int64_t capacity, int64_t* h_count, void* stream) {
  g_last_error[0] = '\0';
  mls_status st = contour_check(ctx, d_fields, d, grid, d_iso, n_iso, d_cases, d_segments,
                                d_seg_ids, capacity, h_count, "h_count");
  if (st != MLS_OK) return st;
  hipError_t e;
  const ContourScratch cs = contour_scratch_plan(d, n_iso, grid);
  if ((st = ensure_scratch(ctx->scratch, cs.need)) != MLS_OK) return st;
  if (!ctx->pinned) {
    e = hipHostMalloc((void**)&ctx->pinned, sizeof(int64_t) * 4, hipHostMallocDefault);
    if (e != hipSuccess) {
      ctx->pinned = nullptr;
      (void)hipGetLastError();
      return fail(MLS_ERR_OUT_OF_MEMORY, "pinned host allocation failed");
    }
  }
  const mls::ContourArgs a = contour_args(d_fields, d, grid, d_iso, n_iso, d_cases, d_segments,
                                          d_seg_ids, capacity, (char*)ctx->scratch.ptr, cs,
                                          nullptr);
  hipStream_t s = (hipStream_t)stream;
  if ((st = scratch_acquire(ctx, s)) != MLS_OK) return st;
  char meta[160];
  std::snprintf(meta, sizeof(meta), "\"d\": %d, \"n_iso\": %d, \"width\": %d, "
                "\"height\": %d, ", d, n_iso, grid->width, grid->height);
  Tracer tr(ctx, s, "contour", meta);
  e = mls::launch_contour(a, s);
  if (e != hipSuccess) return device_fail(e, "contour kernel launch");
  tr.mark("passes");
  tr.finish();
  if ((st = scratch_release(ctx, s)) != MLS_OK) return st;
  e = hipMemcpyAsync(ctx->pinned, a.total, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return device_fail(e, "count read-back");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return device_fail(e, "stream synchronise");
  *h_count = ctx->pinned[0];
  if (*h_count > capacity)
    return fail(MLS_ERR_CAPACITY, "%lld segments, capacity %lld", (long long)*h_count,
                (long long)capacity);
  return MLS_OK;
}

mls_status mls_contour_static(mls_context* ctx, const float* d_fields, int32_t d,
                              const mls_grid* grid, const float* d_iso, int32_t n_iso,
                              uint8_t* d_cases, float* d_segments, int32_t* d_seg_ids,
                              int64_t capacity, int64_t* d_count, void* stream) {
  g_last_error[0] = '\0';
  mls_status st = contour_check(ctx, d_fields, d, grid, d_iso, n_iso, d_cases, d_segments,
                                d_seg_ids, capacity, d_count, "d_count");
  if (st != MLS_OK) return st;
  if ((st = check_device_ptr(ctx, d_count, "d_count")) != MLS_OK) return st;
  if (((uintptr_t)d_count % 8) != 0) return fail(MLS_ERR_INVALID_ARG, "d_count must be 8-byte aligned");
  const ContourScratch cs = contour_scratch_plan(d, n_iso, grid);
  if (cs.need > MLS_CONTOUR_STATIC_SCRATCH_BYTES)
    return fail(MLS_ERR_INVALID_ARG, "%d fields x %d isovalues on %d x %d nodes need %zu bytes "
                "of contour scratch; the static scratch holds %zu", d, n_iso, grid->width,
                grid->height, cs.need, (size_t)MLS_CONTOUR_STATIC_SCRATCH_BYTES);
  // the address resolved for this device when the context was created
  char* base = (char*)mls::contour_static_scratch(ctx->device);
  if (!base) return fail(MLS_ERR_DEVICE, "static contour scratch not resolved on device %d",
                         ctx->device);
  const mls::ContourArgs a = contour_args(d_fields, d, grid, d_iso, n_iso, d_cases, d_segments,
                                          d_seg_ids, capacity, base, cs, d_count);
  hipError_t e = mls::launch_contour(a, (hipStream_t)stream);
  if (e != hipSuccess) return device_fail(e, "contour kernel launch");
  return MLS_OK;
}

}  // extern "C"
