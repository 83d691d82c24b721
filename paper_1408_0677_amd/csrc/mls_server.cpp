// Served form of the MLS fit: resident point sets, admission by an HBM
// budget, and continuous batching of fit requests over concurrent streams.
//
// The paper re-evaluates the MLS field on every parameter change of an
// interactive session (Sec. 3.5, Sec. 4.5); a server takes such requests of
// uneven size as they come.  Design:
//   - Point sets are copied once into server memory (put_points) and stay
//     resident; requests refer to them by id.
//   - The server owns `slots` execution slots.  A slot is a HIP stream plus
//     an mls_context whose staging scratch is reserved up front, so admitted
//     work never allocates or frees device memory (hipFree would stall every
//     stream).  Budget = resident points + slots x slot scratch.
//   - A scheduler thread admits queued requests in arrival order whenever a
//     slot is free and the request's scratch fits its slot, and launches the
//     fit on that slot's stream.  Requests in different slots run at the
//     same time; the GPU interleaves their workgroups, so a small request
//     that arrives while a large one runs starts at once instead of waiting
//     for it (continuous batching, not a queue).
//   - Completion is signalled by a host function enqueued behind the fit on
//     the slot's stream; it stamps the end time and frees the slot.
//   - A request that fails validation fails alone at submit; one that can
//     never fit the budget is rejected with MLS_ERR_OVER_BUDGET.
//   - Autotuner (optional, mls_server_tuning): the 16-bit kernels take a
//     slab width (attributes per workgroup, which sets the workgroup's
//     feature-tile count).  The best width depends on the request's shape
//     (basis, D, grid size, N) through occupancy, the number of workgroups
//     and the moment columns every slab repeats.  The first request of a
//     shape class is run once per candidate width on its own slot, timed
//     with stream events, and the fastest width is kept for the class (and
//     written to a cache file if one was given); later requests of the
//     class use it.  The width changes no result bit, so tuning is
//     invisible in the output.
// Results of a request do not depend on what else runs: each fit is
// deterministic and touches only its own slot's scratch.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <deque>
#include <map>
#include <string>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/mls.h"
#include "mls_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct PointSet {
  float* pts = nullptr;
  float* vals = nullptr;
  int64_t n = 0;
  int32_t d = 0;
  size_t bytes = 0;
  int users = 0;          // queued or running requests
  bool released = false;  // free when users drops to 0
};

struct Ticket {
  uint64_t id = 0;
  mls_request req;
  mls_result res;
  bool done = false;
  size_t scratch = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;   // tuner timing
  mls_context* ctx = nullptr;
  Ticket* running = nullptr;
  std::atomic<bool> finished{false};  // set by the stream's host function
  std::atomic<double> t_end{0.0};
};

struct Completion {
  struct mls_server* srv;
  int slot;
};

}  // namespace

// Shape classes and their tuned slab widths.
struct Tuner {
  bool on = false;
  std::string path;                 // cache file, or empty
  std::map<std::string, int> table; // class key -> attributes per slab
};

struct mls_server {
  int device = 0;
  // point-set copies: issued here and waited for before put_points
  // returns, so that no slot stream (non-blocking, unordered with the
  // caller's streams) can read a point set before it is complete
  hipStream_t copy_stream = nullptr;
  Tuner tuner;
  size_t budget = 0;
  size_t slot_scratch = 0;
  size_t points_bytes = 0;
  Clock::time_point t0;
  std::unique_ptr<Slot[]> slots;
  int nslots = 0;
  std::vector<Completion> completions;
  std::map<uint64_t, PointSet> psets;
  std::map<uint64_t, std::unique_ptr<Ticket>> tickets;
  std::deque<Ticket*> queue;
  uint64_t next_pset = 1, next_ticket = 1;
  std::mutex mu;
  std::condition_variable cv;       // scheduler wake-up
  std::condition_variable done_cv;  // waiters
  std::thread sched;
  bool stop = false;
};

namespace {

thread_local char g_srv_error[512] = "";

mls_status sfail(mls_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_srv_error, sizeof(g_srv_error), fmt, ap);
  va_end(ap);
  return s;
}

double seconds_since(const mls_server* s) {
  return std::chrono::duration<double>(Clock::now() - s->t0).count();
}

// Device scratch a fit request needs in its slot (the same plan mls_fit uses).
size_t request_scratch(const mls_request& r, const PointSet& ps) {
  return mls::fit_scratch_bytes(ps.n, ps.d, r.precision, r.weight.kind, r.weight.h, r.grid.x0,
                                r.grid.y0, r.grid.dx, r.grid.dy, r.grid.width, r.grid.height);
}

// Host function behind a request's kernels: stamp the end and wake the
// scheduler.  It takes no lock, so it never waits on a thread that may be
// inside the HIP runtime.
void on_complete(void* arg) {
  Completion* c = (Completion*)arg;
  mls_server* s = c->srv;
  Slot& sl = s->slots[c->slot];
  sl.t_end.store(seconds_since(s));
  sl.finished.store(true);
  s->cv.notify_all();
}

// Retire the requests whose host function has run.  Lock held.
bool retire_finished(mls_server* s) {
  bool any = false;
  for (int i = 0; i < s->nslots; ++i) {
    Slot& sl = s->slots[i];
    if (!sl.running || !sl.finished.load()) continue;
    Ticket* t = sl.running;
    t->res.t_end = sl.t_end.load();
    t->done = true;
    auto it = s->psets.find(t->req.pointset);
    if (it != s->psets.end()) --it->second.users;
    sl.running = nullptr;
    sl.finished.store(false);
    any = true;
  }
  if (any) s->done_cv.notify_all();
  return any;
}

int ilog2(int64_t v) {
  int k = 0;
  while (v > 1) {
    v >>= 1;
    ++k;
  }
  return k;
}

// Shape class of a 16-bit request: precision, basis, weight, D, and the
// node-tile and point counts to the nearest power of two below.
std::string tune_key(const mls_request& r, const PointSet& ps) {
  const int64_t tiles = (int64_t)((r.grid.width + 15) / 16) * ((r.grid.height + 15) / 16);
  char buf[96];
  std::snprintf(buf, sizeof(buf), "p%d b%d w%d d%d t%d n%d", r.precision, r.basis,
                r.weight.kind, ps.d, ilog2(tiles), ilog2(ps.n));
  return buf;
}

// Candidate slab widths: the widest slab for each feature-tile count, the
// four cheapest by the tile-count model (slabs x tiles per slab).
std::vector<int> slab_candidates(int basis, int D) {
  const int m = mls::basis_terms(basis), nmom = mls::moment_terms(basis);
  const int cap = basis == MLS_BASIS_QUADRATIC ? MLS_LP_MAX_SLAB_QUADRATIC
                  : basis == MLS_BASIS_LINEAR  ? MLS_LP_MAX_SLAB_LINEAR
                                               : MLS_LP_MAX_SLAB_CONSTANT;
  std::vector<std::pair<int, int>> c;   // (cost, ds)
  for (int nts = 1; nts <= 8; ++nts) {
    int ds = (16 * nts - nmom) / m;
    ds = std::min(std::min(ds, cap), D);
    if (ds < 1) continue;
    bool seen = false;
    for (auto& e : c) seen |= e.second == ds;
    if (seen) continue;
    int need = 1;
    while (need * 16 < nmom + m * ds) ++need;
    c.push_back({((D + ds - 1) / ds) * need, ds});
  }
  std::sort(c.begin(), c.end());
  std::vector<int> out;
  for (size_t i = 0; i < c.size() && i < 4; ++i) out.push_back(c[i].second);
  return out;
}

void save_tuner(const mls_server* s) {
  if (s->tuner.path.empty()) return;
  FILE* f = std::fopen(s->tuner.path.c_str(), "w");
  if (!f) return;
  for (auto& kv : s->tuner.table) std::fprintf(f, "%s = %d\n", kv.first.c_str(), kv.second);
  std::fclose(f);
}

// Time every candidate slab width on the request itself (each run writes
// the same outputs) and return the fastest.  Runs unlocked: the slot is
// already marked busy with this ticket and its point set is pinned by the
// ticket's use count.
int tune_request(Slot& sl, const mls_request& r, const PointSet& ps,
                 std::unique_lock<std::mutex>& lk) {
  const std::vector<int> cands = slab_candidates(r.basis, ps.d);
  if (cands.size() < 2) return cands.empty() ? 0 : cands[0];
  lk.unlock();
  int best = 0;
  float best_ms = 0.0f;
  for (int c : cands) {
    mls_solve_opts o = r.opts;
    o.lp_slab = c;
    float ms = 0.0f;
    bool ok = true;
    for (int rep = 0; rep < 2 && ok; ++rep) {   // the first run loads the kernel
      ok = hipEventRecord(sl.ev0, sl.stream) == hipSuccess;
      ok = ok && mls_fit(sl.ctx, ps.pts, ps.vals, ps.n, ps.d, r.basis, &r.weight, &r.grid,
                         r.precision, &o, r.d_fields, r.d_degree, (void*)sl.stream) == MLS_OK;
      ok = ok && hipEventRecord(sl.ev1, sl.stream) == hipSuccess;
      ok = ok && hipEventSynchronize(sl.ev1) == hipSuccess;
      ok = ok && hipEventElapsedTime(&ms, sl.ev0, sl.ev1) == hipSuccess;
    }
    if (ok && (best == 0 || ms < best_ms)) {
      best = c;
      best_ms = ms;
    }
  }
  lk.lock();
  return best;
}

// Launch a ticket on a free slot.  Called with the lock held (released
// while a new shape class is tuned).
void launch(mls_server* s, int si, Ticket* t, std::unique_lock<std::mutex>& lk) {
  Slot& sl = s->slots[si];
  PointSet& ps = s->psets[t->req.pointset];
  t->res.t_admit = seconds_since(s);
  sl.running = t;
  mls_request& r = t->req;
  if (s->tuner.on && r.precision != MLS_PREC_F64 && r.opts.lp_slab == 0) {
    const std::string key = tune_key(r, ps);
    auto it = s->tuner.table.find(key);
    if (it == s->tuner.table.end()) {
      const int best = tune_request(sl, r, ps, lk);
      it = s->tuner.table.emplace(key, best).first;
      save_tuner(s);
    }
    r.opts.lp_slab = it->second;
  }
  mls_status st = mls_fit(sl.ctx, ps.pts, ps.vals, ps.n, ps.d, r.basis, &r.weight, &r.grid,
                          r.precision, &r.opts, r.d_fields, r.d_degree, (void*)sl.stream);
  t->res.t_start = seconds_since(s);
  if (st != MLS_OK) {
    t->res.status = st;
    std::snprintf(t->res.detail, sizeof(t->res.detail), "%s", mls_last_error());
    t->res.t_end = t->res.t_start;
    t->done = true;
    --ps.users;
    sl.running = nullptr;
    s->done_cv.notify_all();
    return;
  }
  t->res.status = MLS_OK;
  sl.finished.store(false);
  hipError_t e = hipLaunchHostFunc(sl.stream, on_complete, &s->completions[si]);
  if (e != hipSuccess) {
    // fall back to waiting here; the result is still correct
    (void)hipStreamSynchronize(sl.stream);
    sl.t_end.store(seconds_since(s));
    sl.finished.store(true);
  }
}

bool any_free(mls_server* s) {
  for (int i = 0; i < s->nslots; ++i)
    if (!s->slots[i].running) return true;
  return false;
}

bool any_running(mls_server* s) {
  for (int i = 0; i < s->nslots; ++i)
    if (s->slots[i].running) return true;
  return false;
}

bool any_finished(mls_server* s) {
  for (int i = 0; i < s->nslots; ++i)
    if (s->slots[i].running && s->slots[i].finished.load()) return true;
  return false;
}

void scheduler(mls_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // wake on a finished request, an admissible request, or stop; the
    // timeout covers a notification that raced with the predicate check
    s->cv.wait_for(lk, std::chrono::milliseconds(2), [&] {
      return s->stop || any_finished(s) || (!s->queue.empty() && any_free(s));
    });
    retire_finished(s);
    // admit in arrival order onto free slots
    for (int si = 0; si < s->nslots && !s->queue.empty(); ++si) {
      if (s->slots[si].running) continue;
      Ticket* t = s->queue.front();
      s->queue.pop_front();
      launch(s, si, t, lk);
    }
    // released point sets with no users left
    for (auto it = s->psets.begin(); it != s->psets.end();) {
      if (it->second.released && it->second.users == 0) {
        (void)hipFree(it->second.pts);
        (void)hipFree(it->second.vals);
        s->points_bytes -= it->second.bytes;
        it = s->psets.erase(it);
      } else {
        ++it;
      }
    }
    if (s->stop && s->queue.empty() && !any_running(s)) return;
  }
}

}  // namespace

extern "C" {

const char* mls_server_last_error(void) { return g_srv_error; }

mls_status mls_server_create(int32_t device, size_t hbm_budget_bytes, int32_t slots,
                             size_t slot_scratch_bytes, mls_server** out) {
  g_srv_error[0] = '\0';
  if (!out) return sfail(MLS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (slots < 1 || slots > 64) return sfail(MLS_ERR_INVALID_ARG, "slots = %d; need 1..64", slots);
  if ((size_t)slots * slot_scratch_bytes > hbm_budget_bytes)
    return sfail(MLS_ERR_OVER_BUDGET, "%d slots x %zu scratch bytes exceed the budget %zu",
                 slots, slot_scratch_bytes, hbm_budget_bytes);
  std::unique_ptr<mls_server> s(new (std::nothrow) mls_server);
  if (!s) return sfail(MLS_ERR_OUT_OF_MEMORY, "host allocation failed");
  s->device = device;
  s->budget = hbm_budget_bytes;
  s->slot_scratch = slot_scratch_bytes;
  s->t0 = Clock::now();
  mls_status st;
  s->slots.reset(new (std::nothrow) Slot[slots]);
  if (!s->slots) return sfail(MLS_ERR_OUT_OF_MEMORY, "host allocation failed");
  s->nslots = slots;
  s->completions.resize(slots);
  auto cleanup = [&]() {
    for (int j = 0; j < slots; ++j) {
      if (s->slots[j].ctx) mls_context_destroy(s->slots[j].ctx);
      if (s->slots[j].ev0) (void)hipEventDestroy(s->slots[j].ev0);
      if (s->slots[j].ev1) (void)hipEventDestroy(s->slots[j].ev1);
      if (s->slots[j].stream) (void)hipStreamDestroy(s->slots[j].stream);
    }
  };
  for (int i = 0; i < slots; ++i) {
    s->completions[i] = Completion{s.get(), i};
    if ((st = mls_context_create(device, &s->slots[i].ctx)) != MLS_OK) {
      sfail(st, "slot context: %s", mls_last_error());
      cleanup();
      return st;
    }
    if ((st = mls_context_reserve(s->slots[i].ctx, slot_scratch_bytes)) != MLS_OK) {
      sfail(st, "slot scratch: %s", mls_last_error());
      cleanup();
      return st;
    }
    hipError_t e = hipStreamCreateWithFlags(&s->slots[i].stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&s->slots[i].ev0);
    if (e == hipSuccess) e = hipEventCreate(&s->slots[i].ev1);
    if (e != hipSuccess) {
      cleanup();
      return sfail(MLS_ERR_DEVICE, "stream or event creation: %s", hipGetErrorString(e));
    }
  }
  {
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      cleanup();
      return sfail(MLS_ERR_DEVICE, "copy stream creation: %s", hipGetErrorString(e));
    }
  }
  mls_server* raw = s.release();
  raw->sched = std::thread(scheduler, raw);
  *out = raw;
  return MLS_OK;
}

void mls_server_destroy(mls_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->sched.joinable()) s->sched.join();
  (void)hipSetDevice(s->device);
  for (int i = 0; i < s->nslots; ++i) {
    Slot& sl = s->slots[i];
    if (sl.stream) {
      (void)hipStreamSynchronize(sl.stream);
      (void)hipStreamDestroy(sl.stream);
    }
    if (sl.ev0) (void)hipEventDestroy(sl.ev0);
    if (sl.ev1) (void)hipEventDestroy(sl.ev1);
    if (sl.ctx) mls_context_destroy(sl.ctx);
  }
  if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
  for (auto& kv : s->psets) {
    (void)hipFree(kv.second.pts);
    (void)hipFree(kv.second.vals);
  }
  delete s;
}

mls_status mls_server_tuning(mls_server* s, int32_t enable, const char* cache_path) {
  g_srv_error[0] = '\0';
  if (!s) return sfail(MLS_ERR_INVALID_ARG, "server is NULL");
  if (enable != 0 && enable != 1) return sfail(MLS_ERR_INVALID_ARG, "enable = %d", enable);
  std::lock_guard<std::mutex> lk(s->mu);
  s->tuner.on = enable == 1;
  s->tuner.path = cache_path ? cache_path : "";
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char line[160];
      while (std::fgets(line, sizeof(line), f)) {
        char* eq = std::strrchr(line, '=');
        if (!eq) continue;
        const int ds = std::atoi(eq + 1);
        std::string key(line, eq - line);
        while (!key.empty() && key.back() == ' ') key.pop_back();
        if (ds >= 1 && ds <= MLS_LP_MAX_SLAB_LINEAR && !key.empty()) s->tuner.table[key] = ds;
      }
      std::fclose(f);
    }
  }
  return MLS_OK;
}

int64_t mls_server_tuned_classes(mls_server* s) {
  if (!s) return 0;
  std::lock_guard<std::mutex> lk(s->mu);
  return (int64_t)s->tuner.table.size();
}

mls_status mls_server_put_points(mls_server* s, const float* d_points, const float* d_values,
                                 int64_t n, int32_t d, uint64_t* pointset) {
  g_srv_error[0] = '\0';
  if (!s || !pointset) return sfail(MLS_ERR_INVALID_ARG, "server or pointset is NULL");
  if (!d_points || !d_values) return sfail(MLS_ERR_INVALID_ARG, "points or values are NULL");
  if (n < 1 || n > MLS_MAX_N) return sfail(MLS_ERR_INVALID_ARG, "n = %lld", (long long)n);
  if (d < 1 || d > MLS_MAX_D_LP) return sfail(MLS_ERR_INVALID_ARG, "d = %d", d);
  const size_t bytes = (size_t)n * 2 * sizeof(float) + (size_t)n * d * sizeof(float);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->points_bytes + bytes + (size_t)s->nslots * s->slot_scratch > s->budget)
    return sfail(MLS_ERR_OVER_BUDGET, "point set of %zu bytes does not fit the budget", bytes);
  (void)hipSetDevice(s->device);
  PointSet ps;
  ps.n = n;
  ps.d = d;
  ps.bytes = bytes;
  if (hipMalloc(&ps.pts, (size_t)n * 2 * sizeof(float)) != hipSuccess ||
      hipMalloc(&ps.vals, (size_t)n * d * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    if (ps.pts) (void)hipFree(ps.pts);
    return sfail(MLS_ERR_OUT_OF_MEMORY, "point set allocation failed");
  }
  // a device-to-device hipMemcpy may return before the copy has landed;
  // copy on the server's own stream and wait for it
  hipError_t e = hipMemcpyAsync(ps.pts, d_points, (size_t)n * 2 * sizeof(float),
                                hipMemcpyDefault, s->copy_stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ps.vals, d_values, (size_t)n * d * sizeof(float), hipMemcpyDefault,
                       s->copy_stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->copy_stream);
  if (e != hipSuccess) {
    (void)hipFree(ps.pts);
    (void)hipFree(ps.vals);
    return sfail(MLS_ERR_DEVICE, "point set copy: %s", hipGetErrorString(e));
  }
  const uint64_t id = s->next_pset++;
  s->psets[id] = ps;
  s->points_bytes += bytes;
  *pointset = id;
  return MLS_OK;
}

mls_status mls_server_release_points(mls_server* s, uint64_t pointset) {
  g_srv_error[0] = '\0';
  if (!s) return sfail(MLS_ERR_INVALID_ARG, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->psets.find(pointset);
    if (it == s->psets.end() || it->second.released)
      return sfail(MLS_ERR_INVALID_ARG, "unknown point set %llu", (unsigned long long)pointset);
    it->second.released = true;
  }
  s->cv.notify_all();
  return MLS_OK;
}

mls_status mls_server_submit(mls_server* s, const mls_request* req, uint64_t* ticket) {
  g_srv_error[0] = '\0';
  if (!s || !req || !ticket) return sfail(MLS_ERR_INVALID_ARG, "server, request or ticket NULL");
  std::unique_ptr<Ticket> t(new (std::nothrow) Ticket);
  if (!t) return sfail(MLS_ERR_OUT_OF_MEMORY, "host allocation failed");
  t->req = *req;
  std::memset(&t->res, 0, sizeof(t->res));
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->psets.find(req->pointset);
    if (it == s->psets.end() || it->second.released)
      return sfail(MLS_ERR_INVALID_ARG, "unknown point set %llu",
                   (unsigned long long)req->pointset);
    if (!req->d_fields) return sfail(MLS_ERR_INVALID_ARG, "d_fields is NULL");
    t->scratch = request_scratch(*req, it->second);
    if (t->scratch > s->slot_scratch)
      return sfail(MLS_ERR_OVER_BUDGET, "request needs %zu scratch bytes, a slot has %zu",
                   t->scratch, s->slot_scratch);
    t->id = s->next_ticket++;
    t->res.t_submit = seconds_since(s);
    t->res.status = MLS_PENDING;
    ++it->second.users;
    *ticket = t->id;
    s->queue.push_back(t.get());
    s->tickets[t->id] = std::move(t);
  }
  s->cv.notify_all();
  return MLS_OK;
}

mls_status mls_server_poll(mls_server* s, uint64_t ticket, mls_result* out) {
  g_srv_error[0] = '\0';
  if (!s || !out) return sfail(MLS_ERR_INVALID_ARG, "server or out is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end())
    return sfail(MLS_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
  *out = it->second->res;
  if (!it->second->done) return MLS_PENDING;
  s->tickets.erase(it);
  return MLS_OK;
}

mls_status mls_server_wait(mls_server* s, uint64_t ticket, mls_result* out) {
  g_srv_error[0] = '\0';
  if (!s || !out) return sfail(MLS_ERR_INVALID_ARG, "server or out is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end())
    return sfail(MLS_ERR_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
  Ticket* t = it->second.get();
  s->done_cv.wait(lk, [&] { return t->done; });
  *out = t->res;
  s->tickets.erase(ticket);
  return MLS_OK;
}

}  // extern "C"
