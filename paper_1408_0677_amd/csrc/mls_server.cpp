// Served form of the MLS fit: resident point sets, admission by an HBM
// budget, and continuous batching of fit requests in persistent kernels.
//
// The paper re-evaluates the MLS field on every parameter change of an
// interactive session (Sec. 3.5, Sec. 4.5); a server takes such requests of
// uneven size as they come.  Design:
//   - Point sets are copied once into server memory (put_points) and stay
//     resident; requests refer to them by id.  The admission policy (budget,
//     queue, batches, deadlines, cancellation) is host-only code in
//     mls_admission.h, driven here under the server's lock.
//   - The server owns `slots` execution slots: a HIP stream, a context whose
//     staging scratch is reserved up front, and pinned host and device
//     blocks for batch descriptors and flags.  Budget = resident points +
//     slots x slot scratch (+ the tuner's reservation); admitted work
//     allocates nothing.
//   - A scheduler thread gives every free slot the next batch: the request
//     at the head of the queue and the later queued requests of its kernel
//     class (16-bit one-pass Gaussian fits of one degree, feature-tile
//     count, term count and format), in arrival order, while their staging
//     fits the slot.  A batch is staged request by request into the slot's
//     scratch and runs as one persistent kernel whose workgroups take
//     (request, tile) items from a device counter.  Each request's
//     completion flag, in pinned host memory, is set by the workgroup that
//     finishes its last item; the scheduler polls the flags and retires
//     requests one by one while the batch runs on.  A request that arrives
//     meanwhile joins the next batch a slot takes.  Requests of other kinds
//     (float64, Wendland, the two-pass bfloat16 form) run alone on a slot,
//     their completion signalled by a host function behind them.
//   - Cancellation (mls_server_cancel, or a request's timeout): a queued
//     request leaves the queue at once; a batched one has its pinned cancel
//     flag raised, which the kernel reads before every work item, so its
//     remaining items are skipped.  A request running alone completes.
//   - Autotuner (optional): the node tile is 16 x 16 (the matrix
//     instruction's); the tuned tile dimension is the feature axis, the
//     attributes per slab.  The first request of a coarse shape class is
//     queued to a tuner thread that times the candidate widths on its own
//     stream, context and output buffer while the scheduler serves the class
//     with the library's plan; later requests take the fastest width.  The
//     width changes no result bit.
// A request's results do not depend on what else runs: each tile is
// computed by the same code from the same parameters in a batch and alone
// (mls_fit), and fits touch only their own staging scratch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mls.h"
#include "mls_admission.h"
#include "mls_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kMaxBatch = 64;       // requests per batch
constexpr int kMaxItems = 1 << 16;  // work items per batch

struct Ticket {
  mls_request req;
  mls_result res;
  bool done = false;
  int slot = -1, index = -1;        // where it runs
  mls::FitArgs args;
  int terms = 0;
  int64_t cls = -1;                 // batch class, -1: runs alone
  mls::LPBatchClass bc{};
};

// Byte layout of a batch descriptor block (host copy and device copy):
// counters (head, done[], skipped[]) zeroed per batch, items per request,
// kernel parameters per request, then the (request, block) items; only the
// used part is copied.
struct DescLayout {
  size_t counters, totals, params, items, bytes;
};
size_t align256(size_t v) { return (v + 255) / 256 * 256; }
DescLayout desc_layout() {
  DescLayout L;
  L.counters = 0;
  L.totals = align256((1 + 2 * kMaxBatch) * 4);
  L.params = align256(L.totals + kMaxBatch * 4);
  L.items = align256(L.params + kMaxBatch * mls::lp_params_bytes());
  L.bytes = align256(L.items + (size_t)kMaxItems * 8);
  return L;
}

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done_ev = nullptr;           // behind a batch kernel
  mls_context* ctx = nullptr;
  std::vector<uint64_t> running;          // batch members, or one ticket
  std::vector<bool> retired;
  bool batch = false;
  std::atomic<bool> finished{false};      // single fits: set by the host function
  std::atomic<double> t_end{0.0};
  uint32_t* complete = nullptr;           // pinned, coherent: [kMaxBatch] set by the kernel
  uint32_t* cancel = nullptr;             // [kMaxBatch] read by the kernel
  char* desc = nullptr;                   // pinned descriptor block
  char* dev = nullptr;                    // device copy of it
};

struct Completion {
  struct mls_server* srv;
  int slot;
};

// Device memory of resident point sets.
struct DeviceAllocator : mls::Admission::Allocator {
  bool allocate(size_t bytes, void** p) override {
    if (hipMalloc(p, bytes ? bytes : 1) != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return false;
    }
    return true;
  }
  void release(void* p) override { (void)hipFree(p); }
};

struct PointSetInfo {
  float* pts = nullptr;
  float* vals = nullptr;
  int64_t n = 0;
  int32_t d = 0;
};

struct TuneJob {
  std::string key;
  mls_request req;
  PointSetInfo ps;
};

}  // namespace

struct mls_server {
  int device = 0;
  size_t slot_scratch = 0;
  Clock::time_point t0;
  DeviceAllocator alloc;
  std::unique_ptr<mls::Admission> adm;
  std::map<uint64_t, PointSetInfo> psets;
  std::unique_ptr<Slot[]> slots;
  int nslots = 0;
  std::vector<Completion> completions;
  std::map<uint64_t, std::unique_ptr<Ticket>> tickets;
  hipStream_t copy_stream = nullptr;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::thread sched;
  bool stop = false;
  // tuner
  bool tune_on = false;
  bool tune_ready = false;                // resources allocated, thread started
  std::string tune_path;
  std::map<std::string, int> tune_table;  // class -> attributes per slab (0: library plan)
  std::map<std::string, bool> tune_pending;
  std::deque<TuneJob> tune_jobs;
  std::condition_variable tune_cv;
  std::thread tuner;
  mls_context* tune_ctx = nullptr;
  hipStream_t tune_stream = nullptr;
  hipEvent_t tune_e0 = nullptr, tune_e1 = nullptr;
  void* tune_out = nullptr;
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

// Slot scratch a request needs (the plan mls_fit uses), rounded so that a
// batch can place requests back to back.
size_t request_scratch(const mls_request& r, int64_t n, int32_t d) {
  return align256(mls::fit_scratch_bytes(n, d, r.precision, r.weight.kind, r.weight.h, r.grid.x0,
                                         r.grid.y0, r.grid.dx, r.grid.dy, r.grid.width,
                                         r.grid.height));
}

int ceil_log2(int64_t v) {
  int k = 0;
  while (((int64_t)1 << k) < v) ++k;
  return k;
}

// Tuner shape class: precision, basis, weight kind, D rounded up to a power
// of two, node count rounded up to a power of four.
std::string tune_key(const mls_request& r, int32_t d) {
  const int64_t nodes = (int64_t)r.grid.width * r.grid.height;
  char buf[96];
  std::snprintf(buf, sizeof(buf), "p%d b%d w%d d%d g%d", r.precision, r.basis, r.weight.kind,
                1 << ceil_log2(d), 1 << (2 * ((ceil_log2(nodes) + 1) / 2)));
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
  if (s->tune_path.empty()) return;
  FILE* f = std::fopen(s->tune_path.c_str(), "w");
  if (!f) return;
  for (auto& kv : s->tune_table) std::fprintf(f, "%s = %d\n", kv.first.c_str(), kv.second);
  std::fclose(f);
}

// Drop the records of point sets whose memory is gone (lock held).
void prune_psets(mls_server* s) {
  for (auto it = s->psets.begin(); it != s->psets.end();) {
    if (!s->adm->resident(it->first)) it = s->psets.erase(it);
    else ++it;
  }
}

// Time the candidate widths of one class on the tuner's own stream, context
// and output buffer (lock not held); 0 = keep the library's plan.  The
// device is shared with the slots, so each width is timed in three rounds,
// interleaved with the others, and keeps its fastest time; a width replaces
// the library's plan only when it is at least 5% faster.
int tune_job(mls_server* s, const TuneJob& job) {
  const size_t out_bytes = (size_t)job.ps.d * job.req.grid.width * job.req.grid.height * 4;
  if (out_bytes > s->slot_scratch) return 0;
  int nts0, plan_ds, nslab0;
  mls::lp_slab_plan(job.req.basis, job.ps.d, 0, &nts0, &plan_ds, &nslab0);
  std::vector<int> cands = slab_candidates(job.req.basis, job.ps.d);
  if (std::find(cands.begin(), cands.end(), plan_ds) == cands.end()) cands.push_back(plan_ds);
  std::vector<float> best(cands.size(), 0.0f);
  for (int round = 0; round < 4; ++round) {   // round 0 loads the kernels
    for (size_t k = 0; k < cands.size(); ++k) {
      mls_solve_opts o = job.req.opts;
      o.lp_slab = cands[k];
      float ms = 0.0f;
      bool good = hipEventRecord(s->tune_e0, s->tune_stream) == hipSuccess;
      good = good && mls_fit(s->tune_ctx, job.ps.pts, job.ps.vals, job.ps.n, job.ps.d,
                             job.req.basis, &job.req.weight, &job.req.grid, job.req.precision,
                             &o, (float*)s->tune_out, nullptr, (void*)s->tune_stream) == MLS_OK;
      good = good && hipEventRecord(s->tune_e1, s->tune_stream) == hipSuccess;
      good = good && hipEventSynchronize(s->tune_e1) == hipSuccess;
      good = good && hipEventElapsedTime(&ms, s->tune_e0, s->tune_e1) == hipSuccess;
      if (!good) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(s->tune_stream);
        return 0;
      }
      if (round > 0 && (best[k] == 0.0f || ms < best[k])) best[k] = ms;
    }
  }
  size_t arg = 0, plan = 0;
  for (size_t k = 0; k < cands.size(); ++k) {
    if (best[k] < best[arg]) arg = k;
    if (cands[k] == plan_ds) plan = k;
  }
  return best[arg] < 0.95f * best[plan] ? cands[arg] : 0;
}

void tuner_main(mls_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->tune_cv.wait(lk, [&] { return s->stop || !s->tune_jobs.empty(); });
    if (s->stop) break;
    const TuneJob job = s->tune_jobs.front();
    s->tune_jobs.pop_front();
    lk.unlock();
    const int best = tune_job(s, job);
    lk.lock();
    s->adm->unhold(job.req.pointset);
    prune_psets(s);
    s->tune_table[job.key] = best;
    save_tuner(s);
    s->tune_pending.erase(job.key);
  }
  // jobs never run keep no point set resident
  for (const TuneJob& j : s->tune_jobs) s->adm->unhold(j.req.pointset);
  s->tune_jobs.clear();
  s->tune_pending.clear();
}

// Host function behind a single fit: stamp the end and wake the scheduler.
// It takes no lock, so it never waits on a thread inside the HIP runtime.
void on_complete(void* arg) {
  Completion* c = (Completion*)arg;
  mls_server* s = c->srv;
  Slot& sl = s->slots[c->slot];
  sl.t_end.store(seconds_since(s));
  sl.finished.store(true);
  s->cv.notify_all();
}

// A request is over (lock held).
void retire(mls_server* s, uint64_t t, int status, double t_end, const char* detail) {
  auto it = s->tickets.find(t);
  if (it == s->tickets.end() || it->second->done) return;
  Ticket& k = *it->second;
  k.res.status = status;
  k.res.t_end = t_end;
  if (k.res.t_admit < k.res.t_submit) k.res.t_admit = t_end;
  if (k.res.t_start < k.res.t_admit) k.res.t_start = k.res.t_admit;
  if (detail) std::snprintf(k.res.detail, sizeof(k.res.detail), "%s", detail);
  k.done = true;
  k.slot = k.index = -1;
  s->adm->finish(t);
  prune_psets(s);
  s->done_cv.notify_all();
}

// Run a request alone on a slot (lock held).
void launch_single(mls_server* s, int si, uint64_t t) {
  Slot& sl = s->slots[si];
  Ticket& k = *s->tickets[t];
  const PointSetInfo& ps = s->psets[k.req.pointset];
  sl.batch = false;
  sl.running.assign(1, t);
  sl.retired.assign(1, false);
  k.slot = si;
  k.index = 0;
  k.res.t_admit = seconds_since(s);
  const mls_status st = mls_fit(sl.ctx, ps.pts, ps.vals, ps.n, ps.d, k.req.basis, &k.req.weight,
                                &k.req.grid, k.req.precision, &k.req.opts, k.req.d_fields,
                                k.req.d_degree, (void*)sl.stream);
  k.res.t_start = seconds_since(s);
  if (st != MLS_OK) {
    sl.running.clear();
    retire(s, t, st, k.res.t_start, mls_last_error());
    return;
  }
  sl.finished.store(false);
  if (hipLaunchHostFunc(sl.stream, on_complete, &s->completions[si]) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(sl.stream);
    sl.t_end.store(seconds_since(s));
    sl.finished.store(true);
  }
}

// Run a batch of one class on a slot (lock held): stage every member into
// its share of the slot's scratch, write the descriptors, copy them to the
// device and launch the persistent kernel.
void launch_batch(mls_server* s, int si, const std::vector<uint64_t>& members) {
  Slot& sl = s->slots[si];
  const DescLayout L = desc_layout();
  size_t cap = 0;
  char* base = (char*)mls::context_scratch(sl.ctx, &cap);
  size_t off = 0;
  uint32_t* items = (uint32_t*)(sl.desc + L.items);
  uint32_t* totals = (uint32_t*)(sl.desc + L.totals);
  int64_t n_items = 0;
  bool ok = true;
  sl.batch = true;
  sl.running = members;
  sl.retired.assign(members.size(), false);
  const double t_admit = seconds_since(s);
  for (size_t j = 0; j < members.size(); ++j) {
    Ticket& k = *s->tickets[members[j]];
    const PointSetInfo& ps = s->psets[k.req.pointset];
    k.slot = si;
    k.index = (int)j;
    k.res.t_admit = t_admit;
    sl.complete[j] = 0;
    sl.cancel[j] = 0;
    const mls::FitPlan plan = mls::make_fit_plan(
        ps.n, ps.d, k.req.precision, k.req.weight.kind, k.req.weight.h, k.req.grid.x0,
        k.req.grid.y0, k.req.grid.dx, k.req.grid.dy, k.req.grid.width, k.req.grid.height);
    if (off + plan.total > cap) {   // admission keeps the sum within a slot
      ok = false;
      break;
    }
    char* b = base + off;
    off += align256(plan.total);
    float* shift = (float*)(b + plan.o_shift);
    float* scale = (float*)(b + plan.o_scale);
    float* vals_t = (float*)(b + plan.o_vals);
    if (mls::launch_stage(ps.vals, ps.n, ps.d, (float*)(b + plan.o_pmin),
                          (float*)(b + plan.o_pmax), shift, scale, vals_t, sl.stream) !=
        hipSuccess) {
      ok = false;
      break;
    }
    mls::lp_params_write(k.args, vals_t, shift, scale,
                         sl.desc + L.params + j * mls::lp_params_bytes());
    totals[j] = (uint32_t)k.bc.blocks;
    for (int64_t blk = 0; blk < k.bc.blocks; ++blk) {
      items[2 * n_items] = (uint32_t)j;
      items[2 * n_items + 1] = (uint32_t)blk;
      ++n_items;
    }
  }
  std::memset(sl.desc + L.counters, 0, (1 + 2 * kMaxBatch) * 4);
  uint32_t* counters = (uint32_t*)(sl.dev + L.counters);
  hipError_t e = hipSuccess;
  if (ok) e = hipMemcpyAsync(sl.dev, sl.desc, L.items + (size_t)n_items * 8,
                             hipMemcpyHostToDevice, sl.stream);
  if (ok && e == hipSuccess)
    e = mls::launch_fit_lp_batch(s->tickets[members[0]]->bc, sl.dev + L.params,
                                 (const uint32_t*)(sl.dev + L.items), (int)n_items,
                                 (const uint32_t*)(sl.dev + L.totals), counters, counters + 1,
                                 counters + 1 + kMaxBatch, sl.complete, sl.cancel, 0, sl.stream);
  if (ok && e == hipSuccess) e = hipEventRecord(sl.done_ev, sl.stream);
  const double now = seconds_since(s);
  if (!ok || e != hipSuccess) {
    (void)hipGetLastError();
    (void)hipStreamSynchronize(sl.stream);
    (void)hipGetLastError();
    sl.running.clear();
    for (uint64_t t : members) retire(s, t, MLS_ERR_DEVICE, now, "batch staging or launch failed");
    return;
  }
  for (uint64_t t : members) s->tickets[t]->res.t_start = now;
}

// Retire finished work (lock held): batch members whose completion flag is
// set, single fits whose host function has run; a slot is free again once
// its kernel has left the device.
void poll_slots(mls_server* s) {
  for (int i = 0; i < s->nslots; ++i) {
    Slot& sl = s->slots[i];
    if (sl.running.empty()) continue;
    if (!sl.batch) {
      if (!sl.finished.load()) continue;
      sl.finished.store(false);
      const uint64_t t = sl.running[0];
      sl.running.clear();
      retire(s, t, MLS_OK, sl.t_end.load(), nullptr);
      continue;
    }
    bool all = true;
    for (size_t j = 0; j < sl.running.size(); ++j) {
      if (sl.retired[j]) continue;
      const uint32_t c = __atomic_load_n(&sl.complete[j], __ATOMIC_ACQUIRE);
      if (c == 0) {
        all = false;
        continue;
      }
      sl.retired[j] = true;
      retire(s, sl.running[j], c == 1 ? MLS_OK : MLS_ERR_CANCELLED, seconds_since(s),
             c == 1 ? nullptr : "cancelled: remaining work items skipped");
    }
    const hipError_t q = hipEventQuery(sl.done_ev);
    if (q == hipSuccess) {
      if (all) sl.running.clear();
    } else if (q != hipErrorNotReady) {
      // the batch failed on the device: its unfinished requests fail
      for (size_t j = 0; j < sl.running.size(); ++j)
        if (!sl.retired[j])
          retire(s, sl.running[j], MLS_ERR_DEVICE, seconds_since(s), hipGetErrorString(q));
      sl.running.clear();
    }
    (void)hipGetLastError();
  }
}

bool any_running(const mls_server* s) {
  for (int i = 0; i < s->nslots; ++i)
    if (!s->slots[i].running.empty()) return true;
  return false;
}

bool any_free(const mls_server* s) {
  for (int i = 0; i < s->nslots; ++i)
    if (s->slots[i].running.empty()) return true;
  return false;
}

// Raise the cancel flag of a running batch member (lock held).
void flag_cancel(mls_server* s, uint64_t t) {
  auto it = s->tickets.find(t);
  if (it == s->tickets.end()) return;
  const Ticket& k = *it->second;
  if (k.slot < 0 || !s->slots[k.slot].batch) return;
  __atomic_store_n(&s->slots[k.slot].cancel[k.index], 1u, __ATOMIC_RELEASE);
}

void scheduler(mls_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // batches signal through host memory, so the thread polls while work
    // runs; otherwise it sleeps until a submit, a cancel or stop (or the
    // next deadline check)
    const bool busy = any_running(s);
    s->cv.wait_for(lk, busy ? std::chrono::microseconds(50) : std::chrono::microseconds(5000),
                   [&] { return s->stop || (s->adm->queued() > 0 && any_free(s)); });
    std::vector<uint64_t> cq, fr;
    s->adm->expire(&cq, &fr);
    for (uint64_t t : cq) retire(s, t, MLS_ERR_CANCELLED, seconds_since(s), "timeout in the queue");
    for (uint64_t t : fr) flag_cancel(s, t);
    poll_slots(s);
    for (int si = 0; si < s->nslots && s->adm->queued() > 0; ++si) {
      if (!s->slots[si].running.empty()) continue;
      const std::vector<uint64_t> b = s->adm->next_batch(kMaxBatch, kMaxItems);
      if (b.empty()) break;
      if (s->tickets[b[0]]->cls < 0) launch_single(s, si, b[0]);
      else launch_batch(s, si, b);
    }
    if (s->stop && s->adm->queued() == 0 && !any_running(s)) return;
  }
}

void free_slot(Slot& sl) {
  if (sl.stream) {
    (void)hipStreamSynchronize(sl.stream);
    (void)hipStreamDestroy(sl.stream);
  }
  if (sl.done_ev) (void)hipEventDestroy(sl.done_ev);
  if (sl.ctx) mls_context_destroy(sl.ctx);
  if (sl.complete) (void)hipHostFree(sl.complete);
  if (sl.desc) (void)hipHostFree(sl.desc);
  if (sl.dev) (void)hipFree(sl.dev);
  sl.stream = nullptr;
  sl.done_ev = nullptr;
  sl.ctx = nullptr;
  sl.complete = sl.cancel = nullptr;
  sl.desc = sl.dev = nullptr;
}

void free_tuner(mls_server* s) {
  if (s->tune_stream) {
    (void)hipStreamSynchronize(s->tune_stream);
    (void)hipStreamDestroy(s->tune_stream);
  }
  if (s->tune_e0) (void)hipEventDestroy(s->tune_e0);
  if (s->tune_e1) (void)hipEventDestroy(s->tune_e1);
  if (s->tune_out) (void)hipFree(s->tune_out);
  if (s->tune_ctx) mls_context_destroy(s->tune_ctx);
  s->tune_stream = nullptr;
  s->tune_e0 = s->tune_e1 = nullptr;
  s->tune_out = nullptr;
  s->tune_ctx = nullptr;
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
  s->slot_scratch = slot_scratch_bytes;
  s->t0 = Clock::now();
  mls_server* raw_s = s.get();
  s->adm.reset(new mls::Admission(hbm_budget_bytes, slots, slot_scratch_bytes,
                                  [raw_s] { return seconds_since(raw_s); }, &s->alloc));
  s->slots.reset(new (std::nothrow) Slot[slots]);
  if (!s->slots) return sfail(MLS_ERR_OUT_OF_MEMORY, "host allocation failed");
  s->nslots = slots;
  s->completions.resize(slots);
  auto cleanup = [&]() {
    for (int j = 0; j < slots; ++j) free_slot(s->slots[j]);
    if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
  };
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return sfail(MLS_ERR_DEVICE, "hipSetDevice: %s", hipGetErrorString(e));
  const DescLayout L = desc_layout();
  for (int i = 0; i < slots; ++i) {
    Slot& sl = s->slots[i];
    s->completions[i] = Completion{s.get(), i};
    mls_status st;
    if ((st = mls_context_create(device, &sl.ctx)) != MLS_OK ||
        (st = mls_context_reserve(sl.ctx, slot_scratch_bytes)) != MLS_OK) {
      sfail(st, "slot context: %s", mls_last_error());
      cleanup();
      return st;
    }
    e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done_ev, hipEventDisableTiming);
    // flags the kernel and the host both read and write: coherent pinned
    // memory; descriptors: pinned staging for one copy per batch
    void* flags = nullptr;
    if (e == hipSuccess) e = hipHostMalloc(&flags, 2 * kMaxBatch * 4, hipHostMallocCoherent);
    if (e == hipSuccess) {
      sl.complete = (uint32_t*)flags;
      sl.cancel = sl.complete + kMaxBatch;
      std::memset(flags, 0, 2 * kMaxBatch * 4);
      e = hipHostMalloc((void**)&sl.desc, L.bytes, hipHostMallocDefault);
    }
    if (e == hipSuccess) e = hipMalloc((void**)&sl.dev, L.bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      cleanup();
      return sfail(MLS_ERR_DEVICE, "slot stream, event or batch buffers: %s",
                   hipGetErrorString(e));
    }
  }
  e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    cleanup();
    return sfail(MLS_ERR_DEVICE, "copy stream creation: %s", hipGetErrorString(e));
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
  s->tune_cv.notify_all();
  if (s->sched.joinable()) s->sched.join();
  if (s->tuner.joinable()) s->tuner.join();
  (void)hipSetDevice(s->device);
  for (int i = 0; i < s->nslots; ++i) free_slot(s->slots[i]);
  free_tuner(s);
  if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
  s->adm->for_each_pointset([&](const mls::Admission::PointSet& ps) { s->alloc.release(ps.mem); });
  delete s;
}

mls_status mls_server_tuning(mls_server* s, int32_t enable, const char* cache_path) {
  g_srv_error[0] = '\0';
  if (!s) return sfail(MLS_ERR_INVALID_ARG, "server is NULL");
  if (enable != 0 && enable != 1) return sfail(MLS_ERR_INVALID_ARG, "enable = %d", enable);
  std::lock_guard<std::mutex> lk(s->mu);
  if (enable == 1 && !s->tune_ready) {
    // the tuner's context scratch and output buffer, charged to the budget
    if (s->adm->reserve(2 * s->slot_scratch) != mls::Admission::kOk)
      return sfail(MLS_ERR_OVER_BUDGET, "the tuner's %zu bytes do not fit the budget",
                   2 * s->slot_scratch);
    hipError_t e = hipSetDevice(s->device);
    mls_status st = MLS_OK;
    if (e == hipSuccess) {
      st = mls_context_create(s->device, &s->tune_ctx);
      if (st == MLS_OK) st = mls_context_reserve(s->tune_ctx, s->slot_scratch);
    }
    if (e == hipSuccess && st == MLS_OK) e = hipMalloc(&s->tune_out, s->slot_scratch);
    if (e == hipSuccess && st == MLS_OK)
      e = hipStreamCreateWithFlags(&s->tune_stream, hipStreamNonBlocking);
    if (e == hipSuccess && st == MLS_OK) e = hipEventCreate(&s->tune_e0);
    if (e == hipSuccess && st == MLS_OK) e = hipEventCreate(&s->tune_e1);
    if (e != hipSuccess || st != MLS_OK) {
      (void)hipGetLastError();
      free_tuner(s);
      s->adm->unreserve(2 * s->slot_scratch);
      return st != MLS_OK ? sfail(st, "tuner context: %s", mls_last_error())
                          : sfail(MLS_ERR_OUT_OF_MEMORY, "tuner buffers: %s",
                                  hipGetErrorString(e));
    }
    s->tune_ready = true;
    s->tuner = std::thread(tuner_main, s);
  }
  s->tune_on = enable == 1;
  s->tune_path = cache_path ? cache_path : "";
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char line[160];
      while (std::fgets(line, sizeof(line), f)) {
        char* eq = std::strrchr(line, '=');
        if (!eq) continue;
        const int ds = std::atoi(eq + 1);
        std::string key(line, eq - line);
        while (!key.empty() && key.back() == ' ') key.pop_back();
        if (ds >= 0 && ds <= MLS_LP_MAX_SLAB_LINEAR && !key.empty()) s->tune_table[key] = ds;
      }
      std::fclose(f);
    }
  }
  return MLS_OK;
}

int64_t mls_server_tuned_classes(mls_server* s) {
  if (!s) return 0;
  std::lock_guard<std::mutex> lk(s->mu);
  return (int64_t)s->tune_table.size();
}

int64_t mls_server_tuning_pending(mls_server* s) {
  if (!s) return 0;
  std::lock_guard<std::mutex> lk(s->mu);
  return (int64_t)s->tune_pending.size();
}

mls_status mls_server_put_points(mls_server* s, const float* d_points, const float* d_values,
                                 int64_t n, int32_t d, uint64_t* pointset) {
  g_srv_error[0] = '\0';
  if (!s || !pointset) return sfail(MLS_ERR_INVALID_ARG, "server or pointset is NULL");
  if (!d_points || !d_values) return sfail(MLS_ERR_INVALID_ARG, "points or values are NULL");
  if (n < 1 || n > MLS_MAX_N) return sfail(MLS_ERR_INVALID_ARG, "n = %lld", (long long)n);
  if (d < 1 || d > MLS_MAX_D_LP) return sfail(MLS_ERR_INVALID_ARG, "d = %d", d);
  const size_t pbytes = align256((size_t)n * 2 * sizeof(float));
  const size_t bytes = pbytes + (size_t)n * d * sizeof(float);
  std::lock_guard<std::mutex> lk(s->mu);
  (void)hipSetDevice(s->device);
  uint64_t id = 0;
  void* mem = nullptr;
  const int r = s->adm->put_points(bytes, &id, &mem);
  if (r == mls::Admission::kOverBudget)
    return sfail(MLS_ERR_OVER_BUDGET, "point set of %zu bytes does not fit the budget", bytes);
  if (r != mls::Admission::kOk) return sfail(MLS_ERR_OUT_OF_MEMORY, "point set allocation failed");
  PointSetInfo ps;
  ps.pts = (float*)mem;
  ps.vals = (float*)((char*)mem + pbytes);
  ps.n = n;
  ps.d = d;
  // a device-to-device hipMemcpy may return before the copy has landed;
  // copy on the server's own stream and wait for it
  hipError_t e = hipMemcpyAsync(ps.pts, d_points, (size_t)n * 2 * sizeof(float),
                                hipMemcpyDefault, s->copy_stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ps.vals, d_values, (size_t)n * d * sizeof(float), hipMemcpyDefault,
                       s->copy_stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->copy_stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    s->adm->release_points(id);
    return sfail(MLS_ERR_DEVICE, "point set copy: %s", hipGetErrorString(e));
  }
  s->psets[id] = ps;
  *pointset = id;
  return MLS_OK;
}

mls_status mls_server_release_points(mls_server* s, uint64_t pointset) {
  g_srv_error[0] = '\0';
  if (!s) return sfail(MLS_ERR_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  (void)hipSetDevice(s->device);
  if (s->adm->release_points(pointset) != mls::Admission::kOk)
    return sfail(MLS_ERR_INVALID_ARG, "unknown point set %llu", (unsigned long long)pointset);
  prune_psets(s);
  return MLS_OK;
}

mls_status mls_server_submit(mls_server* s, const mls_request* req, uint64_t* ticket) {
  g_srv_error[0] = '\0';
  if (!s || !req || !ticket) return sfail(MLS_ERR_INVALID_ARG, "server, request or ticket NULL");
  if (!std::isfinite(req->timeout_s) || req->timeout_s < 0.0)
    return sfail(MLS_ERR_INVALID_ARG, "timeout_s = %g; need a finite value >= 0", req->timeout_s);
  std::unique_ptr<Ticket> t(new (std::nothrow) Ticket);
  if (!t) return sfail(MLS_ERR_OUT_OF_MEMORY, "host allocation failed");
  t->req = *req;
  std::memset(&t->res, 0, sizeof(t->res));
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto pit = s->psets.find(req->pointset);
    if (pit == s->psets.end() || !s->adm->pointset(req->pointset))
      return sfail(MLS_ERR_INVALID_ARG, "unknown point set %llu",
                   (unsigned long long)req->pointset);
    const PointSetInfo ps = pit->second;
    // the tuned slab width of the request's class, when there is one
    const std::string key = tune_key(*req, ps.d);
    bool tune_new = false;
    if (s->tune_on && req->precision != MLS_PREC_F64 && req->opts.lp_slab == 0) {
      auto it = s->tune_table.find(key);
      if (it != s->tune_table.end()) t->req.opts.lp_slab = it->second;
      else tune_new = !s->tune_pending.count(key);
    }
    // every check mls_fit makes, now: a request that cannot run fails at
    // submit with the fit's status
    (void)hipSetDevice(s->device);
    const mls_status st = (mls_status)mls::fit_prepare_c(
        s->slots[0].ctx, ps.pts, ps.vals, ps.n, ps.d, t->req.basis, &t->req.weight,
        &t->req.grid, t->req.precision, &t->req.opts, t->req.d_fields, nullptr,
        t->req.d_degree, &t->args, &t->terms);
    if (st != MLS_OK) return sfail(st, "%s", mls_last_error());
    mls::Admission::Request ar;
    ar.pointset = req->pointset;
    ar.scratch = request_scratch(t->req, ps.n, ps.d);
    if (ar.scratch > s->slot_scratch)
      return sfail(MLS_ERR_OVER_BUDGET, "request needs %zu scratch bytes, a slot has %zu",
                   ar.scratch, s->slot_scratch);
    if (t->req.precision != MLS_PREC_F64 &&
        mls::lp_batch_class(t->args, t->req.precision == MLS_PREC_FP16, t->terms, &t->bc) &&
        t->bc.blocks <= kMaxItems) {
      t->cls = (((int64_t)t->bc.deg * 16 + t->bc.nts) * 4 + t->bc.terms) * 2 + (t->bc.fp16 ? 1 : 0);
      ar.work = t->bc.blocks;
    } else {
      t->cls = -1;
      ar.work = 1;
    }
    ar.cls = t->cls;
    if (req->timeout_s > 0.0) ar.deadline = seconds_since(s) + req->timeout_s;
    uint64_t id = 0;
    if (s->adm->submit(ar, &id) != mls::Admission::kOk)
      return sfail(MLS_ERR_INVALID_ARG, "point set %llu is not available",
                   (unsigned long long)req->pointset);
    if (tune_new && s->adm->hold(req->pointset) == mls::Admission::kOk) {
      // first of its class: time the candidates on the tuner thread (the
      // point set stays resident while the job holds it)
      s->tune_pending[key] = true;
      s->tune_jobs.push_back(TuneJob{key, *req, ps});
      s->tune_cv.notify_all();
    }
    t->res.t_submit = s->adm->request(id)->t_submit;
    t->res.status = MLS_PENDING;
    *ticket = id;
    s->tickets[id] = std::move(t);
  }
  s->cv.notify_all();
  return MLS_OK;
}

mls_status mls_server_cancel(mls_server* s, uint64_t ticket) {
  g_srv_error[0] = '\0';
  if (!s) return sfail(MLS_ERR_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  bool removed = false;
  if (it == s->tickets.end() || it->second->done ||
      s->adm->cancel(ticket, &removed) != mls::Admission::kOk)
    return sfail(MLS_ERR_INVALID_ARG, "ticket %llu is not queued or running",
                 (unsigned long long)ticket);
  if (removed) retire(s, ticket, MLS_ERR_CANCELLED, seconds_since(s), "cancelled in the queue");
  else flag_cancel(s, ticket);
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
