// CPU driver of the served form's admission logic (mls_admission.h) with a
// fake allocator and a mock clock; built by tests/test_admission.py (with
// AddressSanitizer and UndefinedBehaviorSanitizer) and run as a program.
// Prints "ok" and exits 0 when every check holds.
#include <cstdio>
#include <cstdlib>
#include <set>

#include "../paper_1408_0677_amd/csrc/mls_admission.h"

using mls::Admission;

#define CHECK(c)                                                    \
  do {                                                              \
    if (!(c)) {                                                     \
      std::printf("check failed at line %d: %s\n", __LINE__, #c); \
      std::exit(1);                                                 \
    }                                                               \
  } while (0)

struct FakeAllocator : Admission::Allocator {
  size_t live_bytes = 0;
  size_t capacity = 1u << 30;
  std::set<void*> live;
  bool allocate(size_t bytes, void** p) override {
    if (live_bytes + bytes > capacity) return false;
    *p = std::malloc(bytes ? bytes : 1);
    live.insert(*p);
    live_bytes += bytes;
    sizes[*p] = bytes;
    return true;
  }
  void release(void* p) override {
    CHECK(live.count(p) == 1);
    live.erase(p);
    live_bytes -= sizes[p];
    std::free(p);
  }
  std::map<void*, size_t> sizes;
};

static Admission::Request req(uint64_t ps, size_t scratch, int64_t cls, int64_t work = 10,
                              double deadline = 1e300) {
  Admission::Request r;
  r.pointset = ps;
  r.scratch = scratch;
  r.cls = cls;
  r.work = work;
  r.deadline = deadline;
  return r;
}

int main() {
  double t = 0.0;
  FakeAllocator fa;
  // budget 1000 bytes, 2 slots of 100 bytes scratch: 800 bytes of points
  Admission adm(1000, 2, 100, [&] { return t; }, &fa);
  uint64_t p1, p2, p3;
  void* m;
  CHECK(adm.put_points(500, &p1, &m) == Admission::kOk);
  CHECK(adm.put_points(300, &p2, &m) == Admission::kOk);
  CHECK(adm.put_points(1, &p3, &m) == Admission::kOverBudget);   // 801 > 800
  CHECK(fa.live.size() == 2 && adm.points_bytes() == 800);
  // an allocator failure is out of memory, not over budget
  FakeAllocator tiny;
  tiny.capacity = 10;
  Admission adm2(1000, 1, 10, [&] { return t; }, &tiny);
  CHECK(adm2.put_points(20, &p3, &m) == Admission::kOutOfMemory);

  // submit: unknown point set, scratch beyond a slot
  uint64_t tk;
  CHECK(adm.submit(req(99, 10, 1), &tk) == Admission::kInvalid);
  CHECK(adm.submit(req(p1, 101, 1), &tk) == Admission::kOverBudget);

  // batching: head class, later same-class requests while scratch fits
  uint64_t a, b, c, d, e;
  CHECK(adm.submit(req(p1, 40, 1), &a) == Admission::kOk);
  t = 1.0;
  CHECK(adm.submit(req(p2, 40, 2), &b) == Admission::kOk);
  CHECK(adm.submit(req(p1, 40, 1), &c) == Admission::kOk);
  CHECK(adm.submit(req(p1, 40, 1), &d) == Admission::kOk);   // 120 > 100: next batch
  CHECK(adm.submit(req(p2, 10, -1), &e) == Admission::kOk);  // runs alone
  CHECK(adm.request(c)->t_submit == 1.0);
  std::vector<uint64_t> bt = adm.next_batch(8, 1000);
  CHECK(bt.size() == 2 && bt[0] == a && bt[1] == c);
  CHECK(adm.request(a)->running && adm.request(c)->running);
  bt = adm.next_batch(8, 1000);
  CHECK(bt.size() == 1 && bt[0] == b);
  bt = adm.next_batch(8, 1000);
  CHECK(bt.size() == 1 && bt[0] == d);
  bt = adm.next_batch(8, 1000);
  CHECK(bt.size() == 1 && bt[0] == e);
  CHECK(adm.next_batch(8, 1000).empty());
  // request and work limits
  uint64_t q[4];
  for (int i = 0; i < 4; ++i) CHECK(adm.submit(req(p2, 10, 7, 30), &q[i]) == Admission::kOk);
  bt = adm.next_batch(2, 1000);
  CHECK(bt.size() == 2 && bt[0] == q[0] && bt[1] == q[1]);
  bt = adm.next_batch(8, 40);
  CHECK(bt.size() == 1 && bt[0] == q[2]);
  bt = adm.next_batch(8, 1000);
  CHECK(bt.size() == 1 && bt[0] == q[3]);

  // release a point set in use: memory kept until its requests finish
  CHECK(adm.release_points(p1) == Admission::kOk);
  CHECK(adm.release_points(p1) == Admission::kInvalid);
  CHECK(fa.live.size() == 2);
  CHECK(adm.submit(req(p1, 10, 1), &tk) == Admission::kInvalid);   // released: no new work
  adm.finish(a);
  adm.finish(c);
  CHECK(fa.live.size() == 2);                                       // d still runs on p1
  adm.finish(d);
  CHECK(fa.live.size() == 1 && adm.points_bytes() == 300);
  for (uint64_t k : {b, e, q[0], q[1], q[2], q[3]}) adm.finish(k);

  // cancellation: queued requests leave at once, running ones are marked
  uint64_t x, y;
  CHECK(adm.submit(req(p2, 10, 3), &x) == Admission::kOk);
  CHECK(adm.submit(req(p2, 10, 4), &y) == Admission::kOk);
  bool removed = false;
  CHECK(adm.cancel(x, &removed) == Admission::kOk && removed);
  adm.finish(x);
  bt = adm.next_batch(8, 1000);
  CHECK(bt.size() == 1 && bt[0] == y);
  CHECK(adm.cancel(y, &removed) == Admission::kOk && !removed && adm.request(y)->cancel);
  adm.finish(y);
  CHECK(adm.cancel(y, &removed) == Admission::kInvalid);

  // deadlines on the mock clock
  t = 10.0;
  uint64_t u, v, w;
  CHECK(adm.submit(req(p2, 10, 5, 10, 11.0), &u) == Admission::kOk);
  CHECK(adm.submit(req(p2, 10, 6, 10, 12.0), &v) == Admission::kOk);
  CHECK(adm.submit(req(p2, 10, 6, 10, 30.0), &w) == Admission::kOk);
  bt = adm.next_batch(8, 1000);                 // u runs
  CHECK(bt.size() == 1 && bt[0] == u);
  std::vector<uint64_t> cq, fr;
  t = 11.5;
  adm.expire(&cq, &fr);
  CHECK(cq.empty() && fr.size() == 1 && fr[0] == u);   // running: flagged once
  cq.clear();
  fr.clear();
  adm.expire(&cq, &fr);
  CHECK(cq.empty() && fr.empty());
  t = 12.0;
  adm.expire(&cq, &fr);
  CHECK(cq.size() == 1 && cq[0] == v && fr.empty());   // queued: cancelled
  adm.finish(v);
  bt = adm.next_batch(8, 1000);
  CHECK(bt.size() == 1 && bt[0] == w);
  adm.finish(u);
  adm.finish(w);
  CHECK(adm.queued() == 0);

  // reserved memory (the tuner's) counts against the budget; a held point
  // set stays resident after its release until the hold ends
  CHECK(adm.points_bytes() == 300);
  CHECK(adm.reserve(501) == Admission::kOverBudget);     // 300 + 501 > 800
  CHECK(adm.reserve(400) == Admission::kOk);
  CHECK(adm.put_points(101, &p3, &m) == Admission::kOverBudget);
  CHECK(adm.put_points(100, &p3, &m) == Admission::kOk);
  CHECK(adm.hold(p3) == Admission::kOk && adm.hold(999) == Admission::kInvalid);
  CHECK(adm.release_points(p3) == Admission::kOk);
  CHECK(fa.live.size() == 2 && adm.points_bytes() == 400);
  CHECK(adm.resident(p3) && adm.pointset(p3) == nullptr);
  adm.unhold(p3);
  CHECK(!adm.resident(p3));
  CHECK(fa.live.size() == 1 && adm.points_bytes() == 300);
  adm.unreserve(400);
  CHECK(adm.reserved() == 0 && adm.put_points(500, &p3, &m) == Admission::kOk);
  CHECK(adm.hold(p3) == Admission::kOk);
  adm.unhold(p3);
  CHECK(fa.live.size() == 2);                              // not released: kept

  // shutdown: every remaining point set released through the allocator
  adm.for_each_pointset([&](const Admission::PointSet& ps) { fa.release(ps.mem); });
  CHECK(fa.live.empty());
  std::printf("ok\n");
  return 0;
}
