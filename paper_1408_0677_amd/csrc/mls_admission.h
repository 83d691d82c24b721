// Admission logic of the served form (host only, no HIP): resident point
// sets charged against an HBM budget, a queue of fit requests in arrival
// order, batches of requests that share a kernel class, deadlines and
// cancellation.  The server (mls_server.cpp) drives it under its lock; the
// clock and the allocator are interfaces, so that the whole policy runs on
// the CPU against a fake allocator and a mock clock (tests/admission_driver
// .cpp).
//
// Budget: resident point sets + reserved memory (the tuner's) + slots x
// slot scratch <= budget.  A request
// needs slot scratch (its staging buffers); one that can never fit a slot
// is refused at submit.  A batch takes the request at the head of the queue
// and, if it can share a kernel (class >= 0), the later queued requests of
// the same class, in arrival order, while their scratch fits one slot and
// the batch stays within the request and work-item limits; requests of
// other classes keep their places.  A queued request whose deadline passes
// is cancelled at once; a running one is reported so that the server can
// raise its cancel flag.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <functional>
#include <limits>
#include <map>
#include <vector>

namespace mls {

class Admission {
 public:
  struct Allocator {
    virtual ~Allocator() {}
    virtual bool allocate(size_t bytes, void** ptr) = 0;
    virtual void release(void* ptr) = 0;
  };
  using Clock = std::function<double()>;

  enum Result { kOk = 0, kInvalid = -1, kOutOfMemory = -2, kOverBudget = -5 };

  struct Request {
    uint64_t ticket = 0;
    uint64_t pointset = 0;
    size_t scratch = 0;       // slot scratch it needs
    int64_t cls = -1;         // batch class, -1: runs alone
    int64_t work = 1;         // work items
    double t_submit = 0.0;
    double deadline = std::numeric_limits<double>::infinity();
    bool running = false;
    bool cancel = false;      // cancellation asked for while running
  };

  struct PointSet {
    void* mem = nullptr;
    size_t bytes = 0;
    int users = 0;            // queued or running requests
    bool released = false;
  };

  Admission(size_t budget, int slots, size_t slot_scratch, Clock clock, Allocator* alloc)
      : budget_(budget), slots_(slots), slot_scratch_(slot_scratch), clock_(clock),
        alloc_(alloc) {}

  double now() const { return clock_(); }
  size_t points_bytes() const { return points_bytes_; }
  size_t queued() const { return queue_.size(); }
  bool has_request(uint64_t t) const { return reqs_.count(t) != 0; }
  const Request* request(uint64_t t) const {
    auto it = reqs_.find(t);
    return it == reqs_.end() ? nullptr : &it->second;
  }

  // Memory outside the slots charged against the budget (the tuner's).
  Result reserve(size_t bytes) {
    if (points_bytes_ + reserved_ + bytes + (size_t)slots_ * slot_scratch_ > budget_)
      return kOverBudget;
    reserved_ += bytes;
    return kOk;
  }
  void unreserve(size_t bytes) { reserved_ -= bytes < reserved_ ? bytes : reserved_; }
  size_t reserved() const { return reserved_; }

  // Allocate and charge a point set.
  Result put_points(size_t bytes, uint64_t* id, void** mem) {
    if (points_bytes_ + reserved_ + bytes + (size_t)slots_ * slot_scratch_ > budget_)
      return kOverBudget;
    void* p = nullptr;
    if (!alloc_->allocate(bytes, &p)) return kOutOfMemory;
    PointSet ps;
    ps.mem = p;
    ps.bytes = bytes;
    const uint64_t k = next_pointset_++;
    psets_[k] = ps;
    points_bytes_ += bytes;
    *id = k;
    *mem = p;
    return kOk;
  }

  // Whether a point set's memory is still held (released or not).
  bool resident(uint64_t id) const { return psets_.count(id) != 0; }

  const PointSet* pointset(uint64_t id) const {
    auto it = psets_.find(id);
    return it == psets_.end() || it->second.released ? nullptr : &it->second;
  }

  // Release a point set; its memory goes once no request uses it.
  Result release_points(uint64_t id) {
    auto it = psets_.find(id);
    if (it == psets_.end() || it->second.released) return kInvalid;
    it->second.released = true;
    collect();
    return kOk;
  }

  // Keep a point set resident while work outside the queue (the tuner)
  // reads it; unhold drops the use and frees a released set nobody uses.
  Result hold(uint64_t id) {
    auto it = psets_.find(id);
    if (it == psets_.end() || it->second.released) return kInvalid;
    ++it->second.users;
    return kOk;
  }
  void unhold(uint64_t id) {
    auto it = psets_.find(id);
    if (it == psets_.end()) return;
    --it->second.users;
    collect();
  }

  // Queue a request (r.ticket assigned here).
  Result submit(Request r, uint64_t* ticket) {
    auto it = psets_.find(r.pointset);
    if (it == psets_.end() || it->second.released) return kInvalid;
    if (r.scratch > slot_scratch_) return kOverBudget;
    r.ticket = next_ticket_++;
    r.t_submit = now();
    r.running = false;
    r.cancel = false;
    ++it->second.users;
    reqs_[r.ticket] = r;
    queue_.push_back(r.ticket);
    *ticket = r.ticket;
    return kOk;
  }

  // Cancel: a queued request leaves the queue at once (returns true in
  // *removed); a running one is marked (the caller raises its flag).
  Result cancel(uint64_t ticket, bool* removed) {
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return kInvalid;
    *removed = false;
    if (!it->second.running) {
      drop_queued(ticket);
      *removed = true;
    } else {
      it->second.cancel = true;
    }
    return kOk;
  }

  // Deadlines passed: queued requests are removed (cancelled_queued),
  // running ones are marked and listed once (flag_running).
  void expire(std::vector<uint64_t>* cancelled_queued, std::vector<uint64_t>* flag_running) {
    const double t = now();
    std::vector<uint64_t> late;
    for (auto& kv : reqs_)
      if (kv.second.deadline <= t) late.push_back(kv.first);
    for (uint64_t k : late) {
      Request& r = reqs_[k];
      if (!r.running) {
        drop_queued(k);
        cancelled_queued->push_back(k);
      } else if (!r.cancel) {
        r.cancel = true;
        flag_running->push_back(k);
      }
    }
  }

  // The next batch for a free slot (empty if the queue is).
  std::vector<uint64_t> next_batch(int max_requests, int64_t max_work, int lookahead = 64) {
    std::vector<uint64_t> out;
    if (queue_.empty()) return out;
    const uint64_t head = queue_.front();
    Request& h = reqs_[head];
    out.push_back(head);
    size_t scratch = h.scratch;
    int64_t work = h.work;
    if (h.cls >= 0) {
      int seen = 0;
      for (size_t q = 1; q < queue_.size() && seen < lookahead; ++q, ++seen) {
        if ((int)out.size() >= max_requests) break;
        const Request& r = reqs_[queue_[q]];
        if (r.cls != h.cls) continue;
        if (scratch + r.scratch > slot_scratch_ || work + r.work > max_work) break;
        out.push_back(r.ticket);
        scratch += r.scratch;
        work += r.work;
      }
    }
    for (uint64_t k : out) {
      reqs_[k].running = true;
      for (auto it = queue_.begin(); it != queue_.end(); ++it)
        if (*it == k) {
          queue_.erase(it);
          break;
        }
    }
    return out;
  }

  // A running (or cancelled queued) request is over: drop it and release
  // its point-set use.
  void finish(uint64_t ticket) {
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return;
    auto ps = psets_.find(it->second.pointset);
    if (ps != psets_.end()) --ps->second.users;
    reqs_.erase(it);
    collect();
  }

  // Free released point sets nobody uses.
  void collect() {
    for (auto it = psets_.begin(); it != psets_.end();) {
      if (it->second.released && it->second.users == 0) {
        alloc_->release(it->second.mem);
        points_bytes_ -= it->second.bytes;
        it = psets_.erase(it);
      } else {
        ++it;
      }
    }
  }

  // Every point set (freed at shutdown).
  template <typename F>
  void for_each_pointset(F f) {
    for (auto& kv : psets_) f(kv.second);
  }

 private:
  void drop_queued(uint64_t ticket) {
    for (auto it = queue_.begin(); it != queue_.end(); ++it)
      if (*it == ticket) {
        queue_.erase(it);
        break;
      }
  }

  size_t budget_;
  int slots_;
  size_t slot_scratch_;
  Clock clock_;
  Allocator* alloc_;
  size_t points_bytes_ = 0, reserved_ = 0;
  uint64_t next_pointset_ = 1, next_ticket_ = 1;
  std::map<uint64_t, PointSet> psets_;
  std::map<uint64_t, Request> reqs_;
  std::deque<uint64_t> queue_;
};

}  // namespace mls
