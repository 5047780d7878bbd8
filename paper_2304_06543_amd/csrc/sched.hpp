// sched.hpp -- admission policy of the LBDD request server (host only, no HIP).
//
// Requests wait in arrival order.  A request is admitted when its device
// footprint fits in the free part of the HBM budget and a job slot is free.
// When the oldest waiting request does not fit, younger requests that do fit
// may go ahead of it, but only `max_bypass` times in a row: after that the
// oldest one blocks the queue until enough memory frees up.  A request larger
// than the whole budget is admitted once nothing else is in flight, so every
// request eventually runs.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>

namespace lbdd {

struct AdmissionQueue {
  struct Item {
    uint64_t id;
    size_t footprint;
  };

  explicit AdmissionQueue(int max_bypass = 8) : max_bypass_(max_bypass) {}

  void push(uint64_t id, size_t footprint) { q_.push_back(Item{id, footprint}); }
  size_t size() const { return q_.size(); }
  bool empty() const { return q_.empty(); }

  // Remove a waiting request (cancellation); false if it is not waiting.
  bool erase(uint64_t id) {
    for (auto it = q_.begin(); it != q_.end(); ++it)
      if (it->id == id) {
        if (it == q_.begin()) bypassed_ = 0;
        q_.erase(it);
        return true;
      }
    return false;
  }

  // Remove every waiting request whose id satisfies pred (expiry), passing
  // each removed id to out; returns how many were removed.
  template <class Pred, class Out>
  size_t erase_if(Pred pred, Out out) {
    size_t m = 0;
    for (auto it = q_.begin(); it != q_.end();) {
      if (pred(it->id)) {
        if (it == q_.begin()) bypassed_ = 0;
        out(it->id);
        it = q_.erase(it);
        ++m;
      } else {
        ++it;
      }
    }
    return m;
  }

  // Next request to admit given the free budget, the number of jobs in flight
  // and whether a job slot is free; sets *id and returns true, or false when
  // nothing may be admitted now.  The chosen request is removed.
  bool next(size_t free_bytes, int inflight, bool slot_free, uint64_t *id) {
    if (q_.empty() || !slot_free) return false;
    const Item &head = q_.front();
    if (head.footprint <= free_bytes || inflight == 0) {
      *id = head.id;
      q_.pop_front();
      bypassed_ = 0;
      return true;
    }
    if (bypassed_ >= max_bypass_) return false;   // the oldest request waits for memory
    for (auto it = q_.begin() + 1; it != q_.end(); ++it)
      if (it->footprint <= free_bytes) {
        *id = it->id;
        q_.erase(it);
        ++bypassed_;
        return true;
      }
    return false;
  }

 private:
  std::deque<Item> q_;
  int max_bypass_;
  int bypassed_ = 0;
};

// Device memory an instance of k centers and n units holds while it is being
// solved: the permuted cost matrix and the per-center member lists (4nk each),
// per-unit arrays, the k x k table (with its high words) and the k x k x 8
// best-transfer lists,
// plus the transient setup buffers (the
// unpermuted cost matrix copy and sort keys).
inline size_t instance_footprint(int32_t k, int64_t n) {
  const size_t nk = (size_t)n * (size_t)k;
  return nk * 4 * 3 + (size_t)n * (4 * 4 + 8 + 4 + 16) + (size_t)k * k * (8 + 4 + 8 * 8 + 1 + 8) +
         (size_t)k * 16 + 4096;
}

}  // namespace lbdd
