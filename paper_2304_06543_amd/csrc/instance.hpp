// instance.hpp -- host-side state of one LBDD instance (shared by the C ABI
// translation units).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "lbdd_dev.hpp"

namespace lbdd {
// the calling thread's last failure, read by lbdd_last_error()
extern thread_local std::string g_err;
// record a failure description and return `code`
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
}  // namespace lbdd

struct lbdd_instance {
  int32_t k = 0;                        // centers of the graph (strict: + the dummy center)
  int64_t n = 0;
  bool strict = false;                  // a strict-LBDD instance (Appendix B)
  int32_t k_user = 0;                   // centers given by the caller
  int32_t dummy = -1;                   // index of the dummy center, -1 if none
  int64_t dummy_cost = 0;               // its cost for every unit (largest entry + 1)
  hipStream_t st = nullptr;
  int64_t enqueued = 0;                 // iterations launched so far
  int32_t *cm = nullptr, *smin = nullptr, *cap = nullptr, *pen = nullptr;
  int32_t *assign = nullptr, *load = nullptr, *members = nullptr, *slot = nullptr;
  int32_t *unperm = nullptr;            // [n] staging for lbdd_assignment
  int64_t *order = nullptr, *scalars = nullptr;
  uint64_t *W = nullptr;
  uint32_t *Wh = nullptr;
  uint32_t *WhT = nullptr;
  uint64_t *best = nullptr;
  uint8_t *meta = nullptr;
  uint64_t *thr = nullptr;
  int64_t *poff = nullptr;              // penalty tables (null: constant penalties)
  int32_t *pval = nullptr;

  lbdd::InstView view() const {
    lbdd::InstView v;
    v.k = k; v.strict = strict ? 1 : 0; v.n = n; v.cm = cm; v.smin = smin; v.cap = cap; v.pen = pen;
    v.assign = assign; v.load = load; v.members = members; v.slot = slot; v.W = W; v.Wh = Wh; v.WhT = WhT;
    v.best = best; v.meta = meta; v.thr = thr;
    v.scalars = scalars;
    v.poff = poff; v.pval = pval;
    return v;
  }
};

