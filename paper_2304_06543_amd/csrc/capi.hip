// capi.hip -- the C ABI declared in include/lbdd.h.
//
// An instance owns its device state for its whole life: the cost matrix with
// rows permuted into processing order, the allotment, per-center member lists
// and loads, the best-transfer table W and a few int64 scalars (objective,
// progress, status, counters).  Nothing crosses the host/device boundary
// between lbdd_create and the calls that return results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbdd.h"
#include "instance.hpp"
#include "lbdd_dev.hpp"
#include "road.hpp"
#include "scan_batch.hpp"

namespace {

using lbdd::fail;
using lbdd::g_err;

int hip_fail(hipError_t e, const char *what) {
  if (e == hipErrorOutOfMemory)
    return fail(LBDD_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
  return fail(LBDD_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

// All device memory of an instance is stream-ordered on the instance's
// stream, and every copy is an async copy on that stream followed by a wait
// for that stream only: nothing here waits for the whole device, so an
// instance can be created, read and freed while other kernels (a batch or a
// request server) keep running.
template <class T>
hipError_t dalloc(T **p, size_t count, hipStream_t st) {
  return hipMallocAsync(reinterpret_cast<void **>(p), count * sizeof(T) + 1, st);
}

hipError_t copy_sync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind, hipStream_t st) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

void release(lbdd_instance *h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->st);
  void *ptrs[] = {h->cm, h->smin, h->cap, h->pen, h->assign, h->load, h->members,
                  h->slot, h->unperm, h->order, h->scalars, h->W, h->Wh, h->WhT, h->best, h->meta, h->thr,
                  h->poff, h->pval};
  for (void *p : ptrs)
    if (p) (void)hipFreeAsync(p, h->st);
  (void)hipStreamSynchronize(h->st);
  delete h;
}

// Read the device scalars after the stream has drained.
int read_scalars(lbdd_instance *h, int64_t *sc) {
  HIP_TRY(copy_sync(sc, h->scalars, sizeof(int64_t) * lbdd::SC_COUNT, hipMemcpyDeviceToHost, h->st),
          "copy scalars");
  if (sc[lbdd::SC_STATUS] != 0)
    return fail(LBDD_E_INTERNAL,
                "solve stopped at iteration %lld: Bellman-Ford found a negative cycle that the "
                "refinement invariants rule out (status %lld)",
                (long long)sc[lbdd::SC_DONE], (long long)sc[lbdd::SC_STATUS]);
  return LBDD_OK;
}

constexpr int64_t ITERS_PER_LAUNCH = 1 << 21;   // one launch covers every workload here

}  // namespace

namespace lbdd {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace lbdd

extern "C" {

const char *lbdd_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

// lbdd_create, lbdd_create_strict and lbdd_create_penalty_table.  A strict
// instance with excess demand gets the dummy center as its center k
// (capacity n - sum, cost largest entry + 1); its penalties are unused.  With
// penalty tables (pen_off, pen_val) `penalty` is NULL.
int create_instance(int32_t k, int64_t n, const int32_t *cm, const int32_t *capacity,
                    const int32_t *penalty, const int64_t *pen_off, const int32_t *pen_val,
                    uint32_t flags, void *hip_stream, bool strict, lbdd_instance **out) {
  g_err.clear();
  if (!out) return fail(LBDD_E_INVAL, "out is NULL");
  *out = nullptr;
  if (k < 1 || k > LBDD_MAX_K) return fail(LBDD_E_INVAL, "k=%d outside [1, %d]", k, LBDD_MAX_K);
  if (n < 1 || n > LBDD_MAX_N) return fail(LBDD_E_INVAL, "n=%lld outside [1, 2^31-1]", (long long)n);
  const bool table = pen_off != nullptr || pen_val != nullptr;
  if (!cm || !capacity || (!penalty && !strict && !table) || (table && (!pen_off || !pen_val)))
    return fail(LBDD_E_INVAL, "NULL input array");
  if (flags & ~LBDD_CM_DEVICE) return fail(LBDD_E_INVAL, "unknown flags 0x%x", flags);
  std::vector<int32_t> first;                     // a table's first values stand in for pen[]
  if (table) {
    if (pen_off[0] != 0) return fail(LBDD_E_INVAL, "pen_off[0]=%lld, expected 0", (long long)pen_off[0]);
    for (int32_t s = 0; s < k; ++s) {
      if (pen_off[s + 1] <= pen_off[s])
        return fail(LBDD_E_INVAL, "center %d has no penalty values (pen_off not increasing)", s);
      for (int64_t i = pen_off[s]; i < pen_off[s + 1]; ++i) {
        if (pen_val[i] < 1 || pen_val[i] >= lbdd::CM_LIMIT)
          return fail(LBDD_E_INVAL, "pen_val[%lld]=%d outside [1, 2^30)", (long long)i, pen_val[i]);
        if (i > pen_off[s] && pen_val[i] < pen_val[i - 1])
          return fail(LBDD_E_INVAL, "penalties of center %d decrease at pen_val[%lld]", s, (long long)i);
      }
      first.push_back(pen_val[pen_off[s]]);
    }
    penalty = first.data();
  }
  int64_t total = 0;
  for (int32_t s = 0; s < k; ++s) {
    if (capacity[s] < 0) return fail(LBDD_E_INVAL, "capacity[%d]=%d < 0", s, capacity[s]);
    total += capacity[s];
    if (!strict && (penalty[s] < 1 || penalty[s] >= lbdd::CM_LIMIT))
      return fail(LBDD_E_INVAL, "penalty[%d]=%d outside [1, 2^30)", s, penalty[s]);
  }
  const bool dummy = strict && total < n;
  if (dummy && k == LBDD_MAX_K)
    return fail(LBDD_E_INVAL, "excess demand needs a dummy center: k=%d must be below %d", k, LBDD_MAX_K);
  const int32_t k_user = k;
  std::vector<int32_t> capx(capacity, capacity + k), penx;
  if (strict) {
    if (dummy) { capx.push_back((int32_t)(n - total)); k += 1; }
    penx.assign((size_t)k, 1);                    // strict-LBDD has no penalties
    penalty = penx.data();
  }
  capacity = capx.data();
  lbdd_instance *h = new (std::nothrow) lbdd_instance;
  if (!h) return fail(LBDD_E_NOMEM, "host allocation");
  h->k = k; h->n = n; h->st = static_cast<hipStream_t>(hip_stream);
  h->strict = strict; h->k_user = k_user; h->dummy = dummy ? k_user : -1;
  const size_t nk = (size_t)n * (size_t)k;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = dalloc(&h->cm, nk, h->st);
  if (e == hipSuccess) e = dalloc(&h->smin, (size_t)n, h->st);
  if (e == hipSuccess) e = dalloc(&h->cap, (size_t)k, h->st);
  if (e == hipSuccess) e = dalloc(&h->pen, (size_t)k, h->st);
  if (e == hipSuccess) e = dalloc(&h->assign, (size_t)n, h->st);
  if (e == hipSuccess) e = dalloc(&h->load, (size_t)k, h->st);
  if (e == hipSuccess) e = dalloc(&h->members, nk, h->st);
  if (e == hipSuccess) e = dalloc(&h->slot, (size_t)n, h->st);
  if (e == hipSuccess) e = dalloc(&h->unperm, (size_t)n, h->st);
  if (e == hipSuccess) e = dalloc(&h->order, (size_t)n, h->st);
  if (e == hipSuccess) e = dalloc(&h->scalars, (size_t)lbdd::SC_COUNT, h->st);
  if (e == hipSuccess) e = dalloc(&h->W, (size_t)k * k, h->st);
  if (e == hipSuccess) e = dalloc(&h->Wh, (size_t)k * k, h->st);
  if (e == hipSuccess) e = dalloc(&h->WhT, (size_t)k * k, h->st);
  if (e == hipSuccess) e = dalloc(&h->best, (size_t)k * k * lbdd::BEST_M, h->st);
  if (e == hipSuccess) e = dalloc(&h->meta, (size_t)k * k, h->st);
  if (e == hipSuccess) e = dalloc(&h->thr, (size_t)k * k, h->st);
  if (table && e == hipSuccess) e = dalloc(&h->poff, (size_t)k + 1, h->st);
  if (table && e == hipSuccess) e = dalloc(&h->pval, (size_t)pen_off[k], h->st);
  if (e != hipSuccess) { release(h); return hip_fail(e, "device allocation"); }

  // setup scratch: the unpermuted CM (host input only), sort keys, a flag
  const int32_t *cm_dev = cm;
  int32_t *cm_tmp = nullptr, *cm_ext = nullptr, *bad = nullptr, *mx = nullptr;
  int32_t mx_h = 0;                  // read by an async copy: lives until the sync below
  void *work = nullptr;
  int64_t opts[2] = {0, 0};          // read by an async copy: lives until the sync below
  int rc = LBDD_OK;
  do {
    if (!(flags & LBDD_CM_DEVICE)) {
      const size_t nk_user = (size_t)n * (size_t)k_user;
      if ((e = dalloc(&cm_tmp, nk_user, h->st)) != hipSuccess) { rc = hip_fail(e, "device allocation"); break; }
      if ((e = hipMemcpyAsync(cm_tmp, cm, nk_user * 4, hipMemcpyHostToDevice, h->st)) != hipSuccess) {
        rc = hip_fail(e, "copy CM to device"); break;
      }
      cm_dev = cm_tmp;
    }
    if (dummy) {
      // Appendix B: a column for the dummy center, (largest entry + 1) for every unit
      if ((e = dalloc(&cm_ext, nk, h->st)) != hipSuccess || (e = dalloc(&mx, 1, h->st)) != hipSuccess) {
        rc = hip_fail(e, "device allocation"); break;
      }
      if ((e = hipMemcpyAsync(mx, &mx_h, 4, hipMemcpyHostToDevice, h->st)) != hipSuccess ||
          (e = lbdd::launch_extend_dummy(k_user, n, cm_dev, cm_ext, mx, h->st)) != hipSuccess ||
          (e = hipMemcpyAsync(&mx_h, mx, 4, hipMemcpyDeviceToHost, h->st)) != hipSuccess) {
        rc = hip_fail(e, "dummy center"); break;
      }
      cm_dev = cm_ext;
    }
    if ((e = hipMallocAsync(&work, lbdd::setup_work_bytes(k, n), h->st)) != hipSuccess) { rc = hip_fail(e, "device allocation"); break; }
    if ((e = dalloc(&bad, 1, h->st)) != hipSuccess) { rc = hip_fail(e, "device allocation"); break; }
    int32_t zero = 0;
    if ((e = hipMemcpyAsync(bad, &zero, 4, hipMemcpyHostToDevice, h->st)) != hipSuccess) { rc = hip_fail(e, "init flag"); break; }
    if ((e = hipMemcpyAsync(h->cap, capacity, (size_t)k * 4, hipMemcpyHostToDevice, h->st)) != hipSuccess ||
        (e = hipMemcpyAsync(h->pen, penalty, (size_t)k * 4, hipMemcpyHostToDevice, h->st)) != hipSuccess) {
      rc = hip_fail(e, "copy capacities/penalties"); break;
    }
    if (table &&
        ((e = hipMemcpyAsync(h->poff, pen_off, ((size_t)k + 1) * 8, hipMemcpyHostToDevice, h->st)) != hipSuccess ||
         (e = hipMemcpyAsync(h->pval, pen_val, (size_t)pen_off[k] * 4, hipMemcpyHostToDevice, h->st)) != hipSuccess)) {
      rc = hip_fail(e, "copy penalty tables"); break;
    }
    if ((e = lbdd::launch_setup(k, n, cm_dev, h->cm, h->smin, h->order, bad, work, h->st)) != hipSuccess) {
      rc = hip_fail(e, "setup kernels"); break;
    }
    if ((e = lbdd::launch_init_state(h->view(), h->st)) != hipSuccess) { rc = hip_fail(e, "init kernel"); break; }
    // the per-instance options, in adjacent scalar slots
    static_assert(lbdd::SC_SINK_EVERY == lbdd::SC_RATIO + 1, "option slots");
    opts[0] = lbdd::tuned_search_ratio(k, n);
    opts[1] = lbdd::DEFAULT_SINK_EVERY;
    if ((e = hipMemcpyAsync(h->scalars + lbdd::SC_RATIO, opts, sizeof opts, hipMemcpyHostToDevice, h->st)) != hipSuccess) {
      rc = hip_fail(e, "init options"); break;
    }
    int32_t bad_h = 0;
    if ((e = hipMemcpyAsync(&bad_h, bad, 4, hipMemcpyDeviceToHost, h->st)) != hipSuccess ||
        (e = hipStreamSynchronize(h->st)) != hipSuccess) {
      rc = hip_fail(e, "setup"); break;
    }
    if (bad_h) rc = fail(LBDD_E_INVAL, dummy ? "cost matrix has an entry outside [0, 2^30 - 1) (the dummy "
                                               "center costs one more than the largest)"
                                             : "cost matrix has an entry outside [0, 2^30)");
    h->dummy_cost = (int64_t)mx_h + 1;
  } while (0);
  (void)hipStreamSynchronize(h->st);
  if (cm_tmp) (void)hipFreeAsync(cm_tmp, h->st);
  if (cm_ext) (void)hipFreeAsync(cm_ext, h->st);
  if (mx) (void)hipFreeAsync(mx, h->st);
  if (work) (void)hipFreeAsync(work, h->st);
  if (bad) (void)hipFreeAsync(bad, h->st);
  if (rc != LBDD_OK) { release(h); return rc; }
  *out = h;
  return LBDD_OK;
}

}  // namespace

extern "C" {

int lbdd_create(int32_t k, int64_t n, const int32_t *cm, const int32_t *capacity,
                const int32_t *penalty, uint32_t flags, void *hip_stream, lbdd_instance **out) {
  return create_instance(k, n, cm, capacity, penalty, nullptr, nullptr, flags, hip_stream, false, out);
}

int lbdd_create_strict(int32_t k, int64_t n, const int32_t *cm, const int32_t *capacity,
                       uint32_t flags, void *hip_stream, lbdd_instance **out) {
  return create_instance(k, n, cm, capacity, nullptr, nullptr, nullptr, flags, hip_stream, true, out);
}

int lbdd_create_penalty_table(int32_t k, int64_t n, const int32_t *cm, const int32_t *capacity,
                              const int64_t *pen_off, const int32_t *pen_val, uint32_t flags,
                              void *hip_stream, lbdd_instance **out) {
  if (!pen_off || !pen_val) return fail(LBDD_E_INVAL, "NULL penalty table");
  return create_instance(k, n, cm, capacity, nullptr, pen_off, pen_val, flags, hip_stream, false, out);
}

int lbdd_centers(lbdd_instance *h, int32_t *k_graph) {
  if (!h || !k_graph) return fail(LBDD_E_INVAL, "NULL argument");
  *k_graph = h->k;
  return LBDD_OK;
}

// scalar slot of an option, or -1
static int option_slot(int32_t option) {
  return option == LBDD_OPT_SEARCH_RATIO ? lbdd::SC_RATIO
       : option == LBDD_OPT_SINK_EVERY ? lbdd::SC_SINK_EVERY : -1;
}

int lbdd_set_option(lbdd_instance *h, int32_t option, int64_t value) {
  if (!h) return fail(LBDD_E_INVAL, "NULL handle");
  const int slot = option_slot(option);
  if (slot < 0) return fail(LBDD_E_INVAL, "unknown option %d", option);
  if (option == LBDD_OPT_SEARCH_RATIO && (value < lbdd::SEARCH_RATIO_AUTO || value > lbdd::MAX_SEARCH_RATIO))
    return fail(LBDD_E_INVAL, "search ratio %lld outside [-1, 2^20]", (long long)value);
  if (option == LBDD_OPT_SINK_EVERY && (value < 0 || value > lbdd::MAX_SINK_EVERY))
    return fail(LBDD_E_INVAL, "sink period %lld outside [0, 2^20]", (long long)value);
  HIP_TRY(copy_sync(h->scalars + slot, &value, sizeof value, hipMemcpyHostToDevice, h->st), "set option");
  return LBDD_OK;
}

int lbdd_get_option(lbdd_instance *h, int32_t option, int64_t *value) {
  if (!h || !value) return fail(LBDD_E_INVAL, "NULL argument");
  const int slot = option_slot(option);
  if (slot < 0) return fail(LBDD_E_INVAL, "unknown option %d", option);
  HIP_TRY(copy_sync(value, h->scalars + slot, sizeof *value, hipMemcpyDeviceToHost, h->st), "get option");
  return LBDD_OK;
}

int lbdd_solve_iters(lbdd_instance *h, int64_t iters) {
  if (!h) return fail(LBDD_E_INVAL, "NULL handle");
  if (iters < 0) return fail(LBDD_E_INVAL, "iters < 0");
  int64_t end = h->enqueued + iters;
  if (end > h->n || end < h->enqueued) end = h->n;
  const lbdd::InstView v = h->view();
  for (int64_t r = h->enqueued; r < end; r += ITERS_PER_LAUNCH) {
    const int64_t r1 = (end - r > ITERS_PER_LAUNCH) ? r + ITERS_PER_LAUNCH : end;
    HIP_TRY(lbdd::launch_solve(v, r, r1, h->st), "solve kernel launch");
    h->enqueued = r1;
  }
  return LBDD_OK;
}

int lbdd_solve(lbdd_instance *h) {
  if (!h) return fail(LBDD_E_INVAL, "NULL handle");
  return lbdd_solve_iters(h, h->n);
}

int lbdd_objective(lbdd_instance *h, int64_t *out) {
  if (!h || !out) return fail(LBDD_E_INVAL, "NULL argument");
  int64_t sc[lbdd::SC_COUNT];
  int rc = read_scalars(h, sc);
  if (rc) return rc;
  int64_t obj = sc[lbdd::SC_OBJECTIVE];
  if (h->dummy >= 0) {
    // Equation (3) counts the allotted units only: the dummy center's cost,
    // the same for every complete allotment, is taken out again
    int32_t at_dummy = 0;
    HIP_TRY(copy_sync(&at_dummy, h->load + h->dummy, 4, hipMemcpyDeviceToHost, h->st), "copy load");
    obj -= (int64_t)at_dummy * h->dummy_cost;
  }
  *out = obj;
  return LBDD_OK;
}

int lbdd_progress(lbdd_instance *h, int64_t *iters_done) {
  if (!h || !iters_done) return fail(LBDD_E_INVAL, "NULL argument");
  int64_t sc[lbdd::SC_COUNT] = {};
  int rc = read_scalars(h, sc);
  *iters_done = sc[lbdd::SC_DONE];
  return rc;
}

int lbdd_assignment(lbdd_instance *h, int32_t *out, uint32_t flags) {
  if (!h || !out) return fail(LBDD_E_INVAL, "NULL argument");
  if (flags & ~LBDD_OUT_DEVICE) return fail(LBDD_E_INVAL, "unknown flags 0x%x", flags);
  int32_t *dst = (flags & LBDD_OUT_DEVICE) ? out : h->unperm;
  HIP_TRY(lbdd::launch_unpermute(h->n, h->order, h->assign, h->dummy, dst, h->st), "unpermute kernel");
  int64_t sc[lbdd::SC_COUNT];
  int rc = read_scalars(h, sc);
  if (rc) return rc;
  if (!(flags & LBDD_OUT_DEVICE))
    HIP_TRY(copy_sync(out, h->unperm, (size_t)h->n * 4, hipMemcpyDeviceToHost, h->st), "copy assignment");
  return LBDD_OK;
}

int lbdd_snapshot(lbdd_instance *h, int32_t *load, uint64_t *W, int64_t *order) {
  if (!h) return fail(LBDD_E_INVAL, "NULL handle");
  int64_t sc[lbdd::SC_COUNT];
  int rc = read_scalars(h, sc);
  if (rc) return rc;
  if (load) HIP_TRY(copy_sync(load, h->load, (size_t)h->k * 4, hipMemcpyDeviceToHost, h->st), "copy load");
  if (W) HIP_TRY(copy_sync(W, h->W, (size_t)h->k * h->k * 8, hipMemcpyDeviceToHost, h->st), "copy W");
  if (order) HIP_TRY(copy_sync(order, h->order, (size_t)h->n * 8, hipMemcpyDeviceToHost, h->st), "copy order");
  return LBDD_OK;
}

int lbdd_stats(lbdd_instance *h, int64_t *out, int32_t count) {
  if (!h || (!out && count > 0) || count < 0) return fail(LBDD_E_INVAL, "bad argument");
  int64_t sc[lbdd::SC_COUNT];
  HIP_TRY(copy_sync(sc, h->scalars, sizeof sc, hipMemcpyDeviceToHost, h->st), "copy scalars");
  int64_t all[lbdd::SC_NSTATS + 1];
  for (int i = 0; i < lbdd::SC_NSTATS; ++i) all[i] = sc[lbdd::SC_STAT0 + i];
  int dev = 0, khz = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev), "clock rate");
  all[lbdd::SC_NSTATS] = khz;
  const int m = count < lbdd::SC_NSTATS + 1 ? count : lbdd::SC_NSTATS + 1;
  for (int i = 0; i < m; ++i) out[i] = all[i];
  return m;
}

void lbdd_destroy(lbdd_instance *h) { release(h); }

int lbdd_solve_batch(lbdd_instance **hs, int32_t m, void *hip_stream) {
  g_err.clear();
  if (m < 0 || (m > 0 && !hs)) return fail(LBDD_E_INVAL, "bad instance list");
  if (m == 0) return LBDD_OK;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  std::vector<int32_t> idx;
  for (int32_t i = 0; i < m; ++i) {
    if (!hs[i]) return fail(LBDD_E_INVAL, "instance %d is NULL", i);
    for (int32_t j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(LBDD_E_INVAL, "instance %d appears twice", i);
    if (hs[i]->enqueued < hs[i]->n) idx.push_back(i);
  }
  if (idx.empty()) return LBDD_OK;
  // largest remaining work first (longest-processing-time order)
  std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) {
    const double wa = (double)(hs[a]->n - hs[a]->enqueued) * hs[a]->k;
    const double wb = (double)(hs[b]->n - hs[b]->enqueued) * hs[b]->k;
    return wa > wb;
  });
  const int32_t mm = (int32_t)idx.size();
  // device buffer: queue head (padded to 256 bytes), then the items
  const size_t head_bytes = 256;
  std::vector<unsigned char> host(head_bytes + sizeof(lbdd::BatchItem) * (size_t)mm, 0);
  lbdd::BatchItem *items = reinterpret_cast<lbdd::BatchItem *>(host.data() + head_bytes);
  for (int32_t i = 0; i < mm; ++i) {
    items[i].inst = hs[idx[i]]->view();
    items[i].r_begin = hs[idx[i]]->enqueued;
  }
  // the batch runs after whatever is pending on each instance's stream
  hipEvent_t ev = nullptr;
  HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
  for (int32_t i : idx) {
    if (hs[i]->st == st) continue;
    HIP_TRY(hipEventRecord(ev, hs[i]->st), "hipEventRecord");
    HIP_TRY(hipStreamWaitEvent(st, ev, 0), "hipStreamWaitEvent");
  }
  void *dev = nullptr;
  HIP_TRY(hipMallocAsync(&dev, host.size(), st), "device allocation");
  HIP_TRY(hipMemcpyAsync(dev, host.data(), host.size(), hipMemcpyHostToDevice, st), "copy batch items");
  HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");   // host buffer may go
  const size_t lds = lbdd::batch_lds_bytes(items, mm);
  const int workers = lbdd::batch_workers(lds, mm);
  HIP_TRY(lbdd::launch_solve_batch(reinterpret_cast<const lbdd::BatchItem *>(
                                       static_cast<unsigned char *>(dev) + head_bytes),
                                   mm, static_cast<int32_t *>(dev), lds, workers, st),
          "batch kernel launch");
  HIP_TRY(hipFreeAsync(dev, st), "hipFreeAsync");
  // later calls on each instance's own stream see the batch's results
  HIP_TRY(hipEventRecord(ev, st), "hipEventRecord");
  for (int32_t i : idx) {
    hs[i]->enqueued = hs[i]->n;
    if (hs[i]->st != st) HIP_TRY(hipStreamWaitEvent(hs[i]->st, ev, 0), "hipStreamWaitEvent");
  }
  HIP_TRY(hipEventDestroy(ev), "hipEventDestroy");
  return LBDD_OK;
}

size_t lbdd_road_cm_work_bytes(int32_t V, int32_t k) {
  if (V < 1 || k < 1) return 0;
  return lbdd::road_work_bytes(V, k);
}

int lbdd_road_cost_matrix(int32_t V, const int64_t *row_ptr, const int32_t *col, const int32_t *length,
                          int32_t k, const int32_t *centers, int64_t n, const int32_t *units, int32_t *cm,
                          void *work, void *hip_stream) {
  g_err.clear();
  if (V < 1) return fail(LBDD_E_INVAL, "V=%d < 1", V);
  if (k < 1 || k > LBDD_MAX_K) return fail(LBDD_E_INVAL, "k=%d outside [1, %d]", k, LBDD_MAX_K);
  if (n < 1 || n > LBDD_MAX_N) return fail(LBDD_E_INVAL, "n=%lld outside [1, 2^31-1]", (long long)n);
  if (!row_ptr || !col || !length || !centers || !units || !cm || !work)
    return fail(LBDD_E_INVAL, "NULL argument");
  const int rc = lbdd::road_cost_matrix(V, row_ptr, col, length, k, centers, n, units, cm, work,
                                        static_cast<hipStream_t>(hip_stream));
  if (rc < 0) return hip_fail(static_cast<hipError_t>(-rc), "road network kernels");
  if (rc == 1)
    return fail(LBDD_E_INVAL, "road network: offsets not starting at 0 or decreasing, a vertex index "
                              "outside [0, V) or an arc length outside [0, 2^30)");
  if (rc == 2) return fail(LBDD_E_INVAL, "some unit is unreachable from some center, or 2^30 or more away");
  return LBDD_OK;
}

size_t lbdd_best_transfers_batch_work_bytes(int32_t m, const int32_t *k, const int64_t *n) {
  if (m < 1 || m > LBDD_MAX_SCAN_ITEMS || !k || !n) return 0;
  for (int32_t i = 0; i < m; ++i)
    if (k[i] < 1 || k[i] > LBDD_MAX_K || n[i] < 0 || n[i] > LBDD_MAX_N) return 0;
  return lbdd::batch_scan_work_bytes(m, k, n);
}

int lbdd_best_transfers_batch(int32_t m, const int32_t *k, const int64_t *n, const int32_t *const *cm,
                              const int32_t *const *assign, const int32_t *const *rank, uint64_t *const *W,
                              void *work, uint32_t flags, void *hip_stream) {
  g_err.clear();
  if (m < 1 || !k || !n || !cm || !assign || !rank || !W || !work) return fail(LBDD_E_INVAL, "bad argument");
  if (m > LBDD_MAX_SCAN_ITEMS) return fail(LBDD_E_INVAL, "m=%d items: at most %d per call", m, LBDD_MAX_SCAN_ITEMS);
  if (flags & ~LBDD_SCAN_REUSE_GROUPING) return fail(LBDD_E_INVAL, "unknown flags 0x%x", flags);
  for (int32_t i = 0; i < m; ++i) {
    if (k[i] < 1 || k[i] > LBDD_MAX_K) return fail(LBDD_E_INVAL, "item %d: k=%d outside [1, %d]", i, k[i], LBDD_MAX_K);
    if (n[i] < 0 || n[i] > LBDD_MAX_N) return fail(LBDD_E_INVAL, "item %d: n=%lld outside [0, 2^31-1]", i, (long long)n[i]);
    if (!W[i] || (n[i] > 0 && (!cm[i] || !assign[i] || !rank[i]))) return fail(LBDD_E_INVAL, "item %d: NULL array", i);
    if (lbdd::batch_scan_np(k[i], cm[i]) > 8)
      return fail(LBDD_E_INVAL, "item %d: k=%d needs more than 8 column groups per lane (4-byte loads when "
                                "k %% 4 != 0); scan it with lbdd_best_transfers", i, k[i]);
  }
  HIP_TRY(lbdd::launch_batch_scan(m, k, n, cm, assign, rank, W, work, flags & LBDD_SCAN_REUSE_GROUPING,
                                  static_cast<hipStream_t>(hip_stream)),
          "batched scan kernels");
  return LBDD_OK;
}

size_t lbdd_best_transfers_work_bytes(int32_t k, int64_t n) {
  if (k < 1 || n < 0) return 0;
  return lbdd::scan_work_bytes(k, n);
}

int lbdd_best_transfers(int32_t k, int64_t n, const int32_t *cm, const int32_t *assign,
                        const int32_t *rank, uint64_t *W, void *work, uint32_t flags,
                        void *hip_stream) {
  g_err.clear();
  if (k < 1 || k > LBDD_MAX_K) return fail(LBDD_E_INVAL, "k=%d outside [1, %d]", k, LBDD_MAX_K);
  if (n < 0 || n > LBDD_MAX_N) return fail(LBDD_E_INVAL, "n=%lld outside [0, 2^31-1]", (long long)n);
  if (!W || !work || (n > 0 && (!cm || !assign || !rank))) return fail(LBDD_E_INVAL, "NULL argument");
  if (flags & ~LBDD_SCAN_REUSE_GROUPING) return fail(LBDD_E_INVAL, "unknown flags 0x%x", flags);
  HIP_TRY(lbdd::launch_full_scan(k, n, cm, assign, rank, W, work, flags & LBDD_SCAN_REUSE_GROUPING,
                                 static_cast<hipStream_t>(hip_stream)),
          "scan kernels");
  return LBDD_OK;
}

}  // extern "C"
