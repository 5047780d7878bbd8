// noalloc.hip -- lbdd_best_transfers_noalloc: the whole-matrix best-transfer
// scan with its workspace in a fixed device array of this library, for
// callers that cannot allocate device memory.
//
// The workspace of lbdd_best_transfers (the units grouped by center, counts,
// offsets, cursors) lives in `scratch`, a file-scope device array that every
// GPU the library runs on holds until the process ends.  In host code the
// array's name only stands for the symbol: its device address on the current
// device comes from hipGetSymbolAddress, taken once per device on the first
// call there and kept; kernels receive that address, never the name.  The
// call itself allocates nothing: the scan's kernels clear what must start at
// zero (counts, cursors, the table) with fill kernels.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "../../include/lbdd.h"
#include "instance.hpp"
#include "lbdd_dev.hpp"

namespace {

__device__ __align__(256) unsigned char scratch[LBDD_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
std::map<int, void *> g_scratch;   // device ordinal -> address of its scratch

// Address of this device's scratch (nullptr and the error on failure).
void *device_scratch(hipError_t *err) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) { *err = e; return nullptr; }
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_scratch.find(dev);
  if (it != g_scratch.end()) return it->second;
  void *p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr) {
    *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
    return nullptr;
  }
  g_scratch[dev] = p;
  return p;
}

}  // namespace

extern "C" {

int lbdd_best_transfers_noalloc(int32_t k, int64_t n, const int32_t *cm, const int32_t *assign,
                                const int32_t *rank, uint64_t *W, uint32_t flags, void *hip_stream) {
  using lbdd::fail;
  lbdd::g_err.clear();
  if (k < 1 || k > LBDD_MAX_K) return fail(LBDD_E_INVAL, "k=%d outside [1, %d]", k, LBDD_MAX_K);
  if (n < 0 || n > LBDD_MAX_N) return fail(LBDD_E_INVAL, "n=%lld outside [0, 2^31-1]", (long long)n);
  if (!W || (n > 0 && (!cm || !assign || !rank))) return fail(LBDD_E_INVAL, "NULL argument");
  if (flags & ~LBDD_SCAN_REUSE_GROUPING) return fail(LBDD_E_INVAL, "unknown flags 0x%x", flags);
  const size_t need = lbdd::scan_work_bytes(k, n);
  if (need > (size_t)LBDD_NOALLOC_SCRATCH_BYTES)
    return fail(LBDD_E_INVAL, "k=%d, n=%lld need %zu bytes of workspace, more than the %d-byte scratch",
                k, (long long)n, need, LBDD_NOALLOC_SCRATCH_BYTES);
  hipError_t e = hipSuccess;
  void *work = device_scratch(&e);
  if (!work) return fail(LBDD_E_DEVICE, "scratch address: %s", hipGetErrorString(e));
  e = lbdd::launch_full_scan(k, n, cm, assign, rank, W, work, flags & LBDD_SCAN_REUSE_GROUPING,
                             static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(LBDD_E_DEVICE, "scan kernels: %s", hipGetErrorString(e));
  return LBDD_OK;
}

}  // extern "C"
