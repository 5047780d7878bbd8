// scan_batch.hpp -- host launcher of the batched best-transfer scan
// (scan_batch.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbdd {

// column groups per lane an item needs (at most 8 are supported)
int batch_scan_np(int32_t k, const int32_t *cm);
size_t batch_scan_work_bytes(int32_t m, const int32_t *k, const int64_t *n);
hipError_t launch_batch_scan(int32_t m, const int32_t *k, const int64_t *n, const int32_t *const *cm,
                             const int32_t *const *assign, const int32_t *const *rank, uint64_t *const *W,
                             void *work, bool reuse, hipStream_t st);

}  // namespace lbdd
