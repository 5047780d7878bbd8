// ceiling.hip -- lbdd_read_ceiling: a plain streaming read of a device
// buffer, the bandwidth ceiling the cost-matrix scans are measured against.
//
// Each workgroup reads one contiguous share of the buffer in 16-byte
// nontemporal loads, eight in flight per thread, folds them by XOR, and each
// wavefront XORs its fold into one 64-bit word, so the kernel writes nothing
// else and the compiler keeps every load.
#include <hip/hip_runtime.h>

#include "../../include/lbdd.h"
#include "instance.hpp"
#include "lbdd_dev.hpp"

namespace {

constexpr int RC_THREADS = 256;
constexpr int RC_UNROLL = 8;
typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t fold(v4i a) { return (uint32_t)(a.x ^ a.y ^ a.z ^ a.w); }

// Each workgroup streams one contiguous share of the buffer, RC_UNROLL
// 16-byte loads per thread in flight, nontemporal (the data is read once).
__global__ __launch_bounds__(RC_THREADS) void read_ceiling_kernel(const v4i *__restrict__ p, int64_t n16,
                                                                  unsigned long long *out) {
  const int64_t per = (n16 + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per;
  const int64_t b1 = b0 + per < n16 ? b0 + per : n16;
  int64_t i = b0 + threadIdx.x;
  uint32_t acc = 0;
  for (; i + (RC_UNROLL - 1) * RC_THREADS < b1; i += RC_UNROLL * RC_THREADS) {
    v4i v[RC_UNROLL];
#pragma unroll
    for (int u = 0; u < RC_UNROLL; ++u) v[u] = __builtin_nontemporal_load(p + i + u * RC_THREADS);
#pragma unroll
    for (int u = 0; u < RC_UNROLL; ++u) acc ^= fold(v[u]);
  }
  for (; i < b1; i += RC_THREADS) acc ^= fold(__builtin_nontemporal_load(p + i));
  for (int off = 32; off > 0; off >>= 1) acc ^= __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0 && acc) atomicXor(out, (unsigned long long)acc);
}

}  // namespace

extern "C" {

int lbdd_read_ceiling(const void *src, int64_t bytes, uint64_t *sink, int32_t blocks, void *hip_stream) {
  using lbdd::fail;
  lbdd::g_err.clear();
  if (!src || !sink) return fail(LBDD_E_INVAL, "NULL argument");
  if (bytes < 0 || bytes % 16 != 0 || (uintptr_t)src % 16 != 0)
    return fail(LBDD_E_INVAL, "bytes must be a non-negative multiple of 16 and src 16-byte aligned");
  if (blocks < 1 || blocks > 65536) return fail(LBDD_E_INVAL, "blocks=%d outside [1, 65536]", blocks);
  if (bytes == 0) return LBDD_OK;
  read_ceiling_kernel<<<blocks, RC_THREADS, 0, static_cast<hipStream_t>(hip_stream)>>>(
      static_cast<const v4i *>(src), bytes / 16, reinterpret_cast<unsigned long long *>(sink));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LBDD_E_DEVICE, "read kernel: %s", hipGetErrorString(e));
  return LBDD_OK;
}

}  // extern "C"
