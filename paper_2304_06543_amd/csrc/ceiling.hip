// ceiling.hip -- lbdd_read_ceiling: a plain streaming read of a device
// buffer, the bandwidth ceiling the cost-matrix scans are measured against.
//
// Each thread reads 16-byte words four strides apart per step (four loads in
// flight), folds them by XOR, and each wavefront XORs its fold into one
// 64-bit word, so the kernel writes nothing else and the compiler keeps
// every load.
#include <hip/hip_runtime.h>

#include "../../include/lbdd.h"
#include "instance.hpp"
#include "lbdd_dev.hpp"

namespace {

constexpr int RC_THREADS = 256;

__global__ __launch_bounds__(RC_THREADS) void read_ceiling_kernel(const uint4 *__restrict__ p, int64_t n16,
                                                                  unsigned long long *out) {
  const int64_t stride = (int64_t)gridDim.x * RC_THREADS;
  int64_t i = (int64_t)blockIdx.x * RC_THREADS + threadIdx.x;
  uint32_t acc = 0;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const uint4 a = p[i], b = p[i + stride], c = p[i + 2 * stride], d = p[i + 3 * stride];
    acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
  }
  for (; i < n16; i += stride) {
    const uint4 a = p[i];
    acc ^= a.x ^ a.y ^ a.z ^ a.w;
  }
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
      static_cast<const uint4 *>(src), bytes / 16, reinterpret_cast<unsigned long long *>(sink));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LBDD_E_DEVICE, "read kernel: %s", hipGetErrorString(e));
  return LBDD_OK;
}

}  // extern "C"
