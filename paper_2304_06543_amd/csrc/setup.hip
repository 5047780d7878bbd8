// setup.hip -- step 1 of ASRAL's main loop (Algorithm 2): every unit's most
// suitable center (the cheapest, smallest index on ties) and the MinDistance
// processing order (ascending cheapest cost, then unit index), followed by a
// permutation of the cost-matrix rows into that order.
//
// The extract-min heap of the paper is replaced by one sort of the unique
// 64-bit keys (cheapest cost << 32 | unit): unique keys need no stability,
// so LDS bitonic tiles plus merge passes (each element finds its output slot
// by a binary search in the partner run) give the exact order.
#include "lbdd_dev.hpp"

namespace lbdd {

namespace {

constexpr int ROWMIN_THREADS = 256;
constexpr int SORT_THREADS = 1024;
constexpr int SORT_TILE = 2 * SORT_THREADS;

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int mask, int width) {
  uint32_t lo = __shfl_xor((uint32_t)v, mask, width);
  uint32_t hi = __shfl_xor((uint32_t)(v >> 32), mask, width);
  return (uint64_t)hi << 32 | lo;
}

// One lane group of G lanes (power of two, <= 64) per row: lanes stride the
// row's columns (coalesced), keep (cost << 32 | column) minima, and reduce with
// xor-shuffles inside the group.  Also flags any cost outside [0, 2^30).
template <int G>
__global__ __launch_bounds__(ROWMIN_THREADS) void rowmin_kernel(int32_t k, int64_t n,
                                                                const int32_t *__restrict__ cm,
                                                                int32_t *__restrict__ smin,
                                                                uint64_t *__restrict__ keys,
                                                                int32_t *__restrict__ bad) {
  const int lane = threadIdx.x % G;
  const int64_t groups_per_grid = (int64_t)gridDim.x * (ROWMIN_THREADS / G);
  int64_t d = (int64_t)blockIdx.x * (ROWMIN_THREADS / G) + threadIdx.x / G;
  for (; d < n; d += groups_per_grid) {
    const int32_t *row = cm + d * k;
    uint64_t best = ~0ull;
    bool badv = false;
    for (int c = lane; c < k; c += G) {
      int32_t v = row[c];
      badv |= (v < 0) | (v >= CM_LIMIT);
      uint64_t key = (uint64_t)(uint32_t)v << 32 | (uint32_t)c;
      best = key < best ? key : best;
    }
    for (int m = G / 2; m > 0; m >>= 1) {
      uint64_t o = shfl_xor_u64(best, m, G);
      best = o < best ? o : best;
    }
    if (badv) atomicOr(bad, 1);
    if (lane == 0) {
      smin[d] = (int32_t)(uint32_t)best;
      keys[d] = (best >> 32) << 32 | (uint64_t)d;   // (cheapest cost, unit)
    }
  }
}

// Sort SORT_TILE keys per block in LDS (bitonic); the tail is padded with
// all-ones keys that are never written back.
__global__ __launch_bounds__(SORT_THREADS) void tile_sort_kernel(int64_t n, uint64_t *keys) {
  __shared__ uint64_t s[SORT_TILE];
  const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
  for (int i = threadIdx.x; i < SORT_TILE; i += SORT_THREADS)
    s[i] = (base + i < n) ? keys[base + i] : ~0ull;
  for (int size = 2; size <= SORT_TILE; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      const int i = threadIdx.x;
      const int lo = 2 * stride * (i / stride) + (i % stride);
      const int hi = lo + stride;
      const bool asc = (lo & size) == 0;
      uint64_t a = s[lo], b = s[hi];
      if ((a > b) == asc) { s[lo] = b; s[hi] = a; }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < SORT_TILE; i += SORT_THREADS)
    if (base + i < n) keys[base + i] = s[i];
}

// number of entries of the sorted run a[0..len) that are < key
__device__ inline int64_t count_less(const uint64_t *a, int64_t len, uint64_t key) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Merge sorted runs of length L pairwise: an element's output slot is its
// index in its own run plus the number of smaller keys in the partner run.
__global__ void merge_pass_kernel(int64_t n, int64_t L, const uint64_t *__restrict__ in,
                                  uint64_t *__restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t key = in[i];
  const int64_t run = i / L;
  const int64_t start = (run & ~1ll) * L;
  if ((run & 1) == 0) {
    const int64_t b0 = start + L;
    const int64_t blen = b0 < n ? (n - b0 < L ? n - b0 : L) : 0;
    out[start + (i - start) + count_less(in + b0, blen, key)] = key;
  } else {
    out[start + (i - start - L) + count_less(in + start, L, key)] = key;
  }
}

__global__ void finish_order_kernel(int64_t n, const uint64_t *__restrict__ keys,
                                    const int32_t *__restrict__ smin,
                                    int64_t *__restrict__ order, int32_t *__restrict__ smin_perm) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t d = (int64_t)(uint32_t)keys[r];
  order[r] = d;
  smin_perm[r] = smin[d];
}

// cm_perm row r = cm row order[r]; one wave per row, 16-byte accesses when the
// row length allows it.
template <bool VEC4>
__global__ __launch_bounds__(256) void permute_rows_kernel(int32_t k, int64_t n,
                                                           const int32_t *__restrict__ cm,
                                                           const int64_t *__restrict__ order,
                                                           int32_t *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * 4;
  for (int64_t r = (int64_t)blockIdx.x * 4 + threadIdx.x / 64; r < n; r += waves) {
    const int64_t d = order[r];
    if (VEC4) {
      const int4 *src = reinterpret_cast<const int4 *>(cm + d * k);
      int4 *dst = reinterpret_cast<int4 *>(out + r * k);
      for (int c = lane; c < k / 4; c += 64) dst[c] = src[c];
    } else {
      for (int c = lane; c < k; c += 64) out[r * k + c] = cm[d * k + c];
    }
  }
}

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Largest entry of the cost matrix (strict-LBDD with excess demand, Appendix
// B: the dummy center costs one more than it for every unit).
__global__ __launch_bounds__(256) void cm_max_kernel(int64_t count, const int32_t *__restrict__ cm,
                                                     int32_t *__restrict__ mx) {
  int32_t m = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    m = max(m, cm[i]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(mx, m);
}

// cm_ext [n][k+1]: the k given columns, then the dummy center's column.
__global__ __launch_bounds__(256) void extend_dummy_kernel(int32_t k, int64_t n,
                                                           const int32_t *__restrict__ cm,
                                                           const int32_t *__restrict__ mx,
                                                           int32_t *__restrict__ out) {
  const int64_t k1 = (int64_t)k + 1;
  const int32_t dummy = *mx + 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n * k1; i += stride) {
    const int64_t d = i / k1, j = i - d * k1;
    out[i] = j < k ? cm[d * k + j] : dummy;
  }
}

}  // namespace

hipError_t launch_extend_dummy(int32_t k, int64_t n, const int32_t *cm, int32_t *cm_ext, int32_t *mx,
                               hipStream_t st) {
  cm_max_kernel<<<2048, 256, 0, st>>>(n * (int64_t)k, cm, mx);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  extend_dummy_kernel<<<4096, 256, 0, st>>>(k, n, cm, mx, cm_ext);
  return hipGetLastError();
}

size_t setup_work_bytes(int32_t k, int64_t n) {
  (void)k;
  return align_up((size_t)n * 4) + 2 * align_up((size_t)n * 8);
}

hipError_t launch_setup(int32_t k, int64_t n, const int32_t *cm_in, int32_t *cm_perm,
                        int32_t *smin_perm, int64_t *order, int32_t *bad_flag, void *work,
                        hipStream_t st) {
  char *w = static_cast<char *>(work);
  int32_t *smin = reinterpret_cast<int32_t *>(w);
  uint64_t *ka = reinterpret_cast<uint64_t *>(w + align_up((size_t)n * 4));
  uint64_t *kb = reinterpret_cast<uint64_t *>(w + align_up((size_t)n * 4) + align_up((size_t)n * 8));

  int G = 1;
  while (G < k && G < 64) G <<= 1;
  const int64_t rows_per_block = ROWMIN_THREADS / G;
  int64_t blocks = (n + rows_per_block - 1) / rows_per_block;
  if (blocks > 65536) blocks = 65536;
  switch (G) {
#define ROWMIN_CASE(g) case g: rowmin_kernel<g><<<(unsigned)blocks, ROWMIN_THREADS, 0, st>>>(k, n, cm_in, smin, ka, bad_flag); break;
    ROWMIN_CASE(1) ROWMIN_CASE(2) ROWMIN_CASE(4) ROWMIN_CASE(8)
    ROWMIN_CASE(16) ROWMIN_CASE(32) ROWMIN_CASE(64)
#undef ROWMIN_CASE
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;

  const int64_t tiles = (n + SORT_TILE - 1) / SORT_TILE;
  tile_sort_kernel<<<(unsigned)tiles, SORT_THREADS, 0, st>>>(n, ka);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  uint64_t *src = ka, *dst = kb;
  const unsigned mblocks = (unsigned)((n + 255) / 256);
  for (int64_t L = SORT_TILE; L < n; L <<= 1) {
    merge_pass_kernel<<<mblocks, 256, 0, st>>>(n, L, src, dst);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    uint64_t *t = src; src = dst; dst = t;
  }
  finish_order_kernel<<<mblocks, 256, 0, st>>>(n, src, smin, order, smin_perm);
  if ((e = hipGetLastError()) != hipSuccess) return e;

  int64_t pblocks = (n + 3) / 4;
  if (pblocks > 65536) pblocks = 65536;
  if (k % 4 == 0 && (uintptr_t)cm_in % 16 == 0)
    permute_rows_kernel<true><<<(unsigned)pblocks, 256, 0, st>>>(k, n, cm_in, order, cm_perm);
  else
    permute_rows_kernel<false><<<(unsigned)pblocks, 256, 0, st>>>(k, n, cm_in, order, cm_perm);
  return hipGetLastError();
}

}  // namespace lbdd
