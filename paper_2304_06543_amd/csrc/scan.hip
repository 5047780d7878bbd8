// scan.hip -- best-transfer table of a whole allotment (definition of Gamma,
// Section 3.2, condensed to the cheapest edge per ordered center pair as in
// the NCyc definition, Section 3.3):
//   W[u][v] = min over units d allotted to u of key(CM(d,v) - CM(d,u), rank(d)).
//
// HBM-bound streaming kernel.  Units are first grouped by their center (a
// counting sort of the allotment into a list of (unit, rank) pairs), so that a
// workgroup streams rows that all share one source center u and its partial
// result is one row of k keys instead of a k x k table.  Lanes own column
// quads (16-byte loads); per-lane running minima stay in registers for the
// whole chunk, are combined across the workgroup with LDS atomics and leave
// with one global atomic min per column per chunk.  Keys are unique, so the
// result does not depend on the order in which rows or chunks are reduced.
#include "lbdd_dev.hpp"

namespace lbdd {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int CHUNK_ROWS = 512;

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct ScanWork {
  int32_t *count;      // [k]   units per center
  int32_t *cursor;     // [k]   scatter cursors
  int64_t *offset;     // [k+1] start of each center in the unit list
  int64_t *chunk_off;  // [k+1] first chunk of each center
  int2 *units;         // [n]   (unit, rank) grouped by center
};

ScanWork carve(void *work, int32_t k, int64_t n) {
  char *p = static_cast<char *>(work);
  ScanWork w;
  w.count = reinterpret_cast<int32_t *>(p); p += align_up((size_t)k * 4);
  w.cursor = reinterpret_cast<int32_t *>(p); p += align_up((size_t)k * 4);
  w.offset = reinterpret_cast<int64_t *>(p); p += align_up((size_t)(k + 1) * 8);
  w.chunk_off = reinterpret_cast<int64_t *>(p); p += align_up((size_t)(k + 1) * 8);
  w.units = reinterpret_cast<int2 *>(p);
  (void)n;
  return w;
}

__global__ void fill_kernel(int64_t count, uint64_t value, uint64_t *out, int32_t k,
                            int32_t *zero_a, int32_t *zero_b) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    out[i] = value;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += stride) {
    zero_a[i] = 0;
    zero_b[i] = 0;
  }
}

// units per center; entries outside [0, k) count as not allotted
__global__ void histogram_kernel(int32_t k, int64_t n, const int32_t *__restrict__ assign,
                                 int32_t *__restrict__ count) {
  extern __shared__ int32_t h[];
  for (int i = threadIdx.x; i < k; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n; d += stride) {
    const int32_t u = assign[d];
    if (u >= 0 && u < k) atomicAdd(&h[u], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += blockDim.x)
    if (h[i]) atomicAdd(&count[i], h[i]);
}

// exclusive prefix sums of the counts and of the per-center chunk counts
// (k <= LBDD_MAX_K; one workgroup, sequential over 1024-wide blocks)
__global__ __launch_bounds__(1024) void offsets_kernel(int32_t k, const int32_t *__restrict__ count,
                                                       int64_t *__restrict__ offset,
                                                       int64_t *__restrict__ chunk_off) {
  __shared__ int64_t a[1024], b[1024];
  __shared__ int64_t carry_a, carry_b;
  if (threadIdx.x == 0) { carry_a = 0; carry_b = 0; }
  __syncthreads();
  for (int base = 0; base < k; base += 1024) {
    const int i = base + threadIdx.x;
    const int64_t c = i < k ? count[i] : 0;
    a[threadIdx.x] = c;
    b[threadIdx.x] = (c + CHUNK_ROWS - 1) / CHUNK_ROWS;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {   // inclusive Hillis-Steele scan
      const int64_t va = threadIdx.x >= off ? a[threadIdx.x - off] : 0;
      const int64_t vb = threadIdx.x >= off ? b[threadIdx.x - off] : 0;
      __syncthreads();
      a[threadIdx.x] += va;
      b[threadIdx.x] += vb;
      __syncthreads();
    }
    if (i < k) {
      offset[i] = carry_a + a[threadIdx.x] - c;
      chunk_off[i] = carry_b + b[threadIdx.x] - (c + CHUNK_ROWS - 1) / CHUNK_ROWS;
    }
    __syncthreads();
    if (threadIdx.x == 0) { carry_a += a[1023]; carry_b += b[1023]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { offset[k] = carry_a; chunk_off[k] = carry_b; }
}

__global__ void scatter_kernel(int32_t k, int64_t n, const int32_t *__restrict__ assign,
                               const int32_t *__restrict__ rank, const int64_t *__restrict__ offset,
                               int32_t *__restrict__ cursor, int2 *__restrict__ units) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < n; d += stride) {
    const int32_t u = assign[d];
    if (u < 0 || u >= k) continue;
    const int32_t j = atomicAdd(&cursor[u], 1);
    units[offset[u] + j] = make_int2((int32_t)d, rank[d]);
  }
}

__device__ inline uint64_t umin(uint64_t a, uint64_t b) { return b < a ? b : a; }

// Lane layout: LPR lanes per row (a power of two <= 64), each lane owns NP
// column groups of VEC consecutive columns: group q = lane_in_row + j*LPR.
template <int VEC, int LPR, int NP>
__global__ __launch_bounds__(SCAN_THREADS) void scan_kernel(int32_t k, const int32_t *__restrict__ cm,
                                                            const int2 *__restrict__ units,
                                                            const int64_t *__restrict__ offset,
                                                            const int64_t *__restrict__ chunk_off,
                                                            uint64_t *__restrict__ W) {
  extern __shared__ uint64_t red[];   // [k]
  const int64_t c = blockIdx.x;
  // center of this chunk: largest u with chunk_off[u] <= c
  int lo = 0, hi = k;   // invariant: chunk_off[lo] <= c < chunk_off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (chunk_off[mid] <= c) lo = mid; else hi = mid;
  }
  const int u = lo;
  const int64_t r0 = offset[u] + (c - chunk_off[u]) * CHUNK_ROWS;
  int64_t r1 = r0 + CHUNK_ROWS;
  if (r1 > offset[u + 1]) r1 = offset[u + 1];

  for (int i = threadIdx.x; i < k; i += SCAN_THREADS) red[i] = KEY_NONE;

  constexpr int SLOTS = SCAN_THREADS / LPR;        // rows processed side by side
  const int lane = threadIdx.x % LPR;
  const int slot = threadIdx.x / LPR;
  uint64_t best[NP][VEC];
#pragma unroll
  for (int j = 0; j < NP; ++j)
#pragma unroll
    for (int e = 0; e < VEC; ++e) best[j][e] = KEY_NONE;

  for (int64_t r = r0 + slot; r < r1; r += SLOTS) {
    const int2 ur = units[r];
    const int32_t *row = cm + (int64_t)ur.x * k;
    const uint32_t bias = 0x80000000u - (uint32_t)row[u];   // delta + 2^31 = v + bias
    const uint64_t rk = (uint32_t)ur.y;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const int q = lane + j * LPR;
      if (q * VEC >= k) break;
      int32_t v[VEC];
      if (VEC == 4) {
        const int4 t = reinterpret_cast<const int4 *>(row)[q];
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
      } else {
        v[0] = row[q];
      }
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const uint64_t key = (uint64_t)((uint32_t)v[e] + bias) << 32 | rk;
        best[j][e] = umin(best[j][e], key);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    const int q = lane + j * LPR;
    if (q * VEC >= k) break;
#pragma unroll
    for (int e = 0; e < VEC; ++e)
      if (best[j][e] != KEY_NONE)
        atomicMin((unsigned long long *)&red[q * VEC + e], (unsigned long long)best[j][e]);
  }
  __syncthreads();
  for (int v = threadIdx.x; v < k; v += SCAN_THREADS)
    if (v != u && red[v] != KEY_NONE)
      atomicMin((unsigned long long *)&W[(int64_t)u * k + v], (unsigned long long)red[v]);
}

template <int VEC, int LPR, int NP>
hipError_t launch_scan_t(int32_t k, const int32_t *cm, const ScanWork &w, int64_t nchunks,
                         uint64_t *W, hipStream_t st) {
  scan_kernel<VEC, LPR, NP><<<(unsigned)nchunks, SCAN_THREADS, (size_t)k * 8, st>>>(
      k, cm, w.units, w.offset, w.chunk_off, W);
  return hipGetLastError();
}

template <int VEC>
hipError_t dispatch_scan(int32_t k, const int32_t *cm, const ScanWork &w, int64_t nchunks,
                         uint64_t *W, hipStream_t st) {
  const int groups = (k + VEC - 1) / VEC;      // column groups per row
  if (groups <= 1) return launch_scan_t<VEC, 1, 1>(k, cm, w, nchunks, W, st);
  if (groups <= 2) return launch_scan_t<VEC, 2, 1>(k, cm, w, nchunks, W, st);
  if (groups <= 4) return launch_scan_t<VEC, 4, 1>(k, cm, w, nchunks, W, st);
  if (groups <= 8) return launch_scan_t<VEC, 8, 1>(k, cm, w, nchunks, W, st);
  if (groups <= 16) return launch_scan_t<VEC, 16, 1>(k, cm, w, nchunks, W, st);
  if (groups <= 32) return launch_scan_t<VEC, 32, 1>(k, cm, w, nchunks, W, st);
  if (groups <= 64) return launch_scan_t<VEC, 64, 1>(k, cm, w, nchunks, W, st);
  if (groups <= 128) return launch_scan_t<VEC, 64, 2>(k, cm, w, nchunks, W, st);
  if (groups <= 256) return launch_scan_t<VEC, 64, 4>(k, cm, w, nchunks, W, st);
  if (groups <= 512) return launch_scan_t<VEC, 64, 8>(k, cm, w, nchunks, W, st);
  if (groups <= 1024) return launch_scan_t<VEC, 64, 16>(k, cm, w, nchunks, W, st);
  return launch_scan_t<VEC, 64, 32>(k, cm, w, nchunks, W, st);
}

}  // namespace

size_t scan_work_bytes(int32_t k, int64_t n) {
  return 2 * align_up((size_t)k * 4) + 2 * align_up((size_t)(k + 1) * 8) + align_up((size_t)n * 8);
}

// Upper bound on the chunk count for n units over k centers.
static int64_t max_chunks(int32_t k, int64_t n) { return n / CHUNK_ROWS + k; }

hipError_t launch_full_scan(int32_t k, int64_t n, const int32_t *cm, const int32_t *assign,
                            const int32_t *rank, uint64_t *W, void *work, hipStream_t st) {
  ScanWork w = carve(work, k, n);
  hipError_t e;
  fill_kernel<<<256, 256, 0, st>>>((int64_t)k * k, KEY_NONE, W, k, w.count, w.cursor);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int64_t hb = (n + 1023) / 1024;
  if (hb > 2048) hb = 2048;
  histogram_kernel<<<(unsigned)hb, 1024, (size_t)k * 4, st>>>(k, n, assign, w.count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  offsets_kernel<<<1, 1024, 0, st>>>(k, w.count, w.offset, w.chunk_off);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  scatter_kernel<<<(unsigned)hb, 1024, 0, st>>>(k, n, assign, rank, w.offset, w.cursor, w.units);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // The chunk count is only known on the device; launch the upper bound and
  // let surplus workgroups find an empty row range.
  const int64_t nchunks = max_chunks(k, n);
  const bool vec = (k % 4 == 0) && ((uintptr_t)cm % 16 == 0);
  return vec ? dispatch_scan<4>(k, cm, w, nchunks, W, st)
             : dispatch_scan<1>(k, cm, w, nchunks, W, st);
}

}  // namespace lbdd
