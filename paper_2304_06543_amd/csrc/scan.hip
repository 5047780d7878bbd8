// scan.hip -- best-transfer table of a whole allotment (definition of Gamma,
// Section 3.2, condensed to the cheapest edge per ordered center pair as in
// the NCyc definition, Section 3.3):
//   W[u][v] = min over units d allotted to u of key(CM(d,v) - CM(d,u), rank(d)).
//
// HBM-bound streaming kernel.  Units are first grouped by their center (a
// counting sort of the allotment into a list of (unit, rank) pairs, ranked
// inside each workgroup so that only one global atomic per center per
// workgroup is needed).  The grouped list is then split into equal contiguous
// shares, one per workgroup of a grid sized to fill the GPU once: a share
// covers one or a few center segments, and within a segment every row has the
// same source center u, so the partial result is one row of k keys instead of
// a k x k table.  Lanes own column quads (16-byte loads); per-lane running
// minima stay in registers over the segment, are combined across the
// workgroup with LDS atomics and leave with one global atomic min per column
// per segment.  Keys are unique, so the result does not depend on the order
// in which rows or segments are reduced.
#include <map>
#include <mutex>

#include "lbdd_dev.hpp"

namespace lbdd {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCATTER_THREADS = 1024;
constexpr int SCATTER_ITEMS = 4;     // units per thread in the scatter pass

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct ScanWork {
  int32_t *count;      // [k]   units per center
  int32_t *cursor;     // [k]   scatter cursors
  int64_t *offset;     // [k+1] start of each center in the unit list
  int2 *units;         // [n]   (unit, rank) grouped by center
};

ScanWork carve(void *work, int32_t k) {
  char *p = static_cast<char *>(work);
  ScanWork w;
  w.count = reinterpret_cast<int32_t *>(p); p += align_up((size_t)k * 4);
  w.cursor = reinterpret_cast<int32_t *>(p); p += align_up((size_t)k * 4);
  w.offset = reinterpret_cast<int64_t *>(p); p += align_up((size_t)(k + 1) * 8);
  w.units = reinterpret_cast<int2 *>(p);
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

// exclusive prefix sum of the counts (k <= LBDD_MAX_K; one workgroup)
__global__ __launch_bounds__(1024) void offsets_kernel(int32_t k, const int32_t *__restrict__ count,
                                                       int64_t *__restrict__ offset) {
  __shared__ int64_t a[1024];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < k; base += 1024) {
    const int i = base + threadIdx.x;
    const int64_t c = i < k ? count[i] : 0;
    a[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {   // inclusive Hillis-Steele scan
      const int64_t va = threadIdx.x >= off ? a[threadIdx.x - off] : 0;
      __syncthreads();
      a[threadIdx.x] += va;
      __syncthreads();
    }
    if (i < k) offset[i] = carry + a[threadIdx.x] - c;
    __syncthreads();
    if (threadIdx.x == 0) carry += a[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) offset[k] = carry;
}

// Group units by center.  Each workgroup ranks its own units per center in
// LDS, reserves one range per center with a single global atomic, and writes.
__global__ __launch_bounds__(SCATTER_THREADS) void scatter_kernel(
    int32_t k, int64_t n, const int32_t *__restrict__ assign, const int32_t *__restrict__ rank,
    const int64_t *__restrict__ offset, int32_t *__restrict__ cursor, int2 *__restrict__ units) {
  extern __shared__ int32_t sh[];      // [k] local counts, then [k] local bases
  int32_t *h = sh, *lbase = sh + k;
  for (int i = threadIdx.x; i < k; i += SCATTER_THREADS) h[i] = 0;
  __syncthreads();
  const int64_t d0 = (int64_t)blockIdx.x * SCATTER_THREADS * SCATTER_ITEMS + threadIdx.x;
  int32_t u[SCATTER_ITEMS], li[SCATTER_ITEMS];
#pragma unroll
  for (int j = 0; j < SCATTER_ITEMS; ++j) {
    const int64_t d = d0 + (int64_t)j * SCATTER_THREADS;
    u[j] = d < n ? assign[d] : -1;
    li[j] = (u[j] >= 0 && u[j] < k) ? atomicAdd(&h[u[j]], 1) : -1;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += SCATTER_THREADS)
    lbase[i] = h[i] ? atomicAdd(&cursor[i], h[i]) : 0;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < SCATTER_ITEMS; ++j) {
    if (li[j] < 0) continue;
    const int64_t d = d0 + (int64_t)j * SCATTER_THREADS;
    units[offset[u[j]] + lbase[u[j]] + li[j]] = make_int2((int32_t)d, rank[d]);
  }
}

__device__ inline uint64_t umin(uint64_t a, uint64_t b) { return b < a ? b : a; }

// Lane layout: LPR lanes per row (a power of two <= 64), each lane owns NP
// column groups of VEC consecutive columns: group q = lane_in_row + j*LPR.
// Each row slot keeps ROWS rows in flight and prefetches the (unit, rank)
// entries of its next ROWS rows while they load, so no iteration waits on a
// dependent list load.
typedef int v4i __attribute__((ext_vector_type(4)));   // native 16-byte vector
// rows in flight per slot: at most 32 loaded values per lane (4 rows when a
// lane holds at most 8 columns, e.g. k <= 512 with 16-byte loads)
template <int VEC, int NP>
constexpr int rows_in_flight() {
  constexpr int r = 32 / (VEC * NP);
  return r < 1 ? 1 : (r > 4 ? 4 : r);
}

template <int VEC, int LPR, int NP, int ROWS>
__device__ inline void scan_rows(int32_t k, int u, const int32_t *__restrict__ cm, const int2 (&ur)[ROWS],
                                 int nvalid, int lane, uint64_t (&best)[NP][VEC]) {
  int32_t v[ROWS][NP][VEC];
  uint32_t bias[ROWS];
#pragma unroll
  for (int t = 0; t < ROWS; ++t) {
    if (t >= nvalid) break;
    const int32_t *row = cm + (int64_t)ur[t].x * k;
    bias[t] = 0x80000000u - (uint32_t)__builtin_nontemporal_load(row + u);
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const int q = lane + j * LPR;
      if (q * VEC >= k) break;
      if constexpr (VEC == 4) {
        const v4i x = __builtin_nontemporal_load(reinterpret_cast<const v4i *>(row) + q);
        v[t][j][0] = x[0]; v[t][j][1] = x[1]; v[t][j][2] = x[2]; v[t][j][3] = x[3];
      } else {
        v[t][j][0] = __builtin_nontemporal_load(row + q);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < ROWS; ++t) {
    if (t >= nvalid) break;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const int q = lane + j * LPR;
      if (q * VEC >= k) break;
#pragma unroll
      for (int e = 0; e < VEC; ++e)
        best[j][e] = umin(best[j][e], (uint64_t)((uint32_t)v[t][j][e] + bias[t]) << 32 | (uint32_t)ur[t].y);
    }
  }
}

template <int VEC, int LPR, int NP>
__global__ __launch_bounds__(SCAN_THREADS) void scan_kernel(int32_t k, const int32_t *__restrict__ cm,
                                                            const int2 *__restrict__ units,
                                                            const int64_t *__restrict__ offset,
                                                            uint64_t *__restrict__ W) {
  extern __shared__ uint64_t red[];   // [k]
  const int64_t total = offset[k];
  const int64_t b = blockIdx.x, G = gridDim.x;
  const int64_t r_lo = total * b / G, r_hi = total * (b + 1) / G;
  if (r_lo >= r_hi) return;
  // center of row r_lo: largest u with offset[u] <= r_lo
  int u;
  {
    int lo = 0, hi = k;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (offset[mid] <= r_lo) lo = mid; else hi = mid;
    }
    u = lo;
  }
  constexpr int SLOTS = SCAN_THREADS / LPR;
  constexpr int ROWS = rows_in_flight<VEC, NP>();
  constexpr int STEP = ROWS * SLOTS;
  const int lane = threadIdx.x % LPR;
  const int slot = threadIdx.x / LPR;
  int64_t seg = r_lo;
  while (seg < r_hi) {
    while (offset[u + 1] <= seg) ++u;            // skip centers with no units here
    const int64_t seg_end = offset[u + 1] < r_hi ? offset[u + 1] : r_hi;
    for (int i = threadIdx.x; i < k; i += SCAN_THREADS) red[i] = KEY_NONE;
    uint64_t best[NP][VEC];
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int e = 0; e < VEC; ++e) best[j][e] = KEY_NONE;
    int2 nxt[ROWS];
    int64_t r = seg + slot;
#pragma unroll
    for (int t = 0; t < ROWS; ++t)
      nxt[t] = (r + t * SLOTS < seg_end) ? units[r + t * SLOTS] : make_int2(0, 0);
    for (; r < seg_end; r += STEP) {
      int2 cur[ROWS];
#pragma unroll
      for (int t = 0; t < ROWS; ++t) cur[t] = nxt[t];
      const int64_t rn = r + STEP;
#pragma unroll
      for (int t = 0; t < ROWS; ++t)
        nxt[t] = (rn + t * SLOTS < seg_end) ? units[rn + t * SLOTS] : make_int2(0, 0);
      const int64_t left = (seg_end - r + SLOTS - 1) / SLOTS;
      scan_rows<VEC, LPR, NP, ROWS>(k, u, cm, cur, left < ROWS ? (int)left : ROWS, lane, best);
    }
    __syncthreads();                             // red initialised
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
    __syncthreads();                             // red reused by the next segment
    seg = seg_end;
  }
}

// MULT resident waves of workgroups: as many per CU as registers and LDS allow.
template <int VEC, int LPR, int NP>
hipError_t launch_scan_t(int32_t k, const int32_t *cm, const ScanWork &w, int cus, int mult,
                         uint64_t *W, hipStream_t st) {
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void *>(&scan_kernel<VEC, LPR, NP>), SCAN_THREADS, (size_t)k * 8);
  if (e != hipSuccess) return e;
  const int blocks = cus * (per_cu > 0 ? per_cu : 1) * mult;
  scan_kernel<VEC, LPR, NP><<<blocks, SCAN_THREADS, (size_t)k * 8, st>>>(k, cm, w.units, w.offset, W);
  return hipGetLastError();
}

// The instantiated tile shapes (VEC, LPR, NP).
struct Shape {
  int vec, lpr, np;
};
constexpr Shape SHAPES[] = {
    {4, 1, 1},  {4, 2, 1},  {4, 4, 1},  {4, 8, 1},  {4, 16, 1}, {4, 16, 2}, {4, 16, 4},
    {4, 16, 8}, {4, 32, 1}, {4, 32, 2}, {4, 32, 4}, {4, 32, 8}, {4, 64, 1}, {4, 64, 2},
    {4, 64, 4}, {4, 64, 8}, {1, 1, 1},  {1, 2, 1},  {1, 4, 1},  {1, 8, 1},  {1, 16, 1},
    {1, 32, 1}, {1, 64, 1}, {1, 64, 2}, {1, 64, 4}, {1, 64, 8}, {1, 64, 16}, {1, 64, 32},
};

hipError_t launch_shape(const ScanCfg &c, int32_t k, const int32_t *cm, const ScanWork &w, int cus,
                        uint64_t *W, hipStream_t st) {
#define LBDD_SCAN_CASE(V, L, P) \
  if (c.vec == V && c.lpr == L && c.np == P) return launch_scan_t<V, L, P>(k, cm, w, cus, c.mult, W, st);
  LBDD_SCAN_CASE(4, 1, 1) LBDD_SCAN_CASE(4, 2, 1) LBDD_SCAN_CASE(4, 4, 1) LBDD_SCAN_CASE(4, 8, 1)
  LBDD_SCAN_CASE(4, 16, 1) LBDD_SCAN_CASE(4, 16, 2) LBDD_SCAN_CASE(4, 16, 4) LBDD_SCAN_CASE(4, 16, 8)
  LBDD_SCAN_CASE(4, 32, 1) LBDD_SCAN_CASE(4, 32, 2) LBDD_SCAN_CASE(4, 32, 4) LBDD_SCAN_CASE(4, 32, 8)
  LBDD_SCAN_CASE(4, 64, 1) LBDD_SCAN_CASE(4, 64, 2) LBDD_SCAN_CASE(4, 64, 4) LBDD_SCAN_CASE(4, 64, 8)
  LBDD_SCAN_CASE(1, 1, 1) LBDD_SCAN_CASE(1, 2, 1) LBDD_SCAN_CASE(1, 4, 1) LBDD_SCAN_CASE(1, 8, 1)
  LBDD_SCAN_CASE(1, 16, 1) LBDD_SCAN_CASE(1, 32, 1) LBDD_SCAN_CASE(1, 64, 1) LBDD_SCAN_CASE(1, 64, 2)
  LBDD_SCAN_CASE(1, 64, 4) LBDD_SCAN_CASE(1, 64, 8) LBDD_SCAN_CASE(1, 64, 16) LBDD_SCAN_CASE(1, 64, 32)
#undef LBDD_SCAN_CASE
  return hipErrorInvalidValue;
}

// configurations chosen by the autotuner, per (k, load width)
std::mutex g_tuned_mu;
std::map<int64_t, ScanCfg> g_tuned;
int64_t tuned_key(int32_t k, bool vec4) { return (int64_t)k * 2 + (vec4 ? 1 : 0); }

}  // namespace

bool scan_cfg_valid(int32_t k, const ScanCfg &c) {
  if (c.mult < 1 || c.mult > 4) return false;
  if ((int64_t)c.lpr * c.np * c.vec < k) return false;   // every column has a lane
  for (const Shape &sh : SHAPES)
    if (sh.vec == c.vec && sh.lpr == c.lpr && sh.np == c.np) return true;
  return false;
}

// Lanes per row follow the number of column groups up to a wavefront, then
// each lane takes more groups.
ScanCfg scan_default_cfg(int32_t k, bool vec4) {
  const int vec = vec4 ? 4 : 1;
  const int groups = (k + vec - 1) / vec;
  ScanCfg c{vec, 64, 1, 1};
  if (groups <= 64) {
    int l = 1;
    while (l < groups) l *= 2;
    c.lpr = l;
  } else {
    int np = 2;
    while (64 * np < groups) np *= 2;
    c.np = np;
  }
  return c;
}

// Candidates: every instantiated shape that covers k columns without more
// than four times the lanes it needs, with one or two resident waves of
// workgroups; the default configuration comes first.
int scan_candidates(int32_t k, bool vec4, ScanCfg *out, int max) {
  int m = 0;
  const ScanCfg d = scan_default_cfg(k, vec4);
  if (m < max) out[m++] = d;
  for (const Shape &sh : SHAPES) {
    if (sh.vec != (vec4 ? 4 : 1)) continue;
    const int64_t cols = (int64_t)sh.lpr * sh.np * sh.vec;
    if (cols < k || cols > 4 * (int64_t)k + 4 * sh.vec) continue;
    for (int mult = 1; mult <= 2; ++mult) {
      const ScanCfg c{sh.vec, sh.lpr, sh.np, mult};
      if (c.lpr == d.lpr && c.np == d.np && c.mult == d.mult) continue;
      if (m < max) out[m++] = c;
    }
  }
  return m;
}

void scan_set_tuned(int32_t k, bool vec4, const ScanCfg &c) {
  std::lock_guard<std::mutex> g(g_tuned_mu);
  g_tuned[tuned_key(k, vec4)] = c;
}

std::vector<ScanTuned> scan_tuned_list() {
  std::lock_guard<std::mutex> g(g_tuned_mu);
  std::vector<ScanTuned> out;
  for (const auto &kv : g_tuned) out.push_back(ScanTuned{(int32_t)(kv.first / 2), (kv.first & 1) != 0, kv.second});
  return out;
}

void scan_clear_tuned() {
  std::lock_guard<std::mutex> g(g_tuned_mu);
  g_tuned.clear();
}

namespace {
__global__ void differ_kernel(const uint64_t *__restrict__ a, const uint64_t *__restrict__ b,
                              int64_t count, int32_t *flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    bad |= a[i] != b[i];
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}
}  // namespace

// *flag |= (a != b) over count entries (the flag is not cleared here).
hipError_t launch_differ(const uint64_t *a, const uint64_t *b, int64_t count, int32_t *flag,
                         hipStream_t st) {
  differ_kernel<<<256, 256, 0, st>>>(a, b, count, flag);
  return hipGetLastError();
}

bool scan_vec4_ok(int32_t k, const int32_t *cm) { return (k % 4 == 0) && ((uintptr_t)cm % 16 == 0); }


size_t scan_work_bytes(int32_t k, int64_t n) {
  return 2 * align_up((size_t)k * 4) + align_up((size_t)(k + 1) * 8) + align_up((size_t)n * 8);
}

// Clear W and, unless an earlier call's grouping is reused, group the units
// by center.
hipError_t launch_scan_group(int32_t k, int64_t n, const int32_t *assign, const int32_t *rank,
                             uint64_t *W, void *work, bool regroup, hipStream_t st) {
  ScanWork w = carve(work, k);
  hipError_t e;
  // the counts are cleared too, unless the grouping of a previous call is reused
  fill_kernel<<<256, 256, 0, st>>>((int64_t)k * k, KEY_NONE, W, regroup ? k : 0, w.count, w.cursor);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (n == 0 || !regroup) return hipSuccess;
  int64_t hb = (n + 1023) / 1024;
  if (hb > 2048) hb = 2048;
  histogram_kernel<<<(unsigned)hb, 1024, (size_t)k * 4, st>>>(k, n, assign, w.count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  offsets_kernel<<<1, 1024, 0, st>>>(k, w.count, w.offset);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t per_block = (int64_t)SCATTER_THREADS * SCATTER_ITEMS;
  scatter_kernel<<<(unsigned)((n + per_block - 1) / per_block), SCATTER_THREADS, (size_t)k * 8, st>>>(
      k, n, assign, rank, w.offset, w.cursor, w.units);
  return hipGetLastError();
}

// The streaming pass over the grouped units with tile configuration c.
hipError_t launch_scan_only(int32_t k, const int32_t *cm, void *work, const ScanCfg &c, uint64_t *W,
                            hipStream_t st) {
  if (!scan_cfg_valid(k, c)) return hipErrorInvalidValue;
  int dev = 0, cus = 0;
  hipError_t e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  return launch_shape(c, k, cm, carve(work, k), cus, W, st);
}

hipError_t launch_full_scan(int32_t k, int64_t n, const int32_t *cm, const int32_t *assign,
                            const int32_t *rank, uint64_t *W, void *work, bool reuse_grouping,
                            hipStream_t st) {
  hipError_t e = launch_scan_group(k, n, assign, rank, W, work, !reuse_grouping, st);
  if (e != hipSuccess || n == 0) return e;
  const bool vec4 = scan_vec4_ok(k, cm);
  ScanCfg c = scan_default_cfg(k, vec4);
  tune_cache_autoload();
  {
    std::lock_guard<std::mutex> g(g_tuned_mu);
    auto it = g_tuned.find(tuned_key(k, vec4));
    if (it != g_tuned.end()) c = it->second;
  }
  return launch_scan_only(k, cm, work, c, W, st);
}

}  // namespace lbdd
