// scan_batch.hip -- best-transfer tables of many allotments in one sequence of
// launches (definition of Gamma, Section 3.2, condensed per ordered center
// pair): for every item i,
//   W_i[u][v] = min over units d allotted to u of key(CM_i(d,v) - CM_i(d,u), rank_i(d)).
//
// The same streaming design as the single-instance scan, made independent of
// the number of items: every pass is one launch over all items.
//   fill       workgroups over (item, table slice) clear the tables and counters;
//   histogram  workgroups own 4096-unit blocks of the concatenated units of all
//   scatter    items (the item of a block by binary search over block offsets)
//              and group each item's units by center with one global atomic
//              per center per workgroup;
//   offsets    one workgroup per item;
//   scan       the host cuts every item's rows into chunks of about equal
//              weight (a row weighs its length plus a fixed cost; at least
//              two chunks per resident workgroup, none below ~256 KB, none
//              across items); the workgroups claim chunks from a counter and
//              a chunk walks (item, center) segments.  Items with 16-byte
//              and with 4-byte loads run as two launches.  The lane layout is chosen per item at run time:
//              LPR lanes per row (a power of two up to 64) and NP column
//              groups of 1 or 4 columns per lane, so small and large k both
//              keep full wavefronts and 16-byte loads where the rows allow.
//              Each launch is compiled for its load width and the largest
//              NP among its items, so each keeps as many rows in flight as
//              its own registers allow.
// Keys are unique, so no result depends on the order of the reductions.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "scan_batch.hpp"

namespace lbdd {

namespace {

constexpr uint64_t NONE = ~0ull;
constexpr int BS_THREADS = 256;         // scan workgroup
constexpr int BG_THREADS = 1024;        // grouping workgroups
constexpr int BG_ITEMS = 4;             // units per thread in the grouping passes
constexpr int64_t BG_UNITS = (int64_t)BG_THREADS * BG_ITEMS;
constexpr int CHUNKS_PER_BLOCK = 2;     // scan chunks per resident workgroup (at least)

inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct Item {
  const int32_t *cm;
  const int32_t *assign;
  const int32_t *rank;
  uint64_t *W;
  int32_t *count;        // [k]
  int32_t *cursor;       // [k]
  int64_t *offset;       // [k + 1]
  int2 *units;           // [n] (unit, rank) grouped by center
  int64_t n;
  int64_t row0;          // first row of the item in the concatenated rows
  int64_t blk0;          // first grouping block of the item
  int32_t k;
  int32_t vec4;          // 16-byte loads
  int32_t lpr;           // lanes per row
  int32_t np;            // column groups per lane
};

__device__ inline uint64_t umin(uint64_t a, uint64_t b) { return b < a ? b : a; }

// index of the last item whose first grouping block is <= b
__device__ inline int find_item(const Item *items, int m, int64_t b) {
  int lo = 0, hi = m;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (items[mid].blk0 <= b) lo = mid; else hi = mid;
  }
  return lo;
}

// A row costs its k elements plus a fixed ROW_COST (its unit entry, its
// anchor cost and the per-row bookkeeping), in elements.
constexpr int64_t ROW_COST = 16;
// smallest chunk of the streaming pass, in weighted elements (~256 KB)
constexpr int64_t MIN_CHUNK = 1 << 16;

// Grouped rows [lo, hi) of one item: the unit of work of the streaming pass.
struct Chunk {
  int64_t lo, hi;
  int32_t item;
  int32_t pad;
};

// clears every table, the grouping counters (the offsets of a previous
// grouping are left as they are) and the scan's chunk counter
// (grid: blockIdx.y = item, blockIdx.x = a slice of FILL_SLICE table entries)
constexpr int64_t FILL_SLICE = 1 << 14;
__global__ __launch_bounds__(256) void bfill_kernel(const Item *__restrict__ items, int32_t *next) {
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 2) next[threadIdx.x] = 0;   // one counter per load width
  const Item it = items[blockIdx.y];
  const int64_t kk = (int64_t)it.k * it.k;
  const int64_t i1 = ((int64_t)blockIdx.x + 1) * FILL_SLICE < kk ? ((int64_t)blockIdx.x + 1) * FILL_SLICE : kk;
  for (int64_t i = (int64_t)blockIdx.x * FILL_SLICE + threadIdx.x; i < i1; i += 256) it.W[i] = NONE;
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < it.k; i += 256) {
      it.count[i] = 0;
      it.cursor[i] = 0;
    }
}

// units per center of each item; assign outside [0, k) is not allotted
__global__ __launch_bounds__(BG_THREADS) void bhist_kernel(const Item *__restrict__ items, int m) {
  extern __shared__ int32_t h[];
  const Item it = items[find_item(items, m, blockIdx.x)];
  for (int i = threadIdx.x; i < it.k; i += BG_THREADS) h[i] = 0;
  __syncthreads();
  const int64_t d0 = ((int64_t)blockIdx.x - it.blk0) * BG_UNITS;
#pragma unroll
  for (int j = 0; j < BG_ITEMS; ++j) {
    const int64_t d = d0 + (int64_t)j * BG_THREADS + threadIdx.x;
    if (d < it.n) {
      const int32_t u = it.assign[d];
      if (u >= 0 && u < it.k) atomicAdd(&h[u], 1);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < it.k; i += BG_THREADS)
    if (h[i]) atomicAdd(&it.count[i], h[i]);
}

// exclusive prefix sums of each item's counts, one workgroup per item
__global__ __launch_bounds__(1024) void boffsets_kernel(const Item *__restrict__ items) {
  __shared__ int64_t a[1024];
  __shared__ int64_t carry;
  const Item it = items[blockIdx.x];
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < it.k; base += 1024) {
    const int i = base + threadIdx.x;
    const int64_t c = i < it.k ? it.count[i] : 0;
    a[threadIdx.x] = c;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int64_t va = threadIdx.x >= off ? a[threadIdx.x - off] : 0;
      __syncthreads();
      a[threadIdx.x] += va;
      __syncthreads();
    }
    if (i < it.k) it.offset[i] = carry + a[threadIdx.x] - c;
    __syncthreads();
    if (threadIdx.x == 0) carry += a[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) it.offset[it.k] = carry;
}

// group each item's units by center: local ranks in LDS, one global range
// reservation per center per workgroup
__global__ __launch_bounds__(BG_THREADS) void bscatter_kernel(const Item *__restrict__ items, int m) {
  extern __shared__ int32_t sh[];        // [k] local counts, then [k] local bases
  const Item it = items[find_item(items, m, blockIdx.x)];
  int32_t *h = sh, *lbase = sh + it.k;
  for (int i = threadIdx.x; i < it.k; i += BG_THREADS) h[i] = 0;
  __syncthreads();
  const int64_t d0 = ((int64_t)blockIdx.x - it.blk0) * BG_UNITS;
  int32_t u[BG_ITEMS], li[BG_ITEMS];
#pragma unroll
  for (int j = 0; j < BG_ITEMS; ++j) {
    const int64_t d = d0 + (int64_t)j * BG_THREADS + threadIdx.x;
    u[j] = d < it.n ? it.assign[d] : -1;
    li[j] = (u[j] >= 0 && u[j] < it.k) ? atomicAdd(&h[u[j]], 1) : -1;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < it.k; i += BG_THREADS)
    lbase[i] = h[i] ? atomicAdd(&it.cursor[i], h[i]) : 0;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < BG_ITEMS; ++j) {
    if (li[j] < 0) continue;
    const int64_t d = d0 + (int64_t)j * BG_THREADS + threadIdx.x;
    it.units[it.offset[u[j]] + lbase[u[j]] + li[j]] = make_int2((int32_t)d, it.rank[d]);
  }
}

typedef int v4i __attribute__((ext_vector_type(4)));

// rows in flight per lane: at most 32 loaded values, and at most 4 rows of
// 16-byte loads or 8 rows of 4-byte loads (short rows need more of them in
// flight to keep enough bytes moving)
template <int NP, bool VEC4>
constexpr int bs_rows() {
  constexpr int r = 32 / (NP * (VEC4 ? 4 : 1));
  constexpr int cap = VEC4 ? 4 : 8;
  return r < 1 ? 1 : (r > cap ? cap : r);
}

// fold up to ROWS rows of center u into the lane's running minima; a lane
// owns column groups lane + j * lpr (j < np) of 4 (VEC4) or 1 columns
template <int NP, int ROWS, bool VEC4>
__device__ inline void brows(const Item &it, int u, const int2 (&ur)[ROWS], int nvalid, int lane,
                             uint64_t (&best)[NP][VEC4 ? 4 : 1]) {
  constexpr int VW = VEC4 ? 4 : 1;
  int32_t v[ROWS][NP][VW];
  uint32_t bias[ROWS];
  const int k = it.k;
#pragma unroll
  for (int t = 0; t < ROWS; ++t) {
    if (t >= nvalid) break;
    const int32_t *row = it.cm + (int64_t)ur[t].x * k;
    bias[t] = 0x80000000u - (uint32_t)__builtin_nontemporal_load(row + u);
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const int q = lane + j * it.lpr;
      if (j >= it.np || q * VW >= k) break;
      if constexpr (VEC4) {
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
      const int q = lane + j * it.lpr;
      if (j >= it.np || q * VW >= k) break;
#pragma unroll
      for (int e = 0; e < VW; ++e)
        best[j][e] = umin(best[j][e], (uint64_t)((uint32_t)v[t][j][e] + bias[t]) << 32 | (uint32_t)ur[t].y);
    }
  }
}

// one (item, center) segment of grouped rows [lr, lend): per-lane minima,
// then the workgroup's row of keys through LDS, then the item's table
template <int NP, bool VEC4>
__device__ inline void bsegment(const Item &it, int u, int64_t lr, int64_t lend, uint64_t *red) {
  constexpr int ROWS = bs_rows<NP, VEC4>();
  constexpr int VW = VEC4 ? 4 : 1;
  const int lpr = it.lpr;
  const int lane = threadIdx.x & (lpr - 1);
  const int slot = threadIdx.x / lpr;
  const int slots = BS_THREADS / lpr;
  const int step = ROWS * slots;
  for (int i = threadIdx.x; i < it.k; i += BS_THREADS) red[i] = NONE;
  uint64_t best[NP][VW];
#pragma unroll
  for (int j = 0; j < NP; ++j)
#pragma unroll
    for (int e = 0; e < VW; ++e) best[j][e] = NONE;
  int2 nxt[ROWS];
  int64_t r = lr + slot;
#pragma unroll
  for (int t = 0; t < ROWS; ++t) nxt[t] = (r + t * slots < lend) ? it.units[r + t * slots] : make_int2(0, 0);
  for (; r < lend; r += step) {
    int2 cur[ROWS];
#pragma unroll
    for (int t = 0; t < ROWS; ++t) cur[t] = nxt[t];
    const int64_t rn = r + step;
#pragma unroll
    for (int t = 0; t < ROWS; ++t) nxt[t] = (rn + t * slots < lend) ? it.units[rn + t * slots] : make_int2(0, 0);
    const int64_t left = (lend - r + slots - 1) / slots;
    brows<NP, ROWS, VEC4>(it, u, cur, left < ROWS ? (int)left : ROWS, lane, best);
  }
  __syncthreads();                                // red initialised
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    if (j >= it.np) break;
    const int q = lane + j * lpr;
#pragma unroll
    for (int e = 0; e < VW; ++e) {
      const int col = q * VW + e;
      if (col < it.k && best[j][e] != NONE)
        atomicMin((unsigned long long *)&red[col], (unsigned long long)best[j][e]);
    }
  }
  __syncthreads();
  for (int v = threadIdx.x; v < it.k; v += BS_THREADS)
    if (v != u && red[v] != NONE)
      atomicMin((unsigned long long *)&it.W[(int64_t)u * it.k + v], (unsigned long long)red[v]);
  __syncthreads();                                // red reused by the next segment
}

// The workgroups claim chunks [c0, c1) from a counter until none is left
// (rows cost different time per byte in different items: claiming keeps
// every workgroup busy to the end).  A chunk stays inside one item; its first
// center is found by one parallel pass over the item's offsets.  Items with
// 16-byte and with 4-byte loads run as two launches, each compiled for its
// own load width, so that each keeps the registers (and rows in flight) it
// needs.
template <int NP, bool VEC4>
__global__ __launch_bounds__(BS_THREADS) void bscan_kernel(const Item *__restrict__ items,
                                                           const Chunk *__restrict__ chunks, int32_t c0,
                                                           int32_t c1, int32_t *__restrict__ next) {
  extern __shared__ uint64_t red[];               // [max k]
  __shared__ int32_t claim, first_u;
  for (;;) {
    if (threadIdx.x == 0) claim = c0 + atomicAdd(next, 1);
    __syncthreads();
    const int32_t c = claim;
    __syncthreads();                              // every thread has read the claim
    if (c >= c1) break;
    const Chunk ch = chunks[c];
    const Item it = items[ch.item];
    const int64_t nall = it.offset[it.k];         // units allotted (grouped)
    int64_t lr = ch.lo;
    const int64_t lend = ch.hi < nall ? ch.hi : nall;
    if (lr >= lend) continue;
    for (int t = threadIdx.x; t < it.k; t += BS_THREADS)
      if (it.offset[t] <= lr && lr < it.offset[t + 1]) first_u = t;   // exactly one center
    __syncthreads();
    int u = first_u;
    while (lr < lend) {
      while (it.offset[u + 1] <= lr) ++u;         // centers with no units here
      const int64_t se = it.offset[u + 1] < lend ? it.offset[u + 1] : lend;
      bsegment<NP, VEC4>(it, u, lr, se, red);
      lr = se;
    }
  }
}

// resident workgroups of bscan_kernel<NP, VEC4> (query), or its launch
template <int NP, bool VEC4>
hipError_t launch_bscan(bool query, int &blocks, const Item *items, const Chunk *chunks, int32_t c0, int32_t c1,
                        int32_t kmax, int32_t *next, hipStream_t st) {
  if (query) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
             &per_cu, reinterpret_cast<const void *>(&bscan_kernel<NP, VEC4>), BS_THREADS, (size_t)kmax * 8)) !=
        hipSuccess)
      return e;
    blocks = cus * (per_cu > 0 ? per_cu : 1);
    return hipSuccess;
  }
  bscan_kernel<NP, VEC4><<<blocks, BS_THREADS, (size_t)kmax * 8, st>>>(items, chunks, c0, c1, next);
  return hipGetLastError();
}

// smallest of 1, 2, 4, 8 that is >= np
inline int np_class(int np) { return np <= 1 ? 1 : np <= 2 ? 2 : np <= 4 ? 4 : 8; }

hipError_t launch_bscan_for(bool vec4, int np, bool query, int &blocks, const Item *items, const Chunk *chunks,
                            int32_t c0, int32_t c1, int32_t kmax, int32_t *next, hipStream_t st) {
#define LBDD_BSCAN_CASE(V, P) \
  if (vec4 == V && np == P) return launch_bscan<P, V>(query, blocks, items, chunks, c0, c1, kmax, next, st);
  LBDD_BSCAN_CASE(true, 1) LBDD_BSCAN_CASE(true, 2) LBDD_BSCAN_CASE(true, 4) LBDD_BSCAN_CASE(true, 8)
  LBDD_BSCAN_CASE(false, 1) LBDD_BSCAN_CASE(false, 2) LBDD_BSCAN_CASE(false, 4) LBDD_BSCAN_CASE(false, 8)
#undef LBDD_BSCAN_CASE
  return hipErrorInvalidValue;
}

// lanes per row and column groups per lane of an item: about two groups of
// 4 columns or four single columns per lane, so that short rows share a
// wavefront (more rows, and bytes, in flight per wavefront)
void item_layout(int32_t k, bool vec4, int32_t &lpr, int32_t &np) {
  const int vec = vec4 ? 4 : 1;
  const int groups = (k + vec - 1) / vec;
  const int target = vec4 ? 2 : 4;
  const int need = (groups + target - 1) / target;
  lpr = 1;
  while (lpr < need && lpr < 64) lpr *= 2;
  np = (groups + lpr - 1) / lpr;
}

}  // namespace

// chunks an item can be cut into: one per MIN_CHUNK of its weight, plus one
int64_t max_chunks(int32_t k, int64_t n) { return n == 0 ? 0 : n * (k + ROW_COST) / MIN_CHUNK + 1; }

size_t batch_scan_work_bytes(int32_t m, const int32_t *k, const int64_t *n) {
  int64_t nch = 0;
  for (int32_t i = 0; i < m; ++i) nch += max_chunks(k[i], n[i]);
  size_t b = align_up((size_t)m * sizeof(Item)) + align_up((size_t)nch * sizeof(Chunk)) + 256;
  for (int32_t i = 0; i < m; ++i)
    b += 2 * align_up((size_t)k[i] * 4) + align_up((size_t)(k[i] + 1) * 8) + align_up((size_t)n[i] * 8);
  return b;
}

int batch_scan_np(int32_t k, const int32_t *cm) {
  int32_t lpr, np;
  item_layout(k, k % 4 == 0 && (uintptr_t)cm % 16 == 0, lpr, np);
  return np;
}

// Work buffer: item descriptors, the chunk table, the chunk counter, then
// each item's grouping (counts, cursors, offsets, grouped units).
hipError_t launch_batch_scan(int32_t m, const int32_t *k, const int64_t *n, const int32_t *const *cm,
                             const int32_t *const *assign, const int32_t *const *rank, uint64_t *const *W,
                             void *work, bool reuse, hipStream_t st) {
  int64_t nch_max = 0, weight = 0;
  for (int32_t i = 0; i < m; ++i) {
    nch_max += max_chunks(k[i], n[i]);
    weight += n[i] * (k[i] + ROW_COST);
  }
  const size_t items_bytes = align_up((size_t)m * sizeof(Item));
  const size_t chunk_bytes = align_up((size_t)nch_max * sizeof(Chunk));
  Item *dev_items = static_cast<Item *>(work);
  Chunk *dev_chunks = reinterpret_cast<Chunk *>(static_cast<char *>(work) + items_bytes);
  int32_t *next = reinterpret_cast<int32_t *>(static_cast<char *>(work) + items_bytes + chunk_bytes);
  char *p = reinterpret_cast<char *>(next) + 256;
  // descriptors and chunk table in one host buffer, copied at once
  std::vector<char> host(items_bytes + (size_t)nch_max * sizeof(Chunk));
  Item *items = reinterpret_cast<Item *>(host.data());
  int64_t row0 = 0, blk0 = 0;
  int32_t kmax = 1, np4 = 1, np1 = 1;
  for (int32_t i = 0; i < m; ++i) {
    Item &it = items[i];
    it.cm = cm[i]; it.assign = assign[i]; it.rank = rank[i]; it.W = W[i];
    it.k = k[i]; it.n = n[i];
    it.count = reinterpret_cast<int32_t *>(p); p += align_up((size_t)k[i] * 4);
    it.cursor = reinterpret_cast<int32_t *>(p); p += align_up((size_t)k[i] * 4);
    it.offset = reinterpret_cast<int64_t *>(p); p += align_up((size_t)(k[i] + 1) * 8);
    it.units = reinterpret_cast<int2 *>(p); p += align_up((size_t)n[i] * 8);
    it.row0 = row0; row0 += n[i];
    it.blk0 = blk0; blk0 += (n[i] + BG_UNITS - 1) / BG_UNITS;
    it.vec4 = (k[i] % 4 == 0 && (uintptr_t)cm[i] % 16 == 0) ? 1 : 0;
    item_layout(k[i], it.vec4, it.lpr, it.np);
    if (k[i] > kmax) kmax = k[i];
    if (it.vec4 && it.np > np4) np4 = it.np;
    if (!it.vec4 && it.np > np1) np1 = it.np;
  }
  if (np4 > 8 || np1 > 8) return hipErrorInvalidValue;
  hipError_t e;
  // per load width: resident workgroups, then chunks of about
  // weight / (CHUNKS_PER_BLOCK * blocks), at least MIN_CHUNK, cut inside each
  // item into equal row ranges; 16-byte items' chunks first
  int blocks[2] = {0, 0};
  int32_t cut[3] = {0, 0, 0};
  Chunk *ch = reinterpret_cast<Chunk *>(host.data() + items_bytes);
  int32_t nch = 0;
  for (int kind = 0; kind < 2; ++kind) {
    const bool v4 = kind == 0;
    int64_t wk = 0;
    for (int32_t i = 0; i < m; ++i)
      if ((items[i].vec4 != 0) == v4) wk += n[i] * (k[i] + ROW_COST);
    cut[kind] = nch;
    if (wk == 0) continue;
    if ((e = launch_bscan_for(v4, np_class(v4 ? np4 : np1), true, blocks[kind], nullptr, nullptr, 0, 0, kmax,
                              nullptr, st)) != hipSuccess)
      return e;
    int64_t cw = wk / ((int64_t)CHUNKS_PER_BLOCK * blocks[kind]);
    if (cw < MIN_CHUNK) cw = MIN_CHUNK;
    for (int32_t i = 0; i < m; ++i) {
      if (n[i] == 0 || (items[i].vec4 != 0) != v4) continue;
      int64_t c = (n[i] * (k[i] + ROW_COST) + cw - 1) / cw;
      if (c > max_chunks(k[i], n[i])) c = max_chunks(k[i], n[i]);
      for (int64_t j = 0; j < c; ++j) {
        const int64_t lo = n[i] * j / c, hi = n[i] * (j + 1) / c;
        if (lo < hi) ch[nch++] = Chunk{lo, hi, i, 0};
      }
    }
  }
  cut[2] = nch;
  (void)weight;
  if (!reuse) {
    // in stream order (an earlier call on this stream may still read the
    // same work buffer); the wait keeps the host copy alive until the copy
    // has happened
    if ((e = hipMemcpyAsync(work, host.data(), host.size(), hipMemcpyHostToDevice, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return e;
  }
  const int64_t slices = ((int64_t)kmax * kmax + FILL_SLICE - 1) / FILL_SLICE;
  bfill_kernel<<<dim3((unsigned)slices, (unsigned)m), 256, 0, st>>>(dev_items, next);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (reuse) blk0 = 0;                       // the grouping in work is kept
  if (blk0 > 0) {
    bhist_kernel<<<(unsigned)blk0, BG_THREADS, (size_t)kmax * 4, st>>>(dev_items, m);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (!reuse) {
    boffsets_kernel<<<m, 1024, 0, st>>>(dev_items);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (blk0 > 0) {
    bscatter_kernel<<<(unsigned)blk0, BG_THREADS, (size_t)kmax * 8, st>>>(dev_items, m);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  for (int kind = 0; kind < 2; ++kind) {
    if (cut[kind + 1] == cut[kind]) continue;
    const bool v4 = kind == 0;
    if ((e = launch_bscan_for(v4, np_class(v4 ? np4 : np1), false, blocks[kind], dev_items, dev_chunks, cut[kind],
                              cut[kind + 1], kmax, next + kind, st)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

}  // namespace lbdd
