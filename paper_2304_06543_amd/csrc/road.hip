// road.hip -- the cost matrix from a road network (construction of CM,
// Section 3.5; the paper's datasets, Section 5): CM(d, s) is the length of a
// shortest path from the vertex of center s to the vertex of unit d.
//
// One workgroup per center runs a label-correcting search over the network's
// arcs (CSR, non-negative integer lengths).  Round r relaxes every arc out of
// the vertices whose label dropped in round r - 1, with global atomic minima
// on the labels; a vertex whose label drops is appended to the next round's
// frontier once (a per-vertex round stamp taken by atomic exchange).  A round
// may read labels lowered earlier in the same round: every lowering puts the
// vertex in the next frontier, where it is read again after the barrier, so
// when a round lowers nothing no arc can shorten any label and every label
// is met by a path -- the labels are the shortest distances, whatever order
// the relaxations took.  Distances are unique values, so the result is exact.
// A gather kernel then writes CM rows from the per-center label arrays
// through LDS tiles (reads along units, writes along centers).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "road.hpp"

namespace lbdd {

namespace {

constexpr int RT = 512;                       // threads per search workgroup
constexpr int32_t DINF = INT32_MAX;           // unreached
constexpr int32_t COST_LIMIT = 1 << 30;       // CM entries lie in [0, 2^30)

// Layout of the work buffer for a chunk of `kc` centers over V vertices:
// flags (256 B), then per center dist [V], stamp [V], front [2][V].
struct RoadWork {
  int32_t *flags;    // [0]: bad input, [1]: a distance >= 2^30 or unreached, [2]: round cap hit
  int32_t *dist;     // [kc][V]
  uint32_t *stamp;   // [kc][V] round whose frontier holds the vertex
  int32_t *front;    // [kc][2][V]
};

__host__ __device__ inline RoadWork carve(void *work, int32_t V, int32_t kc) {
  char *p = static_cast<char *>(work);
  RoadWork w;
  w.flags = reinterpret_cast<int32_t *>(p);
  p += 256;
  w.dist = reinterpret_cast<int32_t *>(p);
  p += (size_t)kc * V * 4;
  w.stamp = reinterpret_cast<uint32_t *>(p);
  p += (size_t)kc * V * 4;
  w.front = reinterpret_cast<int32_t *>(p);
  return w;
}

// Input checks that need no arc array: CSR offsets, center and unit vertices.
__global__ void check_vertices_kernel(int32_t V, const int64_t *__restrict__ row_ptr, int32_t k,
                                      const int32_t *__restrict__ centers, int64_t n,
                                      const int32_t *__restrict__ units, int32_t *flags) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int bad = 0;
  if (t0 == 0 && row_ptr[0] != 0) bad = 1;
  for (int64_t u = t0; u < V; u += stride) bad |= row_ptr[u + 1] < row_ptr[u];
  for (int64_t s = t0; s < k; s += stride) bad |= centers[s] < 0 || centers[s] >= V;
  for (int64_t d = t0; d < n; d += stride) bad |= units[d] < 0 || units[d] >= V;
  if (bad) atomicOr(&flags[0], 1);
}

// Arc checks, once the offsets are known to be sane: heads in [0, V), lengths
// in [0, 2^30).
__global__ void check_arcs_kernel(int32_t V, int64_t E, const int32_t *__restrict__ col,
                                  const int32_t *__restrict__ len, int32_t *flags) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < E; i += stride)
    bad |= col[i] < 0 || col[i] >= V || len[i] < 0 || len[i] >= COST_LIMIT;
  if (bad) atomicOr(&flags[0], 1);
}

// Centers c0 .. c0 + gridDim.x - 1, one per workgroup.
__global__ __launch_bounds__(RT) void road_search_kernel(int32_t V, const int64_t *__restrict__ row_ptr,
                                                         const int32_t *__restrict__ col,
                                                         const int32_t *__restrict__ len,
                                                         const int32_t *__restrict__ centers, int32_t c0,
                                                         RoadWork w, int64_t max_rounds) {
  __shared__ int32_t cnt[3];                   // frontier sizes, by round mod 3
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  int32_t *dist = w.dist + (size_t)c * V;
  uint32_t *stamp = w.stamp + (size_t)c * V;
  int32_t *front = w.front + (size_t)c * 2 * V;
  const int32_t src = centers[c0 + c];
  for (int64_t v = tid; v < V; v += RT) {
    dist[v] = v == src ? 0 : DINF;
    stamp[v] = v == src ? 0u : ~0u;
  }
  if (tid == 0) {
    front[0] = src;
    cnt[0] = 1;
    cnt[1] = 0;
    cnt[2] = 0;
  }
  __syncthreads();
  for (int64_t r = 0;; ++r) {
    const int32_t nf = cnt[r % 3];
    if (nf == 0) break;
    if (r >= max_rounds) {                     // cannot happen with lengths >= 0
      if (tid == 0) atomicOr(&w.flags[2], 1);
      break;
    }
    if (tid == 0) cnt[(r + 2) % 3] = 0;        // the round after next starts empty
    int32_t *F = front + (size_t)(r & 1) * V;
    int32_t *Fn = front + (size_t)((r + 1) & 1) * V;
    const uint32_t next = (uint32_t)(r + 1);
    for (int32_t i = tid; i < nf; i += RT) {
      // the label that put u in this frontier was written by an atomic in L2:
      // read it there (a plain load could hit an older copy in this CU's L1)
      const int32_t u = __hip_atomic_load(&F[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int64_t du = __hip_atomic_load(&dist[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int64_t a1 = row_ptr[u + 1];
      for (int64_t a = row_ptr[u]; a < a1; ++a) {
        const int32_t v = col[a];
        const int64_t cand = du + len[a];
        if (cand < dist[v]) {                  // labels only drop: an older copy never skips
          const int32_t old = atomicMin(&dist[v], (int32_t)cand);
          if (cand < old && atomicExch(&stamp[v], next) != next)
            Fn[atomicAdd(&cnt[(r + 1) % 3], 1)] = v;
        }
      }
    }
    __syncthreads();
  }
}

// CM[d][s] = dist of center s at the vertex of unit d, for the chunk's
// centers; 64 units x 64 centers per workgroup through an LDS tile.
__global__ __launch_bounds__(256) void road_gather_kernel(int32_t V, int32_t k, int64_t n,
                                                          const int32_t *__restrict__ units, int32_t c0,
                                                          int32_t kc, RoadWork w, int32_t *__restrict__ cm) {
  __shared__ int32_t tile[64][65];
  const int64_t d0 = (int64_t)blockIdx.x * 64;
  const int t0 = blockIdx.y * 64;
  int bad = 0;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int j = e & 63, t = e >> 6;          // j: unit (fastest), t: center
    const int64_t d = d0 + j;
    if (d < n && t0 + t < kc) tile[t][j] = w.dist[(size_t)(t0 + t) * V + units[d]];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int t = e & 63, j = e >> 6;          // t: center (fastest), j: unit
    const int64_t d = d0 + j;
    if (d < n && t0 + t < kc) {
      const int32_t x = tile[t][j];
      bad |= x >= COST_LIMIT;                  // unreached (DINF) or too far
      cm[d * k + c0 + t0 + t] = x;
    }
  }
  if (bad) atomicOr(&w.flags[1], 1);
}

}  // namespace

size_t road_work_bytes(int32_t V, int32_t k) {
  const int32_t kc = k < ROAD_CHUNK ? k : ROAD_CHUNK;
  return 256 + (size_t)kc * V * 16;
}

// Validates the network (synchronising once to read the offsets' verdict and
// the arc count), then runs the searches and gathers chunk by chunk.
// Returns 0, 1 (bad input), 2 (a unit unreachable or 2^30 or more away) or a
// negative hipError_t.
int road_cost_matrix(int32_t V, const int64_t *row_ptr, const int32_t *col, const int32_t *len, int32_t k,
                     const int32_t *centers, int64_t n, const int32_t *units, int32_t *cm, void *work,
                     hipStream_t st) {
  const int32_t kc_max = k < ROAD_CHUNK ? k : ROAD_CHUNK;
  RoadWork w = carve(work, V, kc_max);
  int32_t flags[3] = {0, 0, 0};
  hipError_t e;
  if ((e = hipMemcpyAsync(w.flags, flags, sizeof flags, hipMemcpyHostToDevice, st)) != hipSuccess) return -(int)e;
  check_vertices_kernel<<<1024, 256, 0, st>>>(V, row_ptr, k, centers, n, units, w.flags);
  if ((e = hipGetLastError()) != hipSuccess) return -(int)e;
  int64_t E = 0;
  if ((e = hipMemcpyAsync(flags, w.flags, sizeof flags, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipMemcpyAsync(&E, row_ptr + V, sizeof E, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return -(int)e;
  if (flags[0]) return 1;
  check_arcs_kernel<<<2048, 256, 0, st>>>(V, E, col, len, w.flags);
  if ((e = hipGetLastError()) != hipSuccess) return -(int)e;
  if ((e = hipMemcpyAsync(flags, w.flags, sizeof flags, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return -(int)e;
  if (flags[0]) return 1;
  const int64_t max_rounds = 4 * (int64_t)V + 8;
  for (int32_t c0 = 0; c0 < k; c0 += kc_max) {
    const int32_t kc = k - c0 < kc_max ? k - c0 : kc_max;
    road_search_kernel<<<kc, RT, 0, st>>>(V, row_ptr, col, len, centers, c0, w, max_rounds);
    if ((e = hipGetLastError()) != hipSuccess) return -(int)e;
    const dim3 grid((unsigned)((n + 63) / 64), (unsigned)((kc + 63) / 64));
    road_gather_kernel<<<grid, 256, 0, st>>>(V, k, n, units, c0, kc, w, cm);
    if ((e = hipGetLastError()) != hipSuccess) return -(int)e;
  }
  if ((e = hipMemcpyAsync(flags, w.flags, sizeof flags, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return -(int)e;
  if (flags[1] || flags[2]) return 2;
  return 0;
}

}  // namespace lbdd
