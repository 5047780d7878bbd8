// solve.hip -- the ASRAL main loop (Algorithm 2) on one workgroup.
//
// Each iteration r (row r of the permuted cost matrix is the r-th unit of the
// MinDistance order):
//   allot     the unit goes to its most suitable center s; the objective grows
//             by CM + (s full ? pen[s] : 0); its k-1 transfer keys are
//             min-inserted into row s of the best-transfer table W.
//   cycle     Negative Cycle Refinement (Algorithm 1) with anchor s, on the
//             NCyc split graph built on the fly from W.  Skipped exactly when
//             the insert left row s of W unchanged: W is then the table of the
//             previous allotment, which has no negative cycle (Lemmas 1-2),
//             so no negative s_out -> s_in path exists.
//   path      when s was full: Negative Path Refinement (Appendix A) on the
//             NPath split graph (edges into s_in are penalty differences).
//   apply     the units on the chosen path move; every center that lost a
//             unit has its row of W recomputed from its members (the scan of
//             the cost matrix), the path's last center min-inserts its new unit.
//
// Bellman-Ford runs in synchronous rounds.  Only nodes whose label changed in
// the previous round are relaxed from: a node that did not change cannot give
// a strictly better label (every target already saw its value one round
// earlier), so labels and predecessors equal those of full rounds.  Candidate
// (label, node) pairs are packed so that one unsigned min keeps the smallest
// label and, on ties, the smallest predecessor node.
//
// One workgroup of 1024 threads owns the instance.  W lives in LDS when it
// fits (k <= ~135) and in global memory (L2-resident) otherwise.
#include "lbdd_dev.hpp"

namespace lbdd {

namespace {

constexpr int NT = 1024;

struct Lds {
  uint64_t *W;      // [k][k] (LDS copy or the global table)
  uint64_t *red;    // [k+1] per-target minimum
  int64_t *dist;    // [k+1]
  int32_t *pred;    // [k+1]
  int32_t *front0;  // [k+1] frontier lists (double-buffered)
  int32_t *front1;
  int32_t *load;    // [k]
  int32_t *cap;     // [k]
  int32_t *pen;     // [k]
  int32_t *mrow;    // [k+1] moved rows of the applied path
  int32_t *mfrom;   // [k+1]
  int32_t *mto;     // [k+1]
};

struct Scalars {
  int64_t obj;
  int64_t stats[SC_NSTATS];
  int32_t status;
  int32_t nfront[2];
  int32_t nmoves;
  int32_t apply;
  int32_t vacant;
};

// Minimum of a per-thread candidate over each target, combined in LDS.
__device__ inline void lds_min(uint64_t *p, uint64_t v) {
  if (v != KEY_NONE) atomicMin((unsigned long long *)p, (unsigned long long)v);
}

// Recompute row u of W from the members of center u (definition of Gamma):
// W[u][w] = min over rows x at u of key(CM[x][w] - CM[x][u], x).
__device__ __forceinline__ void rescan_center(const InstView &I, const Lds &L, Scalars &S, int u) {
  const int k = I.k;
  const int tid = threadIdx.x;
  const int m = L.load[u];
  const int32_t *mem = I.members + (int64_t)u * I.n;
  for (int w = tid; w < k; w += NT) L.red[w] = KEY_NONE;
  __syncthreads();
  if (k <= NT) {
    const int G = NT / k;
    const int w = tid % k, g = tid / k;
    if (g < G && w != u) {
      uint64_t best = KEY_NONE;
      int i = g;
      for (; i + 3 * G < m; i += 4 * G) {
        const int32_t x0 = mem[i], x1 = mem[i + G], x2 = mem[i + 2 * G], x3 = mem[i + 3 * G];
        const int32_t *r0 = I.cm + (int64_t)x0 * k, *r1 = I.cm + (int64_t)x1 * k;
        const int32_t *r2 = I.cm + (int64_t)x2 * k, *r3 = I.cm + (int64_t)x3 * k;
        const int32_t a0 = r0[w] - r0[u], a1 = r1[w] - r1[u];
        const int32_t a2 = r2[w] - r2[u], a3 = r3[w] - r3[u];
        uint64_t k0 = pack_key(a0, x0), k1 = pack_key(a1, x1);
        uint64_t k2 = pack_key(a2, x2), k3 = pack_key(a3, x3);
        k0 = k1 < k0 ? k1 : k0;
        k2 = k3 < k2 ? k3 : k2;
        k0 = k2 < k0 ? k2 : k0;
        best = k0 < best ? k0 : best;
      }
      for (; i < m; i += G) {
        const int32_t x = mem[i];
        const int32_t *rx = I.cm + (int64_t)x * k;
        uint64_t key = pack_key(rx[w] - rx[u], x);
        best = key < best ? key : best;
      }
      lds_min(&L.red[w], best);
    }
  } else {
    for (int w = tid; w < k; w += NT) {
      if (w == u) continue;
      uint64_t best = KEY_NONE;
      for (int i = 0; i < m; ++i) {
        const int32_t x = mem[i];
        const int32_t *rx = I.cm + (int64_t)x * k;
        uint64_t key = pack_key(rx[w] - rx[u], x);
        best = key < best ? key : best;
      }
      L.red[w] = best;
    }
  }
  __syncthreads();
  for (int w = tid; w < k; w += NT) L.W[(int64_t)u * k + w] = L.red[w];
  if (tid == 0) S.stats[ST_ROWS_SCANNED] += m;
  __syncthreads();
}

// Min-insert row x's transfer keys into row v of W; returns (block-wide)
// whether any entry strictly decreased.
__device__ __forceinline__ int insert_row(const InstView &I, const Lds &L, int x, int v) {
  const int k = I.k;
  const int32_t *rx = I.cm + (int64_t)x * k;
  const int32_t base = rx[v];
  int changed = 0;
  for (int w = threadIdx.x; w < k; w += NT) {
    if (w == v) continue;
    const uint64_t key = pack_key(rx[w] - base, (uint32_t)x);
    uint64_t *p = &L.W[(int64_t)v * k + w];
    if (key < *p) { *p = key; changed = 1; }
  }
  return __syncthreads_or(changed);
}

// Weight of edge u -> v on the split graph (node s = s_out, node k = s_in);
// returns false when the edge does not exist.
__device__ inline bool edge_weight(const InstView &I, const Lds &L, int s, int mode, int u, int v,
                                   int64_t &w) {
  const int k = I.k;
  if (u == k || v == s || u == v) return false;
  if (v == k) {
    if (u == s) return false;
    if (mode == 0) {
      const uint64_t key = L.W[(int64_t)u * k + s];
      if (key == KEY_NONE) return false;
      w = key_delta(key);
    } else {
      w = (int64_t)(L.load[u] >= L.cap[u] ? L.pen[u] : 0) - L.pen[s];
    }
    return true;
  }
  const uint64_t key = L.W[(int64_t)u * k + v];
  if (key == KEY_NONE) return false;
  w = key_delta(key);
  return true;
}

// Bellman-Ford from node s on the split graph; leaves dist/pred in LDS.
// Returns false (and sets the status) on a change in round k+1.
__device__ __forceinline__ bool bellman_ford(const InstView &I, const Lds &L, Scalars &S, int s, int mode) {
  const int k = I.k, K1 = k + 1;
  const int tid = threadIdx.x;
  for (int v = tid; v < K1; v += NT) { L.dist[v] = DIST_NONE; L.pred[v] = -1; }
  if (tid == 0) { S.nfront[0] = 1; S.nfront[1] = 0; }
  __syncthreads();
  if (tid == 0) { L.dist[s] = 0; L.front0[0] = s; }
  int cur = 0;
  for (int t = 1; t <= K1; ++t) {
    for (int v = tid; v < K1; v += NT) L.red[v] = KEY_NONE;
    __syncthreads();
    const int nf = S.nfront[cur];
    const int32_t *F = cur ? L.front1 : L.front0;
    if (K1 <= NT) {
      const int G = NT / K1;
      const int v = tid % K1, g = tid / K1;
      if (g < G && v != s) {
        uint64_t best = KEY_NONE;
        for (int j = g; j < nf; j += G) {
          const int u = F[j];
          int64_t w;
          if (!edge_weight(I, L, s, mode, u, v, w)) continue;
          const uint64_t c = pack_cand(L.dist[u] + w, u);
          best = c < best ? c : best;
        }
        lds_min(&L.red[v], best);
      }
    } else {
      for (int v = tid; v < K1; v += NT) {
        if (v == s) continue;
        uint64_t best = KEY_NONE;
        for (int j = 0; j < nf; ++j) {
          const int u = F[j];
          int64_t w;
          if (!edge_weight(I, L, s, mode, u, v, w)) continue;
          const uint64_t c = pack_cand(L.dist[u] + w, u);
          best = c < best ? c : best;
        }
        L.red[v] = best;
      }
    }
    __syncthreads();
    // update: strict improvement only; changed nodes form the next frontier
    for (int v = tid; v < K1; v += NT) {
      const uint64_t c = L.red[v];
      if (c == KEY_NONE) continue;
      const int64_t d = cand_dist(c);
      if (d < L.dist[v]) {
        L.dist[v] = d;
        L.pred[v] = cand_node(c);
        const int idx = atomicAdd(&S.nfront[cur ^ 1], 1);
        (cur ? L.front0 : L.front1)[idx] = v;
      }
    }
    __syncthreads();
    const int nnext = S.nfront[cur ^ 1];
    if (tid == 0) S.stats[ST_BF_ROUNDS] += 1;
    __syncthreads();
    if (nnext == 0) return true;
    if (tid == 0) S.nfront[cur] = 0;   // becomes the list after next
    cur ^= 1;
  }
  if (tid == 0) S.status = -5;   // LBDD_E_INTERNAL: negative cycle reachable
  __syncthreads();
  return false;
}

// One refinement (mode 0: Algorithm 1, mode 1: Appendix A) anchored at s.
__device__ __forceinline__ void refine(const InstView &I, const Lds &L, Scalars &S, int s, int mode) {
  const int k = I.k;
  const int tid = threadIdx.x;
  if (tid == 0) S.stats[mode == 0 ? ST_CYC_SEARCH : ST_PATH_SEARCH] += 1;
  if (!bellman_ford(I, L, S, s, mode)) return;
  const int64_t D = L.dist[k];
  if (D == DIST_NONE || D >= 0) return;       // only strictly negative refinements apply
  if (tid == 0) {
    // walk back from s_in; node list is reversed (path[len-1] == s)
    int len = 0;
    int32_t *path = L.front0;                 // frontier lists are free now
    int v = k;
    for (; v != -1 && len < k + 1; v = L.pred[v]) path[len++] = v;
    // the predecessor chain is a tree rooted at s (labels only change on
    // strict improvement); anything else is an internal error
    const bool bad = v != -1 || len < 2 || path[len - 1] != s;
    if (bad) { S.status = -5; len = 1; }
    const int nedges = len - 1;
    const int nmov = mode == 0 ? nedges : nedges - 1;
    // read every moved unit before any move
    for (int e = 0; e < nmov; ++e) {
      const int u = path[len - 1 - e];
      int v = path[len - 2 - e];
      if (v == k) v = s;
      L.mrow[e] = (int32_t)key_rank(L.W[(int64_t)u * k + v]);
      L.mfrom[e] = u;
      L.mto[e] = v;
    }
    for (int e = 0; e < nmov; ++e) {
      const int x = L.mrow[e], u = L.mfrom[e], v = L.mto[e];
      I.assign[x] = v;
      // swap-remove x from u's member list, append to v's
      const int p = I.slot[x];
      const int last = L.load[u] - 1;
      const int y = I.members[(int64_t)u * I.n + last];
      I.members[(int64_t)u * I.n + p] = y;
      I.slot[y] = p;
      L.load[u] = last;
      const int q = L.load[v];
      I.members[(int64_t)v * I.n + q] = x;
      I.slot[x] = q;
      L.load[v] = q + 1;
    }
    S.nmoves = nmov > 0 ? nmov : 0;
    if (!bad) {
      S.obj += D;
      S.stats[mode == 0 ? ST_CYCLES : ST_PATHS] += 1;
      S.stats[ST_MOVES] += nmov;
    }
  }
  __syncthreads();
  const int nmov = S.nmoves;
  for (int e = 0; e < nmov; ++e) rescan_center(I, L, S, L.mfrom[e]);
  if (mode == 1 && nmov > 0) insert_row(I, L, L.mrow[nmov - 1], L.mto[nmov - 1]);
  __syncthreads();
}

template <bool WLDS>
__global__ __launch_bounds__(NT) void solve_kernel(InstView I, int64_t r_begin, int64_t r_end) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ Scalars S;
  const int k = I.k, K1 = k + 1;
  const int tid = threadIdx.x;
  Lds L;
  unsigned char *p = lds;
  if (WLDS) { L.W = reinterpret_cast<uint64_t *>(p); p += (size_t)k * k * 8; }
  else L.W = I.W;
  L.red = reinterpret_cast<uint64_t *>(p); p += (size_t)K1 * 8;
  L.dist = reinterpret_cast<int64_t *>(p); p += (size_t)K1 * 8;
  L.pred = reinterpret_cast<int32_t *>(p); p += (size_t)K1 * 4;
  L.front0 = reinterpret_cast<int32_t *>(p); p += (size_t)K1 * 4;
  L.front1 = reinterpret_cast<int32_t *>(p); p += (size_t)K1 * 4;
  L.load = reinterpret_cast<int32_t *>(p); p += (size_t)k * 4;
  L.cap = reinterpret_cast<int32_t *>(p); p += (size_t)k * 4;
  L.pen = reinterpret_cast<int32_t *>(p); p += (size_t)k * 4;
  L.mrow = reinterpret_cast<int32_t *>(p); p += (size_t)K1 * 4;
  L.mfrom = reinterpret_cast<int32_t *>(p); p += (size_t)K1 * 4;
  L.mto = reinterpret_cast<int32_t *>(p);

  if (WLDS)
    for (int64_t i = tid; i < (int64_t)k * k; i += NT) L.W[i] = I.W[i];
  for (int i = tid; i < k; i += NT) { L.load[i] = I.load[i]; L.cap[i] = I.cap[i]; L.pen[i] = I.pen[i]; }
  if (tid == 0) {
    S.obj = I.scalars[SC_OBJECTIVE];
    S.status = (int32_t)I.scalars[SC_STATUS];
    for (int j = 0; j < SC_NSTATS; ++j) S.stats[j] = I.scalars[SC_STAT0 + j];
  }
  __syncthreads();
  const bool ok0 = S.status == 0;
  int64_t r = r_begin;
  if (ok0) {
    for (; r < r_end; ++r) {
      const int s = I.smin[r];
      const int32_t *row = I.cm + r * k;
      if (tid == 0) {
        const int ld = L.load[s];
        const int vac = ld < L.cap[s];
        S.vacant = vac;
        I.assign[r] = s;
        I.members[(int64_t)s * I.n + ld] = (int32_t)r;
        I.slot[r] = ld;
        L.load[s] = ld + 1;
        S.obj += (int64_t)row[s] + (vac ? 0 : L.pen[s]);
      }
      const int changed = insert_row(I, L, (int)r, s);   // contains a barrier
      if (changed) refine(I, L, S, s, 0);
      else if (tid == 0) S.stats[ST_CYC_SKIPPED] += 1;
      __syncthreads();
      if (S.status != 0) break;
      if (!S.vacant) refine(I, L, S, s, 1);
      __syncthreads();
      if (S.status != 0) break;
    }
  }
  __syncthreads();
  if (WLDS)
    for (int64_t i = tid; i < (int64_t)k * k; i += NT) I.W[i] = L.W[i];
  for (int i = tid; i < k; i += NT) I.load[i] = L.load[i];
  if (tid == 0) {
    I.scalars[SC_OBJECTIVE] = S.obj;
    I.scalars[SC_STATUS] = S.status;
    const int64_t done = (S.status == 0) ? r_end : r;   // r: iteration that failed
    I.scalars[SC_DONE] = ok0 ? done : I.scalars[SC_DONE];
    S.stats[ST_ITERS] = I.scalars[SC_DONE];
    for (int j = 0; j < SC_NSTATS; ++j) I.scalars[SC_STAT0 + j] = S.stats[j];
  }
}

size_t solve_lds_bytes(int k, bool wlds) {
  const size_t K1 = (size_t)k + 1;
  size_t b = K1 * 8 * 2 + K1 * 4 * 3 + (size_t)k * 4 * 3 + K1 * 4 * 3;
  if (wlds) b += (size_t)k * k * 8;
  return b;
}

}  // namespace

namespace {

__global__ void init_state_kernel(InstView I) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t0; i < I.n; i += stride) I.assign[i] = -1;
  for (int64_t i = t0; i < (int64_t)I.k * I.k; i += stride) I.W[i] = KEY_NONE;
  for (int64_t i = t0; i < I.k; i += stride) I.load[i] = 0;
  for (int64_t i = t0; i < SC_COUNT; i += stride) I.scalars[i] = 0;
}

// out[order[r]] = assign[r]: back from processing order to the caller's order
__global__ void unpermute_kernel(int64_t n, const int64_t *__restrict__ order,
                                 const int32_t *__restrict__ assign, int32_t *__restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) out[order[r]] = assign[r];
}

}  // namespace

hipError_t launch_init_state(const InstView &I, hipStream_t st) {
  init_state_kernel<<<1024, 256, 0, st>>>(I);
  return hipGetLastError();
}

hipError_t launch_unpermute(int64_t n, const int64_t *order, const int32_t *assign, int32_t *out,
                            hipStream_t st) {
  unpermute_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, order, assign, out);
  return hipGetLastError();
}

// W is kept in LDS when the whole per-instance LDS image fits next to the
// static scalars (160 KB per CU on gfx950, a margin left for the compiler).
constexpr size_t LDS_BUDGET = 150 * 1024;

hipError_t launch_solve(const InstView &I, int64_t r_begin, int64_t r_end, hipStream_t st) {
  if (r_end <= r_begin) return hipSuccess;
  const bool wlds = solve_lds_bytes(I.k, true) <= LDS_BUDGET;
  const size_t bytes = solve_lds_bytes(I.k, wlds);
  hipError_t e;
  if (wlds) {
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&solve_kernel<true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    solve_kernel<true><<<1, NT, bytes, st>>>(I, r_begin, r_end);
  } else {
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&solve_kernel<false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
    solve_kernel<false><<<1, NT, bytes, st>>>(I, r_begin, r_end);
  }
  return hipGetLastError();
}

}  // namespace lbdd
