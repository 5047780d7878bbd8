// solve.hip -- the ASRAL main loop (Algorithm 2) on one workgroup.
//
// Each iteration r (row r of the permuted cost matrix is the r-th unit of the
// MinDistance order):
//   allot     the unit goes to its most suitable center s; the objective grows
//             by CM + (s full ? the penalty of its next unit beyond
//             capacity : 0); its k-1 transfer keys are
//             min-inserted into row s of the best-transfer table W.
//   cycle     Negative Cycle Refinement (Algorithm 1) with anchor s, on the
//             NCyc split graph built on the fly from W.  Skipped exactly when
//             the insert left row s of W unchanged: W is then the table of the
//             previous allotment, which has no negative cycle (Lemmas 1-2),
//             so no negative s_out -> s_in path exists.
//   path      when s was full: Negative Path Refinement (Appendix A) on the
//             NPath split graph (edges into s_in are penalty differences).
//   apply     the units on the chosen path move.  W is the head of a bounded
//             best-transfer list per ordered center pair (the BestTransHeap of
//             the paper, truncated to its BEST_M smallest keys): leaving and
//             joining units update the lists, and a list that runs empty while
//             not holding every unit of its center is refilled by a column
//             scan of the center's members in the cost matrix.
//
// The searches give the labels of synchronous Bellman-Ford rounds (shortest
// distance, then fewest edges, then smallest predecessor), packed so that one
// unsigned minimum orders them; that least fixpoint does not depend on the
// order of relaxations.  They run as frontier rounds, as rounds pruned by
// node potentials kept feasible across searches (repaired where moves break
// them), as windowed rounds in the order of (reduced distance, edges), or in
// Dijkstra order bounded to the centers that can still lower s_in; a
// measured cost model picks between rounds and Dijkstra order.  Path
// searches run on sink potentials (the cost of placing one more unit from
// each center).
//
// Strict-LBDD (Appendix B, Algorithm 4) runs the same loop: the unit goes to
// the cheapest center that still has free capacity, only Negative Cycle
// Refinement follows, and W[u][v] also holds the zero-cost dummy transfer
// (DUMMY_KEY) while u has free capacity, so the searches see the dummy units
// without knowing of them; applying a dummy transfer moves no unit.
//
// One workgroup of 1024 threads owns the instance.  W lives in LDS when it
// fits (k <= 135) and in global memory (L2-resident) otherwise.
#include "lbdd_dev.hpp"

namespace lbdd {

namespace {

constexpr int NT = SOLVE_THREADS;

__device__ inline uint64_t umin(uint64_t a, uint64_t b) { return b < a ? b : a; }
__device__ inline int64_t now() { return (int64_t)wall_clock64(); }

// number of set bits of mask in lanes below this one
__device__ inline int lanes_below(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Minimum over the 64 lanes of a wavefront (all lanes active), in every
// lane: within rows of 16 lanes by DPP (swap neighbours, swap pairs, mirror
// the half-row, mirror the row), then across rows by swapping odd with even
// rows and the upper with the lower half.  A swap hands each lane either its
// own value or its partner's in one of its two results, so taking the minimum
// of both is right whichever it is.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_min_step(uint32_t x) {
  const uint32_t y = (uint32_t)__builtin_amdgcn_mov_dpp((int)x, CTRL, 0xf, 0xf, true);
  return y < x ? y : x;
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
  x = dpp_min_step<0xb1>(x);     // quad_perm [1,0,3,2]
  x = dpp_min_step<0x4e>(x);     // quad_perm [2,3,0,1]
  x = dpp_min_step<0x141>(x);    // row_half_mirror
  x = dpp_min_step<0x140>(x);    // row_mirror
  const auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);
  x = min(x, min((uint32_t)p[0], (uint32_t)p[1]));
  const auto q = __builtin_amdgcn_permlane32_swap(x, x, false, false);
  x = min(x, min((uint32_t)q[0], (uint32_t)q[1]));
  return x;
}
// 64-bit minimum as two 32-bit ones: high words, then low words of the lanes
// holding the smallest high word.  The result is the same in every lane.
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_min_u32((uint32_t)(x >> 32)));
  const uint32_t lo = wave_min_u32((uint32_t)(x >> 32) == hi ? (uint32_t)x : 0xffffffffu);
  return (uint64_t)hi << 32 | (uint32_t)__builtin_amdgcn_readfirstlane((int)lo);
}

struct Lds {
  uint64_t *W;      // [k][k] (LDS copy or the global table)
  uint32_t *wh;     // global high words of W while W is global, else null
  uint32_t *wt;     // global high words of W transposed (kept while W is global)
  uint64_t *red;    // [k+1] per-target minimum
  int64_t *dist;    // [k+1]
  int32_t *pred;    // [k+1]
  int32_t *hop;     // [k+1] round in which the label last changed (0 for s)
  int32_t *front0;  // [k+1] frontier lists (double-buffered)
  int32_t *front1;
  int64_t *pot;     // [k] node potentials (see refine)
  int64_t *pot2;    // [k] candidate potentials from the last search
  int64_t *potT;    // [k] sink potentials for path searches (see sink_potential)
  uint32_t *dirty;  // [ceil(k/32)] rows of W changed since potT was last checked
  int32_t *load;    // [k]
  int32_t *cap;     // [k]
  int32_t *pen;     // [k]
  int32_t *mrow;    // [k+1] moved rows of the applied path
  int32_t *mfrom;   // [k+1]
  int32_t *mto;     // [k+1]
  int32_t *trow;    // [k+1] columns to refill
  uint64_t *wmin;   // [NT/64][BEST_M] per-wavefront candidates of a refill (also
                    // per-wavefront minima of other reductions)
};

// W[u][w] = key (idx = u k + w) and, when W is global, its high word in the
// packed and in the transposed array (with W in LDS the searches read both
// from the LDS copy)
__device__ inline void set_w(const Lds &L, int k, int u, int w, int64_t idx, uint64_t key) {
  L.W[idx] = key;
  if (L.wh) {
    L.wh[idx] = (uint32_t)(key >> 32);
    L.wt[(int64_t)w * k + u] = (uint32_t)(key >> 32);
  }
}

struct Scalars {
  int64_t obj;
  int64_t stats[SC_NSTATS];
  int32_t status;
  int32_t nfront[3];   // frontier sizes, by round mod 3
  int32_t nmoves;
  int32_t nrefill;
  int32_t pot_ok;   // pot is feasible for the current W
  int32_t vacant;
  int32_t ratio;    // cost of a Bellman-Ford round in Dijkstra steps, x16, or
                    // SEARCH_RATIO_AUTO: measured (round_t / step_t)
  int32_t depth[2];    // running means, per search mode, of the rounds of
                       // Bellman-Ford searches and of the centers settled by
  int32_t settled[2];  // searches in Dijkstra order, x16
  int32_t round_t;  // running mean of the device ticks per Bellman-Ford round, x16
  int32_t step_t;   // running mean of the device ticks per Dijkstra step, x16
  int32_t nsearch;  // searches run (Bellman-Ford or Dijkstra order)
  uint64_t bound;   // pruned Bellman-Ford: biased bound term (see bellman_ford)
  uint64_t wlo[3];  // windowed rounds: smallest pending window key (see bellman_ford)
  int32_t nrep[3];  // windowed rounds: repeated relaxations in a round
  int64_t wdelta;   // windowed rounds: window width (adapted per window)
  int32_t sink_every;  // path searches per sink-potential computation (0: never)
  int32_t sink_age;    // path searches since the last one
  int32_t potT_ok;     // potT is feasible on every edge of W outside the dirty rows
  int32_t jflags[2];  // join_center's result, by iteration parity
};

}  // namespace

// Dynamic LDS of one workgroup solving an instance with k centers, with or
// without the k x k table in LDS.
__host__ __device__ size_t solve_lds_bytes(int k, bool wlds) {
  const size_t K1 = (size_t)k + 1;
  size_t b = K1 * 8 * 2 + K1 * 4 * 4 + 8 + (size_t)k * 8 * 3 + ((size_t)k + 31) / 32 * 4 + 8 +
             (size_t)k * 4 * 3 +
             K1 * 4 * 3 + K1 * 4 + 8 + (SOLVE_THREADS / 64) * BEST_M * 8;
  if (wlds) b += (size_t)k * k * 8;
  return b;
}

namespace {

// Minimum of a per-thread candidate over each target, combined in LDS.
__device__ inline void lds_min(uint64_t *p, uint64_t v) {
  if (v != KEY_NONE) atomicMin((unsigned long long *)p, (unsigned long long)v);
}

// ---- bounded best-transfer lists ----------------------------------------
// W[u][w] is the head of the list of (u, w) (BEST_M smallest keys of the
// units at u, see lbdd_dev.hpp).  Joining and leaving units update the lists;
// a list that runs empty while some unit of u is not in it ("unknown") is
// refilled by a column rescan over the members of u.  Lists are kept in
// registers while they are updated: no indexing by run-time values.

__device__ inline void list_load(const uint64_t *p, uint64_t (&a)[BEST_M]) {
  const ulonglong2 *q = reinterpret_cast<const ulonglong2 *>(p);
#pragma unroll
  for (int i = 0; i < BEST_M / 2; ++i) {
    const ulonglong2 t = q[i];
    a[2 * i] = t.x;
    a[2 * i + 1] = t.y;
  }
}
__device__ inline void list_store(uint64_t *p, const uint64_t (&a)[BEST_M]) {
  ulonglong2 *q = reinterpret_cast<ulonglong2 *>(p);
#pragma unroll
  for (int i = 0; i < BEST_M / 2; ++i) q[i] = make_ulonglong2(a[2 * i], a[2 * i + 1]);
}
// merge q into the sorted list a (the largest entry falls off the end)
__device__ inline void list_merge(uint64_t (&a)[BEST_M], uint64_t q) {
  uint64_t prev = a[0];
  a[0] = umin(a[0], q);
#pragma unroll
  for (int i = 1; i < BEST_M; ++i) {
    const uint64_t cur = a[i];
    const uint64_t hi = prev > q ? prev : q;     // max(q, old a[i-1])
    a[i] = umin(cur, hi);
    prev = cur;
  }
}

// Threshold below which a joining key touches the list: while every unit is
// held and there is room, always; otherwise only in front of the last held
// key (an unknown list takes nothing: threshold 0).
__device__ inline uint64_t list_threshold(const uint64_t (&a)[BEST_M], int c, bool all) {
  if (all) return KEY_NONE;                      // enters, or clears the all-held flag
  uint64_t t = 0;
#pragma unroll
  for (int i = 0; i < BEST_M; ++i) t = (i == c - 1) ? a[i] : t;
  return t;
}

// Unit x (row x) joins center v: its keys enter v's lists, row v of W follows.
// Returns (block-wide) bit 0: some W entry decreased; bit 1: a decreased entry
// breaks the node potentials.
// The key of unit x (row x) enters the list of (v, w); row v of W follows.
// Sets changed when W[v][w] decreased, breaks when that breaks the node
// potentials.
__device__ __forceinline__ void join_one(const InstView &I, const Lds &L, int x, int v, int w,
                                         int &changed, int &breaks) {
  const int k = I.k;
  const int32_t *rx = I.cm + (int64_t)x * k;
  const int32_t base = rx[v];
  const int32_t delta = rx[w] - base;
  const uint64_t q = pack_key(delta, (uint32_t)x);
  const int64_t idx = (int64_t)v * k + w;
  // with every unit held q always enters; otherwise only in front of a held
  // key (beyond the last held key an unheld unit may be smaller)
  if (!(q < I.thr[idx])) return;
  const uint8_t meta = I.meta[idx];
  const int c = meta & 15;
  const bool all = meta & META_ALL;
  uint64_t a[BEST_M];
  list_load(I.best + idx * BEST_M, a);
  list_merge(a, q);
  list_store(I.best + idx * BEST_M, a);
  const bool full = c == BEST_M;
  const int c2 = full ? BEST_M : c + 1;
  const bool all2 = all && !full;
  I.meta[idx] = (uint8_t)(c2 | (all2 ? META_ALL : 0));
  I.thr[idx] = list_threshold(a, c2, all2);
  if (a[0] < L.W[idx]) {
    set_w(L, k, v, w, idx, a[0]);
    changed = 1;
    breaks |= L.pot[v] + delta < L.pot[w];
  }
}

// Unit x joins center v.  Returns (workgroup-wide) bit 0: some W entry
// decreased; bit 1: a decreased entry breaks the node potentials.  The two
// bits meet in one LDS word (one barrier); iterations alternate between two
// words so the other one can be cleared without another barrier.
__device__ __forceinline__ int join_center(const InstView &I, const Lds &L, Scalars &S, int x, int v,
                                           int parity) {
  const int k = I.k;
  int changed = 0, breaks = 0;
  for (int w = threadIdx.x; w < k; w += NT)
    if (w != v) join_one(I, L, x, v, w, changed, breaks);
  const uint64_t mc = __ballot(changed), mb = __ballot(breaks);
  if ((threadIdx.x & 63) == 0 && (mc | mb)) atomicOr(&S.jflags[parity], (mc ? 1 : 0) | (mb ? 2 : 0));
  __syncthreads();
  const int f = S.jflags[parity];
  if (threadIdx.x == 0) S.jflags[parity ^ 1] = 0;
  return f;
}

// The key of unit x (row x) leaves the list of (u, w).  A list that becomes
// unknown is left for refill_center.
__device__ __forceinline__ void leave_one(const InstView &I, const Lds &L, int x, int u, int w) {
  const int k = I.k;
  const int32_t *rx = I.cm + (int64_t)x * k;
  const int32_t base = rx[u];
  const uint64_t q = pack_key(rx[w] - base, (uint32_t)x);
  const int64_t idx = (int64_t)u * k + w;
  const uint8_t meta = I.meta[idx];
  const int c = meta & 15;
  uint64_t a[BEST_M];
  list_load(I.best + idx * BEST_M, a);
  bool held = false;
#pragma unroll
  for (int i = 0; i < BEST_M; ++i) held |= a[i] == q;
  if (!held) return;                           // not among the c smallest: lists unchanged
#pragma unroll
  for (int i = 0; i < BEST_M - 1; ++i) a[i] = a[i] < q ? a[i] : a[i + 1];
  a[BEST_M - 1] = KEY_NONE;
  list_store(I.best + idx * BEST_M, a);
  I.meta[idx] = (uint8_t)((c - 1) | (meta & META_ALL));
  I.thr[idx] = list_threshold(a, c - 1, meta & META_ALL);
  set_w(L, k, u, w, idx, a[0]);                // stale if unknown; refill sets it
}

// The moved units of an applied refinement leave their old centers' lists,
// then join their new centers' lists.  The old centers of a refinement are
// distinct, and so are the new ones, so each pass updates disjoint lists and
// covers all moves at once (threads over (move, target) pairs).
__device__ __forceinline__ void move_lists(const InstView &I, const Lds &L, int nmov) {
  const int k = I.k;
  const int total = nmov * k;
  for (int t = threadIdx.x; t < total; t += NT) {
    const int e = t / k, w = t - e * k;
    if (w != L.mfrom[e]) leave_one(I, L, L.mrow[e], L.mfrom[e], w);
  }
  __syncthreads();
  int changed = 0, breaks = 0;                   // the potentials are rechecked afterwards
  for (int t = threadIdx.x; t < total; t += NT) {
    const int e = t / k, w = t - e * k;
    if (w != L.mto[e]) join_one(I, L, L.mrow[e], L.mto[e], w, changed, breaks);
  }
  __syncthreads();
}

// Refill the list of (u, w) from the members of u: the BEST_M smallest keys
// (definition of Gamma).  Every thread keeps a sorted top list of its member
// rows; each wavefront takes its BEST_M smallest by BEST_M wavefront minima
// (the one lane holding a minimum pops it: keys are unique), and wavefront 0
// takes the BEST_M smallest of those NT / 64 * BEST_M candidates the same
// way, two per lane.  Two barriers in all.  The wavefront minima use DPP and
// lane swaps that read every lane: they run with all 64 lanes active (a
// disabled lane would read as 0, the smallest key).
__device__ __forceinline__ void refill_column(const InstView &I, const Lds &L, Scalars &S, int u, int w) {
  const int k = I.k;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int m = L.load[u];
  const int32_t *mem = I.members + (int64_t)u * I.n;
  uint64_t b[BEST_M];
#pragma unroll
  for (int i = 0; i < BEST_M; ++i) b[i] = KEY_NONE;
  int i = tid;
  for (; i + NT < m; i += 2 * NT) {              // two member rows in flight
    const int32_t y0 = mem[i], y1 = mem[i + NT];
    const int32_t *r0 = I.cm + (int64_t)y0 * k, *r1 = I.cm + (int64_t)y1 * k;
    const int32_t d0 = r0[w] - r0[u], d1 = r1[w] - r1[u];
    list_merge(b, pack_key(d0, (uint32_t)y0));
    list_merge(b, pack_key(d1, (uint32_t)y1));
  }
  if (i < m) {
    const int32_t y = mem[i];
    const int32_t *ry = I.cm + (int64_t)y * k;
    list_merge(b, pack_key(ry[w] - ry[u], (uint32_t)y));
  }
  // this wavefront's BEST_M smallest: lane r keeps the r-th
  uint64_t mine = KEY_NONE;
#pragma unroll
  for (int r = 0; r < BEST_M; ++r) {
    const uint64_t g = wave_min_u64(b[0]);
    mine = lane == r ? g : mine;
    if (g != KEY_NONE && b[0] == g) {
#pragma unroll
      for (int j = 0; j < BEST_M - 1; ++j) b[j] = b[j + 1];
      b[BEST_M - 1] = KEY_NONE;
    }
  }
  if (lane < BEST_M) L.wmin[wave * BEST_M + lane] = mine;
  __syncthreads();
  if (wave == 0) {
    // NT / 64 * BEST_M = 128 candidates, two per lane (sorted pair)
    static_assert(NT / 64 * BEST_M == 128, "two candidates per lane of one wavefront");
    const uint64_t x0 = L.wmin[lane], x1 = L.wmin[lane + 64];
    uint64_t c0 = umin(x0, x1), c1 = x0 < x1 ? x1 : x0;
    uint64_t out[BEST_M];
#pragma unroll
    for (int r = 0; r < BEST_M; ++r) {
      const uint64_t g = wave_min_u64(c0);
      out[r] = g;
      if (g != KEY_NONE && c0 == g) {
        c0 = c1;
        c1 = KEY_NONE;
      }
    }
    if (tid == 0) {
      const int64_t idx = (int64_t)u * k + w;
      list_store(I.best + idx * BEST_M, out);
      int c = 0;
#pragma unroll
      for (int j = 0; j < BEST_M; ++j) c += out[j] != KEY_NONE;
      I.meta[idx] = (uint8_t)(c | (m <= BEST_M ? META_ALL : 0));
      I.thr[idx] = list_threshold(out, c, m <= BEST_M);
      set_w(L, k, u, w, idx, out[0]);
      S.stats[ST_ROWS_SCANNED] += m;
      S.stats[ST_REFILLS] += 1;
    }
  }
  __syncthreads();
}

// Refill every unknown list of center u (after its unit left and the moves of
// the refinement have all been applied).
__device__ __forceinline__ void refill_center(const InstView &I, const Lds &L, Scalars &S, int u) {
  const int k = I.k;
  if (threadIdx.x == 0) S.nrefill = 0;
  __syncthreads();
  for (int w = threadIdx.x; w < k; w += NT) {
    if (w == u) continue;
    const uint8_t meta = I.meta[(int64_t)u * k + w];
    if ((meta & 15) == 0 && !(meta & META_ALL)) L.trow[atomicAdd(&S.nrefill, 1)] = w;
  }
  __syncthreads();
  const int nr = S.nrefill;
  for (int j = 0; j < nr; ++j) refill_column(I, L, S, u, L.trow[j]);
}

// Refill every unknown list of the old centers of an applied refinement's
// moves: one pass finds them all (most moves leave none), then each is
// refilled.  Refills read only the final member lists, so their order does
// not matter.  More unknown lists than slots (k + 1) falls back to one center
// at a time.
__device__ __forceinline__ void refill_moved(const InstView &I, const Lds &L, Scalars &S, int nmov) {
  const int k = I.k;
  if (threadIdx.x == 0) S.nrefill = 0;
  __syncthreads();
  const int total = nmov * k;
  for (int t = threadIdx.x; t < total; t += NT) {
    const int e = t / k, w = t - e * k;
    const int u = L.mfrom[e];
    if (w == u) continue;
    const uint8_t meta = I.meta[(int64_t)u * k + w];
    if ((meta & 15) == 0 && !(meta & META_ALL)) {
      const int j = atomicAdd(&S.nrefill, 1);
      if (j <= k) L.trow[j] = e << 16 | w;
    }
  }
  __syncthreads();
  const int nr = S.nrefill;
  if (nr <= k + 1) {
    for (int j = 0; j < nr; ++j) {
      const int p = L.trow[j];
      refill_column(I, L, S, L.mfrom[p >> 16], p & 0xffff);
    }
  } else {
    for (int e = 0; e < nmov; ++e) refill_center(I, L, S, L.mfrom[e]);
  }
}

// Potentials certify that W has no negative cycle, which lets searches be
// skipped or run in Dijkstra order.  A search leaves candidate potentials in
// pot2 (Bellman-Ford: the labels, i.e. distances from s; Dijkstra order: the
// labels of the settled centers and shifted old potentials for the others,
// see dijkstra_bounded), feasible (pot2[v] <= pot2[u] + W[u][v]) on every
// edge of the searched table except possibly those out of s and into s.
// An applied refinement then changed only the rows of the centers it moved
// units between.  So checking those rows, row s and column s decides
// feasibility on the whole current table.  nmov = 0 after a search that
// applied nothing.
//
// Where some checked edges fail, pot2 is repaired rather than dropped: W has
// no negative cycle (Lemmas 1 and 2), so the shortest distances lab(v) <= 0
// from a virtual source joined to every center by a 0-weight edge, on the
// reduced weights W[u][v] + pot2[u] - pot2[v], exist, and pot2 + lab is
// feasible on every edge.  Only a failed edge has a negative reduced weight,
// so with every label starting at 0 only the tails of failed edges can lower
// a label in the first round; later rounds relax out of the centers whose
// label dropped (rounds as in bellman_ford, on plain int64 labels).  The
// result is shifted so that the potential of s is 0: every center with units
// has edges to and from s, so its potential stays within 2^30 of 0.
constexpr int64_t REP_BIAS = 1ll << 62;   // repair labels lie in (-2^62, 0]
// Floor of a candidate potential.  Only a center without out-edges (no
// units) can sink this low (one with an edge into s stays within 2^30 of it); raising such a center's potential keeps its in-edges feasible, whose
// sources have out-edges and so potentials far above the floor.
constexpr int64_t POT_FLOOR = -(1ll << 42);
// Repair rounds on the potential P from the tails of failed edges already in
// the frontier list 1 (S.nfront[1] of them, round stamp 1, every label at
// REP_BIAS, i.e. 0): on convergence P += lab, shifted so that P[norm] is
// unchanged plus its own label when norm >= 0.  Returns false without
// convergence (then P is unchanged).
template <bool WLDS>
__device__ __forceinline__ bool repair_rounds(const InstView &I, const Lds &L, Scalars &S, int64_t *P,
                                              int norm) {
  const int k = I.k;
  const int tid = threadIdx.x;
  constexpr int WS = WLDS ? 2 : 1;
  const uint32_t *Whi = WLDS ? reinterpret_cast<const uint32_t *>(L.W) + 1 : L.wh;
  uint64_t *lab = L.red;
  int32_t *stamp = L.trow;
  bool conv = false;
  int64_t rounds = 0;
  for (int t = 1; t <= k + 1; ++t) {
    // round t relaxes out of the frontier of size nfront[t % 3] in list t & 1
    // (see bellman_ford)
    const int nf = S.nfront[t % 3];
    const int32_t *F = (t & 1) ? L.front1 : L.front0;
    int32_t *Fn = (t & 1) ? L.front0 : L.front1;
    int32_t *cnt_next = &S.nfront[(t + 1) % 3];
    if (tid == 0) S.nfront[(t + 2) % 3] = 0;
    for (int64_t x = tid; x < (int64_t)nf * k; x += NT) {
      const int j = (int)(x / k), v = (int)(x - (int64_t)j * k);
      const int u = F[j];
      if (u == v) continue;
      const uint32_t hi = Whi[WS * ((int64_t)u * k + v)];
      if (hi == 0xffffffffu) continue;
      const int64_t cand = (int64_t)(lab[u] - (uint64_t)REP_BIAS) + (int64_t)(int32_t)(hi ^ 0x80000000u) +
                           P[u] - P[v];
      if (cand >= 0) continue;
      const uint64_t c = (uint64_t)(cand + REP_BIAS);
      if (c < atomicMin((unsigned long long *)&lab[v], (unsigned long long)c) &&
          atomicExch(&stamp[v], t + 1) != t + 1)
        Fn[atomicAdd(cnt_next, 1)] = v;
    }
    __syncthreads();
    ++rounds;
    if (*cnt_next == 0) { conv = true; break; }
  }
  if (conv) {
    const int64_t shift = norm >= 0 ? (int64_t)(lab[norm] - (uint64_t)REP_BIAS) : 0;
    for (int u = tid; u < k; u += NT) {
      const int64_t p = P[u] + (int64_t)(lab[u] - (uint64_t)REP_BIAS) - shift;
      P[u] = p < POT_FLOOR ? POT_FLOOR : p;
    }
  }
  if (tid == 0) {
    S.stats[ST_POT_REPAIRS] += 1;
    S.stats[ST_REPAIR_ROUNDS] += rounds;
  }
  __syncthreads();
  return conv;
}

template <bool WLDS>
__device__ __forceinline__ void take_potential(const InstView &I, const Lds &L, Scalars &S, int s,
                                               int nmov) {
  const int k = I.k;
  const int tid = threadIdx.x;
  // high word of W[i]: Whi[WS * i]
  constexpr int WS = WLDS ? 2 : 1;
  const uint32_t *Whi = WLDS ? reinterpret_cast<const uint32_t *>(L.W) + 1 : L.wh;
  // repair labels (biased) and round stamps; the search labels (dist, hop,
  // pred) stay intact for a path search derived from them
  uint64_t *lab = L.red;
  int32_t *stamp = L.trow;                       // last round whose frontier took the center
  const int64_t t_start = tid == 0 ? now() : 0;
  int unknown = 0;
  for (int u = tid; u < k; u += NT) {
    unknown |= L.pot2[u] == DIST_NONE;
    lab[u] = (uint64_t)REP_BIAS;
    stamp[u] = 0;
  }
  if (tid == 0) { S.nfront[0] = S.nfront[1] = S.nfront[2] = 0; }
  __syncthreads();
  // the check; the tails of failed edges form the first frontier (list 1)
  const int nrows = 2 * nmov + 2;                // from/to of every move, row s, column s
  if (!unknown)
    for (int64_t t = tid; t < (int64_t)nrows * k; t += NT) {
      const int j = (int)(t / k), w = (int)(t - (int64_t)j * k);
      int u, v;
      if (j < 2 * nmov) { u = (j & 1) ? L.mto[j >> 1] : L.mfrom[j >> 1]; v = w; }
      else if (j == 2 * nmov) { u = s; v = w; }
      else { u = w; v = s; }
      if (u == v) continue;
      const uint32_t hi = Whi[WS * ((int64_t)u * k + v)];
      if (hi == 0xffffffffu) continue;
      const int64_t d = (int64_t)(int32_t)(hi ^ 0x80000000u);
      if (L.pot2[u] + d < L.pot2[v] && atomicExch(&stamp[u], 1) != 1)
        L.front1[atomicAdd(&S.nfront[1], 1)] = u;
    }
  unknown = __syncthreads_or(unknown);
  bool ok = !unknown;
  if (ok && S.nfront[1] > 0) ok = repair_rounds<WLDS>(I, L, S, L.pot2, s);
  if (ok)
    for (int u = tid; u < k; u += NT) L.pot[u] = L.pot2[u];
  if (tid == 0) {
    S.pot_ok = ok;
    if (ok && nmov > 0) S.stats[ST_POT_KEPT] += 1;
    S.stats[ST_T_POT] += now() - t_start;
  }
  __syncthreads();
}

// The sink potentials potT before a path search: the rows of W that changed
// since potT was last checked (joins, moves) are checked, the tails of their
// failed edges start the repair rounds, and the rows are clean again.  An
// unconverged repair leaves potT invalid (it is computed afresh).
template <bool WLDS>
__device__ __forceinline__ void refresh_sink(const InstView &I, const Lds &L, Scalars &S) {
  const int k = I.k;
  const int tid = threadIdx.x;
  constexpr int WS = WLDS ? 2 : 1;
  const uint32_t *Whi = WLDS ? reinterpret_cast<const uint32_t *>(L.W) + 1 : L.wh;
  uint64_t *lab = L.red;
  int32_t *stamp = L.trow;
  const int64_t t_start = tid == 0 ? now() : 0;
  for (int u = tid; u < k; u += NT) {
    lab[u] = (uint64_t)REP_BIAS;
    stamp[u] = 0;
  }
  if (tid == 0) { S.nfront[0] = S.nfront[1] = S.nfront[2] = 0; S.nrefill = 0; }
  __syncthreads();
  for (int u = tid; u < k; u += NT)
    if ((L.dirty[u >> 5] >> (u & 31)) & 1u) L.mrow[atomicAdd(&S.nrefill, 1)] = u;
  __syncthreads();
  const int nd = S.nrefill;
  for (int64_t t = tid; t < (int64_t)nd * k; t += NT) {
    const int j = (int)(t / k), v = (int)(t - (int64_t)j * k);
    const int u = L.mrow[j];
    if (u == v) continue;
    const uint32_t hi = Whi[WS * ((int64_t)u * k + v)];
    if (hi == 0xffffffffu) continue;
    if (L.potT[u] + (int64_t)(int32_t)(hi ^ 0x80000000u) < L.potT[v] && atomicExch(&stamp[u], 1) != 1)
      L.front1[atomicAdd(&S.nfront[1], 1)] = u;
  }
  __syncthreads();
  const bool ok = S.nfront[1] == 0 || repair_rounds<WLDS>(I, L, S, L.potT, -1);
  for (int i = tid; i < (k + 31) / 32; i += NT) L.dirty[i] = 0;
  if (tid == 0) {
    if (!ok) S.potT_ok = 0;
    S.stats[ST_T_POT] += now() - t_start;
  }
  __syncthreads();
}

// Strict-LBDD: W[u][v] from the head of the list of (u, v) and the dummy
// transfer while u has free capacity (the loads in LDS are current).
__device__ __forceinline__ uint64_t strict_entry(const InstView &I, const Lds &L, int u, int v) {
  if (u == v) return KEY_NONE;
  const uint64_t head = I.best[((int64_t)u * I.k + v) * BEST_M];
  return L.load[u] < L.cap[u] ? umin(head, DUMMY_KEY) : head;
}

// Penalty of the j-th unit (j >= 1) beyond the capacity of center s: the
// constant pen[s], or the j-th value of the center's table (its last value
// for every later unit).
__device__ inline int64_t penalty_at(const InstView &I, const Lds &L, int s, int64_t j) {
  if (!I.pval) return L.pen[s];
  const int64_t b = I.poff[s], len = I.poff[s + 1] - b;
  return I.pval[b + (j < len ? j : len) - 1];
}

// Sink potentials: the node potentials -sigma, sigma(v) the cheapest way to
// give one more unit to some center starting from v: sigma(v) = min(q(v),
// min over w of W[v][w] + sigma(w)), q(v) what one more unit at v pays (0
// while v has room).  These are the shortest distances to a sink that every
// center joins by an edge of weight q(v); W has no negative cycle (Lemmas 1
// and 2), so they exist, and -sigma is feasible on every edge of W.  A path
// search (Appendix A) in Dijkstra order on them settles little beyond the
// centers of its cheapest paths: its bound term P(u) = q(u) - sigma(u) +
// sigma(s) - q(s) takes its smallest value, sigma(s) - q(s), on the center
// that ends a cheapest path, which is also the best candidate.  Computed as
// rounds from the sink over the reversed edges (the transposed high words),
// every center in the first frontier; after a round with no change the
// potentials replace potT (every row clean).  Without convergence (a
// negative cycle) nothing changes and the status records the failed
// invariant.
template <bool WLDS>
__device__ __forceinline__ void sink_potential(const InstView &I, const Lds &L, Scalars &S) {
  const int k = I.k;
  const int tid = threadIdx.x;
  const int64_t t_start = tid == 0 ? now() : 0;
  uint64_t *lab = L.red;                         // sigma + DIST_BIAS
  int32_t *stamp = L.trow;                       // last round whose frontier took the center
  for (int v = tid; v < k; v += NT) {
    const int64_t q = L.load[v] >= L.cap[v] ? penalty_at(I, L, v, (int64_t)L.load[v] - L.cap[v] + 1) : 0;
    lab[v] = (uint64_t)(q + DIST_BIAS);
    stamp[v] = 1;
    L.front1[v] = v;
  }
  if (tid == 0) { S.nfront[0] = 0; S.nfront[1] = k; S.nfront[2] = 0; }
  __syncthreads();
  bool conv = false;
  for (int t = 1; t <= k + 1; ++t) {
    const int nf = S.nfront[t % 3];
    const int32_t *F = (t & 1) ? L.front1 : L.front0;
    int32_t *Fn = (t & 1) ? L.front0 : L.front1;
    int32_t *cnt_next = &S.nfront[(t + 1) % 3];
    if (tid == 0) S.nfront[(t + 2) % 3] = 0;
    for (int64_t x = tid; x < (int64_t)nf * k; x += NT) {
      const int j = (int)(x / k), v = (int)(x - (int64_t)j * k);
      const int w = F[j];
      if (v == w) continue;
      const uint32_t hi = WLDS ? (uint32_t)(L.W[(int64_t)v * k + w] >> 32)
                               : L.wt[(int64_t)w * k + v];   // W[v][w]
      if (hi == 0xffffffffu) continue;
      const uint64_t c = lab[w] + (uint64_t)(int64_t)(int32_t)(hi ^ 0x80000000u);
      if (c < atomicMin((unsigned long long *)&lab[v], (unsigned long long)c) &&
          atomicExch(&stamp[v], t + 1) != t + 1)
        Fn[atomicAdd(cnt_next, 1)] = v;
    }
    __syncthreads();
    if (*cnt_next == 0) { conv = true; break; }
  }
  if (conv)
    for (int v = tid; v < k; v += NT) L.potT[v] = DIST_BIAS - (int64_t)lab[v];
  for (int i = tid; i < (k + 31) / 32; i += NT) L.dirty[i] = 0;
  if (tid == 0) {
    S.potT_ok = conv;
    if (!conv) S.status = -5;                    // LBDD_E_INTERNAL: negative cycle
    S.stats[ST_SINK] += 1;
    S.stats[ST_T_SINK] += now() - t_start;
  }
  __syncthreads();
}

// Label of a center during a search, packed so that one unsigned min orders
// by (distance, edges, predecessor): ((dist + 2^41) << 22) | (edges << 11) |
// pred.  Simple paths have at most k - 1 <= 2047 edges of |delta| < 2^30, so
// |dist| < 2^41 and both small fields fit (a candidate one edge longer than
// a simple path through all centers can carry into the distance field, which
// only makes it larger: it is a cyclic walk and never improves a label).
constexpr int64_t LAB_BIAS = 1ll << 41;
__device__ inline uint64_t lab_pack(int64_t dist, int32_t edges, int32_t pred) {
  return (uint64_t)(dist + LAB_BIAS) << 22 | (uint64_t)edges << 11 | (uint32_t)pred;
}

// Bellman-Ford from node s over the centers of the split graph; leaves the
// center labels dist/pred/hop in LDS (s_in follows with sin_from_labels: it
// has no out-edges, so it never changes a center's label).
// The rounds relax edges out of the centers whose label changed, reading the
// sources' current labels (not those of the previous round) and lowering the
// targets' packed labels with LDS atomic minima.  The packed order is the tie
// rule of synchronous rounds: the label a center ends with is the smallest
// (distance, edges), i.e. its shortest distance and the round in which
// synchronous rounds fix it, and its predecessor the smallest center reaching
// it so; with no negative cycle this least fixpoint does not depend on the
// order of the relaxations, and it is reached in at most as many rounds as
// synchronous rounds need, since every label is at least as good after each
// round.  One barrier per round: a thread whose atomic minimum lowers a
// label appends the center to the next frontier, unless the center's round
// stamp (taken by atomic exchange) shows that another thread already has.
// Only the key's high word of W (delta + 2^31, all ones = no edge) is read.
// Returns false (and sets the status) on a change in round k+1.
//
// Pruned (prune: the node potentials pot are feasible, on every edge except
// those out of s in cycle mode): a center whose label's reduced value
// r(v) = dist(v) + pot[s] - pot[v] is not below a bound Db cannot lead to a
// negative s_in label, so it enters no frontier (its label may still drop).
// Cycle mode: Db = 0 (an edge into s is feasible, so a cycle through v costs
// at least r(v)).  Path mode: Db = -Pmin, Pmin the smallest pot[u] +
// w(u, s_in) - pot[s] (s_in's candidate through u is at least r(u) + Pmin).
// Reduced weights beyond the first hop are non-negative, so every center
// that matters (r < Db) has all of a shortest path's centers below Db too,
// and gets its exact label and predecessor; the others get DIST_NONE.  The
// candidate potentials pot2 follow the rule of the bounded Dijkstra search
// with D = max(Db, 0).
template <bool WLDS>
__device__ __forceinline__ bool bellman_ford(const InstView &I, const Lds &L, Scalars &S, int s, int mode,
                                             bool prune) {
  const int k = I.k;
  const int tid = threadIdx.x;
  const int64_t t_start = tid == 0 ? now() : 0;
  // high word of W[i]: Whi[WS * i] (in the LDS copy of W, or the packed
  // global array next to the global W)
  constexpr int WS = WLDS ? 2 : 1;
  const uint32_t *Whi = WLDS ? reinterpret_cast<const uint32_t *>(L.W) + 1 : L.wh;
  uint64_t *lab = L.red;                      // packed labels
  int32_t *stamp = L.hop;                     // last round whose frontier took the center
  const int64_t pot_s = prune ? L.pot[s] : 0;
  for (int v = tid; v <= k; v += NT) {
    lab[v] = (v == s) ? lab_pack(0, 0, 0) : KEY_NONE;
    stamp[v] = 0;
  }
  if (tid == 0) {
    S.nfront[0] = 0;
    S.nfront[1] = 1;
    S.nfront[2] = 0;
    L.front1[0] = s;
    S.bound = prune && mode == 1 ? KEY_NONE : (uint64_t)DIST_BIAS;   // Db = 0 in cycle mode
  }
  __syncthreads();
  if (prune && mode == 1) {
    const int64_t q_anchor = penalty_at(I, L, s, L.load[s] > L.cap[s] ? (int64_t)L.load[s] - L.cap[s] : 1);
    for (int u = tid; u < k; u += NT) {
      if (u == s) continue;
      const int64_t w =
          (L.load[u] >= L.cap[u] ? penalty_at(I, L, u, (int64_t)L.load[u] - L.cap[u] + 1) : 0) - q_anchor;
      // -(pot[u] + w - pot[s]), biased: the largest term gives Db = -Pmin
      const uint64_t b = (uint64_t)(DIST_BIAS - (L.pot[u] + w - pot_s));
      atomicMin((unsigned long long *)&S.bound, (unsigned long long)(~b));
    }
    __syncthreads();
  }
  // Db (prune only): a center enters a frontier only while r(v) < Db
  const int64_t Db = !prune ? 0 : mode == 0 ? 0
                   : S.bound == KEY_NONE ? -DIST_BIAS        // k = 1: no center to reach
                   : (int64_t)(~S.bound) - DIST_BIAS;
  // target v of this thread and its share g of the frontier (k <= NT: every
  // target gets G = NT / k threads)
  const int G = k <= NT ? NT / k : 1;
  const int tv = k <= NT ? tid % k : tid;
  const int tg = k <= NT ? tid / k : 0;
  int64_t rounds = 0, relax = 0;
  bool conv = false;
  if (!WLDS && prune) {
    // Windowed rounds (the table in global memory, potentials feasible).
    // The centers whose label dropped since they were last relaxed are
    // pending.  A center's window key orders its label by reduced distance,
    // then edges: key = ((r(v) + 2^46) << 11) | edges.  Each window starts at
    // the smallest pending key lo and relaxes, round after round, the
    // pending centers with keys below lo + width until none is left there.
    // A pending center with the smallest key is final: a candidate through
    // any other pending center u costs at least r(u) (reduced weights beyond
    // the first hop are non-negative) with more edges than u, so its key is
    // larger, predecessor ties included.  With width 1 every round relaxes
    // only final labels, so each center is relaxed once; wider windows take
    // fewer rounds but may relax a center again.  The width halves after a
    // window that relaxed a center twice and doubles after a run of windows
    // of one small round.  s goes first, alone (the edges out of s may be
    // negative in reduced terms); the search ends when no pending center is
    // below the bound Db.  Any order reaches the same least fixpoint of the
    // labels.
    // Each round is one pass over the pending flags (the frontier, and the
    // smallest key of the pending centers left out) and one of relaxations
    // (which adds the keys of the centers they make pending), so the next
    // window's start is known when the round ends.
    int32_t *pend = L.mrow;                     // [k] 1: pending
    int32_t *seen = L.hop;                      // [k] window of the center's last relaxation
    for (int v = tid; v < k; v += NT) {
      pend[v] = v == s;
      seen[v] = -1;
    }
    if (tid == 0) {
      for (int c = 0; c < 3; ++c) {
        S.nfront[c] = 0;
        S.nrep[c] = 0;
        S.wlo[c] = KEY_NONE;
      }
    }
    __syncthreads();
    auto wkey = [&](uint64_t l, int v) -> uint64_t {
      const int64_t r = (int64_t)(l >> 22) - LAB_BIAS + pot_s - L.pot[v];
      return (uint64_t)(r + DIST_BIAS) << 11 | ((l >> 11) & 0x7ff);
    };
    const uint64_t key_db = (uint64_t)(Db + DIST_BIAS) << 11;   // keys from here on: r >= Db
    const int64_t cap_rounds = 2 * (int64_t)k + 64;   // a safety net: every round relaxes the
                                                      // smallest pending key, which is final
    int64_t width = S.wdelta;                   // uniform: every thread adapts its own copy
    uint64_t hi = wkey(lab[s], s) + 1;          // window 0: s alone
    int win = 0, win_rounds = 0, nf_first = 0, win_reps = 0, streak = 0;
    conv = true;
    for (int it = 0;; ++it) {
      // counters c + 1 serve the next round: they were last read two rounds ago
      const int c = it % 3;
      if (tid == 0) {
        S.nfront[(c + 1) % 3] = 0;
        S.nrep[(c + 1) % 3] = 0;
        S.wlo[(c + 1) % 3] = KEY_NONE;
      }
      // frontier: the pending centers below hi, with their label bases and
      // row offsets (see the rounds below); one LDS atomic per wavefront for
      // the slots, the repeats and the smallest key left out
      for (int vb = 0; vb < k; vb += NT) {
        const int v = vb + tid;
        uint64_t l = 0, other = KEY_NONE;
        bool take = false, rep = false;
        if (v < k && pend[v]) {
          l = lab[v];
          const uint64_t key = wkey(l, v);
          if (key < hi) {
            take = true;
            rep = seen[v] == win;
            seen[v] = win;
            pend[v] = 0;
          } else {
            other = key;
          }
        }
        const uint64_t tmask = __ballot(take);
        if (tmask) {
          int base = 0;
          if ((tid & 63) == 0) base = atomicAdd(&S.nfront[c], __popcll(tmask));
          base = __builtin_amdgcn_readlane(base, 0);
          if (take) {
            const int j = base + lanes_below(tmask);
            L.front1[j] = v;
            L.dist[j] = (int64_t)((l & ~(uint64_t)0x7ff) + (1ull << 11) + (uint32_t)v);
            L.pred[j] = v * k;
          }
        }
        const uint64_t rmask = __ballot(rep);
        if (rmask && (tid & 63) == 0) atomicAdd(&S.nrep[c], __popcll(rmask));
        const uint64_t m = wave_min_u64(other);
        if (m != KEY_NONE && (tid & 63) == 0) atomicMin((unsigned long long *)&S.wlo[c], (unsigned long long)m);
      }
      __syncthreads();
      const int nf = S.nfront[c];
      if (nf == 0) break;                       // hi is always above the smallest pending key
      if (nf_first == 0) nf_first = nf;
      win_rounds += 1;
      win_reps += S.nrep[c];
      const uint64_t *FB = reinterpret_cast<const uint64_t *>(L.dist);
      constexpr int B = 4;
      // candidate of target v over frontier entries j0, j0 + G, ...; returns
      // the new key when v's label dropped below the bound (v is pending)
      auto relax_pend = [&](int v, int j0) -> uint64_t {
        uint64_t best = KEY_NONE;
        for (int j = j0; j < nf; j += B * G) {
          uint64_t bs[B];
          uint32_t hw[B];
          bool ok[B];
#pragma unroll
          for (int x = 0; x < B; ++x) {
            const int jj = j + x * G;
            ok[x] = jj < nf;
            const int idx = ok[x] ? jj : j;
            bs[x] = FB[idx];
            hw[x] = Whi[WS * (uint32_t)(L.pred[idx] + v)];
          }
#pragma unroll
          for (int x = 0; x < B; ++x) {
            const uint64_t cand = bs[x] + ((uint64_t)(int64_t)(int32_t)(hw[x] ^ 0x80000000u) << 22);
            best = (ok[x] && hw[x] != 0xffffffffu && cand < best) ? cand : best;
          }
        }
        if (best != KEY_NONE && best < atomicMin((unsigned long long *)&lab[v], (unsigned long long)best) &&
            (int64_t)(best >> 22) - LAB_BIAS + pot_s - L.pot[v] < Db) {
          pend[v] = 1;
          return wkey(best, v);
        }
        return KEY_NONE;
      };
      for (int vb = 0; vb < (k <= NT ? 1 : k); vb += NT) {
        uint64_t mk = KEY_NONE;
        if (k <= NT) {
          if (tg < G && tv != s) mk = relax_pend(tv, tg);
        } else {
          const int v = vb + tid;
          if (v < k && v != s) mk = relax_pend(v, 0);
        }
        const uint64_t m = wave_min_u64(mk);
        if (m != KEY_NONE && (tid & 63) == 0) atomicMin((unsigned long long *)&S.wlo[c], (unsigned long long)m);
      }
      rounds += 1;
      relax += (int64_t)nf * k;
      __syncthreads();                          // labels, pending flags and wlo[c] are in place
      const uint64_t lo = S.wlo[c];             // the smallest pending key
      if (lo >= hi || win == 0) {
        // the window is done (s's after its one round: the centers it
        // reaches may lie below s in reduced terms)
        if (win > 0) {
          if (win_reps > 0) {
            width = width > 1 ? width / 2 : 1;
            streak = 0;
          } else if (win_rounds == 1 && nf_first < 8) {
            if (++streak == 4) {
              width = width < (1ll << 50) ? width * 2 : width;
              streak = 0;
            }
          } else {
            streak = 0;
          }
        }
        if (lo == KEY_NONE || lo >= key_db) break;
        hi = lo + (uint64_t)width;
        win += 1;
        win_rounds = nf_first = win_reps = 0;
      }
      if (rounds > cap_rounds) { conv = false; break; }
    }
    if (tid == 0) S.wdelta = width;
    __syncthreads();
  }
  for (int t = 1; t <= k + 1 && !(!WLDS && prune); ++t) {
    // round t relaxes out of the frontier of size nfront[t % 3] in list t & 1,
    // appends to nfront[(t + 1) % 3] and list (t + 1) & 1, and clears
    // nfront[(t + 2) % 3]: that counter was last read before the previous
    // barrier and is next appended to after the coming one
    const int nf = S.nfront[t % 3];
    const int32_t *F = (t & 1) ? L.front1 : L.front0;
    int32_t *Fn = (t & 1) ? L.front0 : L.front1;
    int32_t *cnt_next = &S.nfront[(t + 1) % 3];
    // candidate of target v over frontier entries j = j0, j0+G, ... in
    // batches of four: all loads of a batch are in flight together.  Returns
    // true when v's label dropped and v is not yet in the next frontier
    // (several threads of a target may lower it; the stamp admits one).
    constexpr int B = 4;
    if (!WLDS) {
      // table in global memory: every frontier entry's label base (label
      // without its predecessor, plus one edge, with the entry as
      // predecessor) and row offset are formed once, so a relaxation is a
      // load, a shifted add and a minimum (dist and pred are free until the
      // labels are unpacked)
      for (int j = tid; j < nf; j += NT) {
        const int u = F[j];
        L.dist[j] = (int64_t)((lab[u] & ~(uint64_t)0x7ff) + (1ull << 11) + (uint32_t)u);
        L.pred[j] = u * k;
      }
      __syncthreads();
    }
    const uint64_t *FB = reinterpret_cast<const uint64_t *>(L.dist);
    auto relax_target = [&](int v, int j0) -> bool {
      uint64_t best = KEY_NONE;
      if (!WLDS) {
        for (int j = j0; j < nf; j += B * G) {
          uint64_t bs[B];
          uint32_t hi[B];
          bool ok[B];
#pragma unroll
          for (int x = 0; x < B; ++x) {
            const int jj = j + x * G;
            ok[x] = jj < nf;
            const int idx = ok[x] ? jj : j;
            bs[x] = FB[idx];
            hi[x] = Whi[(uint32_t)(L.pred[idx] + v)];
          }
#pragma unroll
          for (int x = 0; x < B; ++x) {
            const uint64_t c = bs[x] + ((uint64_t)(int64_t)(int32_t)(hi[x] ^ 0x80000000u) << 22);
            best = (ok[x] && hi[x] != 0xffffffffu && c < best) ? c : best;
          }
        }
      }
      for (int j = j0; WLDS && j < nf; j += B * G) {
        int32_t u[B], off[B];
        bool ok[B];
#pragma unroll
        for (int x = 0; x < B; ++x) {
          const int jj = j + x * G;
          ok[x] = jj < nf;
          u[x] = F[ok[x] ? jj : j];
          off[x] = u[x] * k;
        }
        uint64_t lu[B];
        uint32_t hi[B];
#pragma unroll
        for (int x = 0; x < B; ++x) {
          lu[x] = lab[u[x]];
          hi[x] = Whi[WS * ((int64_t)off[x] + v)];
        }
#pragma unroll
        for (int x = 0; x < B; ++x)
          if (ok[x] && hi[x] != 0xffffffffu)
            best = umin(best, (lu[x] & ~(uint64_t)0x7ff) +
                                  ((uint64_t)(int64_t)(int32_t)(hi[x] - 0x80000000u) << 22) +
                                  (1ull << 11) + (uint32_t)u[x]);
      }
      if (best == KEY_NONE || !(best < atomicMin((unsigned long long *)&lab[v], (unsigned long long)best)))
        return false;
      if (prune && (int64_t)(best >> 22) - LAB_BIAS + pot_s - L.pot[v] >= Db) return false;
      return atomicExch(&stamp[v], t) != t;
    };
    // append the centers whose lanes say so: one LDS atomic per wavefront
    auto append = [&](bool app, int v) {
      const uint64_t mask = __ballot(app);
      if (mask) {
        int base = 0;
        if ((tid & 63) == 0) base = atomicAdd(cnt_next, __popcll(mask));
        base = __builtin_amdgcn_readlane(base, 0);
        if (app) Fn[base + lanes_below(mask)] = v;
      }
    };
    if (tid == 0) S.nfront[(t + 2) % 3] = 0;
    if (k <= NT) {
      append(tg < G && tv != s && relax_target(tv, tg), tv);
    } else {
      for (int vb = 0; vb < k; vb += NT) {
        const int v = vb + tid;
        append(v < k && v != s && relax_target(v, 0), v);
      }
    }
    __syncthreads();
    const int nnext = *cnt_next;
    rounds += 1;
    relax += (int64_t)nf * k;
    if (nnext == 0) { conv = true; break; }
  }
  // unpack (hop takes the stamps' place); pruned: only the centers below
  // the bound keep their labels
  const int64_t D = Db > 0 ? Db : 0;
  for (int v = tid; v < k; v += NT) {
    const uint64_t l = lab[v];
    const int64_t d = (int64_t)(l >> 22) - LAB_BIAS;
    const bool r = l != KEY_NONE && (!prune || v == s || d + pot_s - L.pot[v] < Db);
    L.dist[v] = r ? d : DIST_NONE;
    if (!prune) L.pot2[v] = L.dist[v];
    else {
      const int64_t p2 = r ? d : L.pot[v] - pot_s + D;
      L.pot2[v] = p2 < POT_FLOOR ? POT_FLOOR : p2;
    }
    L.hop[v] = r ? (int32_t)((l >> 11) & 0x7ff) : -1;
    L.pred[v] = (r && v != s) ? (int32_t)(l & 0x7ff) : -1;
  }
  if (tid == 0) {
    S.stats[ST_BF_ROUNDS] += rounds;
    S.stats[ST_RELAX] += relax;
    if (prune) S.stats[ST_BF_PRUNED] += 1;
    S.depth[mode] += ((int32_t)rounds * 16 - S.depth[mode]) / 8;
    const int64_t spent = now() - t_start;
    S.stats[ST_T_BF] += spent;
    const int64_t per = spent * 16 / (rounds > 0 ? rounds : 1);
    S.round_t += ((int32_t)min(per, (int64_t)INT32_MAX / 2) - S.round_t) / 8;
    S.nsearch += 1;
    if (!conv) S.status = -5;   // LBDD_E_INTERNAL: negative cycle reachable
  }
  __syncthreads();
  return conv;
}


// Label of s_in from the center labels (dist, hop) of a search from s.
// s_in has no out-edges, so the center labels do not depend on its in-edges
// (cycle mode: W[u][s]; path mode: the penalty difference).  In synchronous
// rounds s_in first reaches its final label best = min_u dist[u] + w(u, s_in)
// in the round after the earliest of those minimisers got its final label
// (hop[u]), and its predecessor is the smallest minimiser with that hop.
// This also answers a path search from the labels of a cycle search that
// applied nothing: both searches relax the same transfer edges.
__device__ __forceinline__ void sin_from_labels(const InstView &I, const Lds &L, int s, int mode) {
  const int k = I.k;
  const int tid = threadIdx.x;
  // path mode: a unit leaving the anchor saves what its last unit beyond
  // capacity pays (the anchor is overloaded whenever a path search runs)
  const int64_t q_anchor =
      mode == 0 ? 0 : penalty_at(I, L, s, L.load[s] > L.cap[s] ? (int64_t)L.load[s] - L.cap[s] : 1);
  auto in_weight = [&](int u, int64_t &w) -> bool {
    if (u == s || L.dist[u] == DIST_NONE) return false;
    if (mode == 0) {
      const uint64_t key = L.W[(int64_t)u * k + s];
      if (key == KEY_NONE) return false;
      w = key_delta(key);
    } else {
      // what one more unit at u would pay, minus what the anchor saves
      w = (L.load[u] >= L.cap[u] ? penalty_at(I, L, u, (int64_t)L.load[u] - L.cap[u] + 1) : 0) - q_anchor;
    }
    return true;
  };
  if (tid == 0) { L.red[0] = KEY_NONE; L.red[1] = KEY_NONE; }
  __syncthreads();
  for (int u = tid; u < k; u += NT) {
    int64_t w;
    if (in_weight(u, w)) atomicMin((unsigned long long *)&L.red[0], (unsigned long long)(L.dist[u] + w + DIST_BIAS));
  }
  __syncthreads();
  const uint64_t best = L.red[0];
  for (int u = tid; u < k; u += NT) {
    int64_t w;
    if (best != KEY_NONE && in_weight(u, w) && (uint64_t)(L.dist[u] + w + DIST_BIAS) == best)
      atomicMin((unsigned long long *)&L.red[1], (unsigned long long)((uint64_t)L.hop[u] << 32 | (uint32_t)u));
  }
  __syncthreads();
  if (tid == 0) {
    if (best == KEY_NONE) {
      L.dist[k] = DIST_NONE;
      L.pred[k] = -1;
    } else {
      L.dist[k] = (int64_t)best - DIST_BIAS;
      L.pred[k] = (int32_t)(uint32_t)L.red[1];
    }
  }
  __syncthreads();
}

// Search from s in Dijkstra order by one wavefront, for when the node
// potentials pot are feasible on every edge except those leaving s (the
// search never enters s, so only its first hops can have negative reduced
// weight w(u, v) + pot[u] - pot[v]).  Centers are settled in the order of
// (reduced label, edges), which is a valid Dijkstra order for these pairs of
// weights, so each settled center has its shortest distance and the fewest
// edges among its shortest paths: the label and the round in which the
// synchronous Bellman-Ford rounds fix it.  Its predecessor is the smallest
// settled center that reaches it with that pair (the smallest candidate of
// that round).  Center v belongs to lane v % 64, slot v / 64.
//
// The search stops as soon as no open center can matter for s_in, whose
// candidate through u is u's label + w(u, s_in):
//   cycle mode: w(u, s) is feasible, so the candidate is at least u's reduced
//     label; after s, centers are settled while the smallest open reduced
//     label is negative;
//   path mode: the candidate is u's reduced label + P(u), P(u) = pot[u] +
//     w(u, s_in) - pot[s]; the search stops once (smallest open reduced
//     label) + min P exceeds both -1 and the best candidate so far.
// Every center that attains s_in's label, if it is negative, is settled, so
// sin_from_labels gives the synchronous rounds' s_in label and path.  Open
// centers get DIST_NONE.  The candidate potentials pot2 are the labels of the
// settled centers and pot[v] - pot[s] + D for the others, D >= 0 the reduced
// label the search stopped at: with D no smaller than any settled reduced
// label and no open center below it, pot2 is feasible on every edge that pot
// was, and on the edges out of s as well.
// Key of an open center: ((reduced label + DJ_BIAS) << 18) | (edges << 9) |
// predecessor, so one unsigned minimum orders by (reduced label, edges) and
// keeps the smallest predecessor among equal pairs.  Reduced labels stay
// within +-2^44 (|potential| <= 2^42, |distance| < k * 2^30 <= 2^39) and
// edges and centers below 512.
constexpr int64_t DJ_BIAS = 1ll << 45;
constexpr int DJ_SHIFT = 18;
template <bool WLDS, int NPL>
__device__ __forceinline__ void dijkstra_bounded(const InstView &I, const Lds &L, Scalars &S, int s,
                                                 int mode) {
  const int k = I.k;
  if (threadIdx.x < 64) {
    // an opaque copy of the lane index: what derives from it is computed here
    // rather than hoisted to the kernel's start, where it would hold
    // registers for the whole solve
    int lane = threadIdx.x;
    asm volatile("" : "+v"(lane));
    // high word of W[i]: Whi[WS * i]
    constexpr int WS = WLDS ? 2 : 1;
    const uint32_t *Whi = WLDS ? reinterpret_cast<const uint32_t *>(L.W) + 1 : L.wh;
    const int64_t t_start = now();
    const int64_t pot_s = L.pot[s];
    // path mode: what the anchor saves per unit it gives up; the bound term
    // P(u) = pot[u] + w(u, s_in) - pot[s] of a center u != s
    const int64_t q_anchor =
        mode == 0 ? 0 : penalty_at(I, L, s, L.load[s] > L.cap[s] ? (int64_t)L.load[s] - L.cap[s] : 1);
    auto bound_term = [&](int u) -> int64_t {
      const int64_t w =
          (L.load[u] >= L.cap[u] ? penalty_at(I, L, u, (int64_t)L.load[u] - L.cap[u] + 1) : 0) - q_anchor;
      return L.pot[u] + w - pot_s;
    };
    // open key of an unsettled center, all ones once settled or while
    // unreached
    uint64_t open[NPL];
    uint32_t done = 0;                           // bit i: slot i settled or beyond k
    uint64_t pm = KEY_NONE;
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      const int v = lane + 64 * i;
      done |= (v >= k ? 1u : 0u) << i;
      open[i] = v == s ? (uint64_t)DJ_BIAS << DJ_SHIFT : KEY_NONE;
      if (v < k) {
        L.dist[v] = DIST_NONE;
        L.pred[v] = -1;
        L.hop[v] = -1;
        if (mode == 1 && v != s) pm = umin(pm, (uint64_t)(bound_term(v) + DJ_BIAS));
      }
    }
    int64_t pmin = 0;
    if (mode == 1) {
      pm = wave_min_u64(pm);
      pmin = pm == KEY_NONE ? DJ_BIAS : (int64_t)pm - DJ_BIAS;   // k = 1: nothing to reach
    }
    int64_t best = INT64_MAX;                    // path mode: best s_in candidate so far
    int64_t top = 0;                             // largest settled reduced label
    int64_t D = -1;                              // reduced label the search stopped at
    int nset = 0;
    for (int step = 0; step < k; ++step) {
      uint64_t m = open[0];
#pragma unroll
      for (int i = 1; i < NPL; ++i) m = umin(m, open[i]);
      m = wave_min_u64(m);
      if (m == KEY_NONE) break;                  // every reachable center is settled
      const int64_t ml = (int64_t)(m >> DJ_SHIFT) - DJ_BIAS;
      if (step > 0 && (mode == 0 ? ml >= 0 : ml + pmin > (best < -1 ? best : -1))) {
        D = ml;
        break;
      }
      // the owner: first slot holding m, first lane of that slot
      int oi = -1;
      uint64_t om = 0;
#pragma unroll
      for (int i = NPL - 1; i >= 0; --i) {
        const uint64_t b = __ballot(open[i] == m);
        if (b) { oi = i; om = b; }
      }
      if (oi < 0) {                              // cannot happen: m is some lane's
        if (lane == 0) S.status = -5;            // LBDD_E_INTERNAL
        break;
      }
      const int ol = __builtin_ctzll(om);
      const int u = ol + 64 * oi;
      // the row of u, this lane's potentials and pot[u] in one round trip
      uint32_t hw[NPL];
      const uint32_t *row = Whi + WS * (size_t)u * k;
#pragma unroll
      for (int i = 0; i < NPL; ++i) hw[i] = row[WS * min(lane + 64 * i, k - 1)];
      const int64_t pot_u = L.pot[u];
      ++nset;
      top = ml > top ? ml : top;
      if (lane == ol) {
        L.dist[u] = ml - pot_s + pot_u;
        L.pred[u] = u == s ? -1 : (int32_t)(m & 511);
        L.hop[u] = (int32_t)((m >> 9) & 511);
      }
      if (mode == 1 && u != s) {
        const int64_t c = ml + bound_term(u);    // s_in's candidate through u
        best = c < best ? c : best;
      }
      done |= (lane == ol ? 1u : 0u) << oi;
      // one more edge, from u
      const uint64_t base = (m & ~(uint64_t)511) + (1u << 9) + (uint32_t)u;
#pragma unroll
      for (int i = 0; i < NPL; ++i) {            // branch-free: selects only
        const bool valid = !((done >> i) & 1u) && hw[i] != 0xffffffffu;
        const int64_t w = (int64_t)(int32_t)(hw[i] ^ 0x80000000u) + (pot_u - L.pot[min(lane + 64 * i, k - 1)]);
        const uint64_t c = valid ? base + ((uint64_t)w << DJ_SHIFT) : KEY_NONE;
        open[i] = ((done >> i) & 1u) ? KEY_NONE : umin(open[i], c);
      }
    }
    if (D < 0) D = top;                          // everything reachable was settled
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      const int v = lane + 64 * i;
      if (v >= k) continue;
      const bool settled = (done >> i) & 1u;
      const int64_t p2 = settled ? L.dist[v] : L.pot[v] - pot_s + D;
      L.pot2[v] = p2 < POT_FLOOR ? POT_FLOOR : p2;
    }
    if (lane == 0) {
      S.settled[mode] += (nset * 16 - S.settled[mode]) / 8;
      S.stats[ST_DJ_SETTLED] += nset;
      const int64_t spent = now() - t_start;
      S.stats[ST_T_DIJKSTRA] += spent;
      const int64_t per = spent * 16 / (nset > 0 ? nset : 1);
      S.step_t += ((int32_t)min(per, (int64_t)INT32_MAX / 2) - S.step_t) / 8;
      S.nsearch += 1;
    }
  }
  __syncthreads();
}

// The same bounded search in Dijkstra order for k > 128, over the
// workgroup's wavefronts: wave w owns centers 64 w .. 64 w + 63, one per
// lane.  A step takes each wave's smallest open key (and its
// center, the first lane holding it) into LDS, one barrier, then every thread
// picks the smallest over the waves (the first wave on equal keys, so the
// center settled is the same as by one wavefront scanning its slots in
// order), reads its own column of the settled center's row and relaxes it.
// The per-wave minima are double-buffered by step parity: a wave writes the
// next step's entry only after the barrier that every wave passes after
// reading this step's.  (k <= 512: the key holds edges and predecessor in
// 9 bits each.)
constexpr int DJ_MAX_K = 512;
template <bool WLDS>
__device__ __forceinline__ void dijkstra_waves(const InstView &I, const Lds &L, Scalars &S, int s,
                                               int mode) {
  const int k = I.k;
  const int tid = threadIdx.x;
  int lane = tid & 63;
  asm volatile("" : "+v"(lane));               // see dijkstra_bounded
  const int wave = tid >> 6;
  const int nw = (k + 63) >> 6;                  // waves that own centers
  const int v = wave * 64 + lane;
  const bool mine = v < k;
  constexpr int WS = WLDS ? 2 : 1;
  const uint32_t *Whi = WLDS ? reinterpret_cast<const uint32_t *>(L.W) + 1 : L.wh;
  uint64_t *wkey = L.wmin;                       // [2][NT / 64] per-wave minima
  int32_t *wnode = L.mrow;                       // [2][NT / 64] their centers (k + 1 >= 32)
  const int64_t t_start = tid == 0 ? now() : 0;
  const int64_t pot_s = L.pot[s];
  const int64_t q_anchor =
      mode == 0 ? 0 : penalty_at(I, L, s, L.load[s] > L.cap[s] ? (int64_t)L.load[s] - L.cap[s] : 1);
  auto bound_term = [&](int u) -> int64_t {
    const int64_t w =
        (L.load[u] >= L.cap[u] ? penalty_at(I, L, u, (int64_t)L.load[u] - L.cap[u] + 1) : 0) - q_anchor;
    return L.pot[u] + w - pot_s;
  };
  const int64_t pv = mine ? L.pot[v] : 0;
  uint64_t open = (mine && v == s) ? (uint64_t)DJ_BIAS << DJ_SHIFT : KEY_NONE;
  bool done = !mine;                             // settled, or no center here
  if (mine) {
    L.dist[v] = DIST_NONE;
    L.pred[v] = -1;
    L.hop[v] = -1;
  }
  int64_t pmin = 0;
  if (mode == 1) {
    const uint64_t pm = wave_min_u64((mine && v != s) ? (uint64_t)(bound_term(v) + DJ_BIAS) : KEY_NONE);
    if (lane == 0) wkey[NT / 64 + wave] = pm;
    __syncthreads();
    uint64_t g = KEY_NONE;
    for (int j = 0; j < nw; ++j) g = umin(g, wkey[NT / 64 + j]);
    pmin = g == KEY_NONE ? DJ_BIAS : (int64_t)g - DJ_BIAS;   // k = 1: nothing to reach
  }
  int64_t best = INT64_MAX;
  int64_t top = 0;
  int64_t D = -1;
  int nset = 0;
  for (int step = 0; step < k; ++step) {
    const int b = (step & 1) * (NT / 64);
    const uint64_t lm = wave_min_u64(open);
    const uint64_t hold = __ballot(open == lm);
    if (lane == 0) {
      wkey[b + wave] = lm;
      wnode[b + wave] = wave * 64 + (hold ? __builtin_ctzll(hold) : 0);
    }
    __syncthreads();
    // every wave wrote its entry (all ones without an open center): read the
    // entries of the DJ_MAX_K / 64 waves that can own centers at once, then
    // take the first smallest
    constexpr int MW = DJ_MAX_K / 64;
    uint64_t xk[MW];
    int32_t xn[MW];
#pragma unroll
    for (int j = 0; j < MW; ++j) {
      xk[j] = wkey[b + j];
      xn[j] = wnode[b + j];
    }
    uint64_t m = KEY_NONE;
    int u = 0;
#pragma unroll
    for (int j = MW - 1; j >= 0; --j) {
      const bool le = xk[j] <= m;
      m = le ? xk[j] : m;
      u = le ? xn[j] : u;
    }
    if (m == KEY_NONE) break;                    // every reachable center is settled
    const int64_t ml = (int64_t)(m >> DJ_SHIFT) - DJ_BIAS;
    if (step > 0 && (mode == 0 ? ml >= 0 : ml + pmin > (best < -1 ? best : -1))) {
      D = ml;
      break;
    }
    const uint32_t hw = mine ? Whi[WS * ((int64_t)u * k + v)] : 0xffffffffu;
    const int64_t pot_u = L.pot[u];
    ++nset;
    top = ml > top ? ml : top;
    if (v == u) {
      L.dist[u] = ml - pot_s + pot_u;
      L.pred[u] = u == s ? -1 : (int32_t)(m & 511);
      L.hop[u] = (int32_t)((m >> 9) & 511);
      done = true;
      open = KEY_NONE;
    }
    if (mode == 1 && u != s) {
      const int64_t c = ml + bound_term(u);      // s_in's candidate through u
      best = c < best ? c : best;
    }
    if (!done && hw != 0xffffffffu) {
      const uint64_t base = (m & ~(uint64_t)511) + (1u << 9) + (uint32_t)u;
      const int64_t w = (int64_t)(int32_t)(hw ^ 0x80000000u) + (pot_u - pv);
      open = umin(open, base + ((uint64_t)w << DJ_SHIFT));
    }
  }
  if (D < 0) D = top;                            // everything reachable was settled
  if (mine) {
    const int64_t p2 = done ? L.dist[v] : pv - pot_s + D;
    L.pot2[v] = p2 < POT_FLOOR ? POT_FLOOR : p2;
  }
  if (tid == 0) {
    S.settled[mode] += (nset * 16 - S.settled[mode]) / 8;
    S.stats[ST_DJ_SETTLED] += nset;
    const int64_t spent = now() - t_start;
    S.stats[ST_T_DIJKSTRA] += spent;
    const int64_t per = spent * 16 / (nset > 0 ? nset : 1);
    S.step_t += ((int32_t)min(per, (int64_t)INT32_MAX / 2) - S.step_t) / 8;
    S.nsearch += 1;
  }
  __syncthreads();
}

// One refinement (mode 0: Algorithm 1, mode 1: Appendix A) anchored at s.
// With have_labels (mode 1 only) the search result is derived from the labels
// of the cycle search just run on the same W.  Returns true when nothing was
// applied and the search succeeded: the labels in LDS then describe the
// current W.
// Without labels the search runs in Dijkstra order, bounded to the centers
// that can matter for s_in, when the node potentials allow it (cycle mode:
// feasible except on edges leaving s, which is all an insert into s can
// break; path mode: feasible) and the cost model prefers it, else as
// Bellman-Ford rounds.
template <bool WLDS>
__device__ __forceinline__ bool refine(const InstView &I, const Lds &L, Scalars &S, int s, int mode,
                                       bool have_labels, bool use_t) {
  const int k = I.k;
  const int tid = threadIdx.x;
  // the potentials the search runs on: the sink potentials (path searches,
  // use_t) or pot; the search reads them through LS
  Lds LS = L;
  if (use_t) LS.pot = L.potT;
  const bool a_ok = S.pot_ok != 0;
  const bool pok = use_t ? S.potT_ok != 0 : a_ok;
  // cost model: a Bellman-Ford search takes `depth` rounds and one in
  // Dijkstra order `settled` steps (running means per mode, x16), and a round
  // costs `ratio` steps (x16): a fixed value, or by default the ratio of the
  // measured times of a round and a step.  The automatic choice first
  // measures each kind in each mode, and then takes the other kind in one
  // search of every 64, so that both measurements follow the workload.
  bool prefer;
  if (S.ratio != SEARCH_RATIO_AUTO) {
    prefer = (int64_t)S.depth[mode] * S.ratio > 16 * (int64_t)S.settled[mode];
  } else if (S.depth[mode] == 0 || S.round_t == 0) {
    prefer = false;                           // Bellman-Ford not yet measured in this mode
  } else if (S.settled[mode] == 0 || S.step_t == 0) {
    prefer = true;                            // nor Dijkstra order
  } else {
    const int64_t ratio = 16 * (int64_t)S.round_t / S.step_t;
    prefer = (int64_t)S.depth[mode] * ratio > 16 * (int64_t)S.settled[mode];
    if ((S.nsearch & 63) == 63) prefer = !prefer;
  }
  const bool dijkstra = !have_labels && pok && k <= DJ_MAX_K && prefer;
  if (tid == 0) {
    S.stats[mode == 0 ? ST_CYC_SEARCH : ST_PATH_SEARCH] += 1;
    if (have_labels) S.stats[ST_PATH_DERIVED] += 1;
    if (dijkstra) S.stats[ST_DIJKSTRA] += 1;
  }
  if (have_labels) {
    sin_from_labels(I, L, s, 1);
  } else if (dijkstra) {
    if (k <= 64) dijkstra_bounded<WLDS, 1>(I, LS, S, s, mode);
    else if (k <= 128) dijkstra_bounded<WLDS, 2>(I, LS, S, s, mode);
    else dijkstra_waves<WLDS>(I, LS, S, s, mode);
    if (S.status != 0) return false;
    sin_from_labels(I, L, s, mode);
  } else {
    if (!bellman_ford<WLDS>(I, LS, S, s, mode, pok)) return false;
    sin_from_labels(I, L, s, mode);
  }
  const bool complete = !have_labels && !dijkstra && !pok;   // unpruned rounds
  const int64_t D = L.dist[k];
  if (D == DIST_NONE || D >= 0) {             // only strictly negative refinements apply
    // nothing moved; a search on the sink potentials leaves pot as it was
    if (!have_labels && !use_t) take_potential<WLDS>(I, L, S, s, 0);
    return complete;                          // labels of every center describe W
  }
  if (tid == 0) {
    S.pot_ok = 0;                             // W is about to change
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
    const int ntrans = mode == 0 ? nedges : nedges - 1;
    // read every moved unit before any move; a dummy transfer (strict-LBDD
    // only) moves no real unit
    int nmov = 0;
    for (int e = 0; e < ntrans; ++e) {
      const int u = path[len - 1 - e];
      int v = path[len - 2 - e];
      if (v == k) v = s;
      const uint64_t key = L.W[(int64_t)u * k + v];
      if (key == DUMMY_KEY) continue;
      L.mrow[nmov] = (int32_t)key_rank(key);
      L.mfrom[nmov] = u;
      L.mto[nmov] = v;
      ++nmov;
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
  const int64_t t0 = tid == 0 ? now() : 0;
  // every unit leaves its old center's lists before any joins the new ones;
  // lists left unknown are refilled from the final members
  move_lists(I, L, nmov);
  refill_moved(I, L, S, nmov);
  if (I.strict) {
    // the moves changed the loads of their centers and no other: their rows
    // take the list heads and the dummy transfers again
    for (int64_t t = tid; t < (int64_t)2 * nmov * k; t += NT) {
      const int j = (int)(t / k), w = (int)(t - (int64_t)j * k);
      const int u = (j & 1) ? L.mto[j >> 1] : L.mfrom[j >> 1];
      set_w(L, k, u, w, (int64_t)u * k + w, strict_entry(I, L, u, w));
    }
  }
  if (tid == 0) S.stats[ST_T_RESCAN] += now() - t0;
  __syncthreads();
  if (S.status == 0) {
    if (!use_t) {
      take_potential<WLDS>(I, L, S, s, nmov);
    } else if (a_ok) {
      // the search ran on the sink potentials: pot itself is checked (and
      // repaired) on the changed rows
      for (int u = tid; u < k; u += NT) L.pot2[u] = L.pot[u];
      __syncthreads();
      take_potential<WLDS>(I, L, S, s, nmov);
    }
  }
  // the moves changed the rows of their centers: potT checks them later
  if (S.sink_every > 0) {
    for (int e = tid; e < nmov; e += NT) {
      atomicOr(&L.dirty[L.mfrom[e] >> 5], 1u << (L.mfrom[e] & 31));
      atomicOr(&L.dirty[L.mto[e] >> 5], 1u << (L.mto[e] & 31));
    }
    __syncthreads();
  }
  return false;
}

// Strict-LBDD allotment (Algorithm 4): the center with free capacity of the
// smallest cost for this unit, smallest index among equal costs.  Every
// thread returns it.  Some center always has room while units remain (the
// capacities, with the dummy center's, sum to at least n); if none has, the
// status records the failed invariant and `fallback` is returned.
__device__ __forceinline__ int strict_center(const InstView &I, const Lds &L, Scalars &S,
                                             const int32_t *row, int fallback) {
  const int k = I.k;
  uint64_t b = KEY_NONE;
  for (int t = threadIdx.x; t < k; t += NT)
    if (L.load[t] < L.cap[t]) b = umin(b, (uint64_t)(uint32_t)row[t] << 32 | (uint32_t)t);
  b = wave_min_u64(b);
  if ((threadIdx.x & 63) == 0) L.wmin[threadIdx.x >> 6] = b;
  __syncthreads();
  uint64_t g = KEY_NONE;
#pragma unroll
  for (int j = 0; j < NT / 64; ++j) g = umin(g, L.wmin[j]);
  if (g == KEY_NONE) {
    if (threadIdx.x == 0) S.status = -5;
    return fallback;
  }
  return (int)(uint32_t)g;
}

// Layout of the dynamic LDS of one solving workgroup (solve_lds_bytes).
template <bool WLDS>
__device__ __forceinline__ Lds carve_lds(const InstView &I, unsigned char *lds) {
  const int k = I.k, K1 = k + 1;
  Lds L;
  unsigned char *p = lds;
  if (WLDS) { L.W = reinterpret_cast<uint64_t *>(p); p += (size_t)k * k * 8; }
  else L.W = I.W;
  L.wh = WLDS ? nullptr : I.Wh;
  L.wt = I.WhT;
  L.red = reinterpret_cast<uint64_t *>(p); p += (size_t)K1 * 8;
  L.dist = reinterpret_cast<int64_t *>(p); p += (size_t)K1 * 8;
  L.pred = reinterpret_cast<int32_t *>(p); p += (size_t)K1 * 4;
  L.hop = reinterpret_cast<int32_t *>(p); p += (size_t)K1 * 4;
  L.front0 = reinterpret_cast<int32_t *>(p); p += (size_t)K1 * 4;
  L.front1 = reinterpret_cast<int32_t *>(p); p += (size_t)K1 * 4;
  p = lds + (((p - lds) + 7) & ~(ptrdiff_t)7);   // offsets keep the LDS address space
  L.pot = reinterpret_cast<int64_t *>(p); p += (size_t)k * 8;
  L.pot2 = reinterpret_cast<int64_t *>(p); p += (size_t)k * 8;
  L.potT = reinterpret_cast<int64_t *>(p); p += (size_t)k * 8;
  L.dirty = reinterpret_cast<uint32_t *>(p); p += ((size_t)k + 31) / 32 * 4;
  p = lds + (((p - lds) + 7) & ~(ptrdiff_t)7);
  L.load = reinterpret_cast<int32_t *>(p); p += (size_t)k * 4;
  L.cap = reinterpret_cast<int32_t *>(p); p += (size_t)k * 4;
  L.pen = reinterpret_cast<int32_t *>(p); p += (size_t)k * 4;
  L.mrow = reinterpret_cast<int32_t *>(p); p += (size_t)K1 * 4;
  L.mfrom = reinterpret_cast<int32_t *>(p); p += (size_t)K1 * 4;
  L.mto = reinterpret_cast<int32_t *>(p); p += (size_t)K1 * 4;
  L.trow = reinterpret_cast<int32_t *>(p); p += (size_t)K1 * 4;
  p = lds + (((p - lds) + 7) & ~(ptrdiff_t)7);   // offsets keep the LDS address space
  L.wmin = reinterpret_cast<uint64_t *>(p);
  return L;
}

// Iterations [r_begin, r_end) of one instance by the calling workgroup.
template <bool WLDS>
__device__ __forceinline__ void solve_range(const InstView &I, int64_t r_begin, int64_t r_end,
                                            unsigned char *lds, Scalars &S) {
  const int k = I.k;
  const int tid = threadIdx.x;
  const Lds L = carve_lds<WLDS>(I, lds);

  if (WLDS)
    for (int64_t i = tid; i < (int64_t)k * k; i += NT) L.W[i] = I.W[i];
  else   // a launch that kept W in LDS left the high words behind
    for (int64_t i = tid; i < (int64_t)k * k; i += NT) {
      const uint32_t hi = (uint32_t)(I.W[i] >> 32);
      const int u = (int)(i / k), w = (int)(i - (int64_t)u * k);
      L.wh[i] = hi;
      L.wt[(int64_t)w * k + u] = hi;
    }
  for (int i = tid; i < k; i += NT) L.pot[i] = 0;
  for (int i = tid; i < (k + 31) / 32; i += NT) L.dirty[i] = 0;
  for (int i = tid; i < k; i += NT) { L.load[i] = I.load[i]; L.cap[i] = I.cap[i]; L.pen[i] = I.pen[i]; }
  if (tid == 0) {
    // the potential is not kept between launches: the first search rebuilds it
    // (an empty table is certified by the zero potential)
    S.pot_ok = r_begin == 0;
    S.depth[0] = S.depth[1] = 0;
    S.settled[0] = S.settled[1] = 0;
    S.round_t = S.step_t = 0;
    S.nsearch = 0;
    S.jflags[0] = S.jflags[1] = 0;
    S.ratio = (int32_t)min(max(I.scalars[SC_RATIO], SEARCH_RATIO_AUTO), MAX_SEARCH_RATIO);
    S.sink_every = (int32_t)min(max(I.scalars[SC_SINK_EVERY], (int64_t)0), (int64_t)MAX_SINK_EVERY);
    S.sink_age = 0;
    S.potT_ok = 0;
    S.wdelta = 1ll << 11;   // one unit of reduced distance
    S.obj = I.scalars[SC_OBJECTIVE];
    S.status = (int32_t)I.scalars[SC_STATUS];
    for (int j = 0; j < SC_NSTATS; ++j) S.stats[j] = I.scalars[SC_STAT0 + j];
  }
  if (tid == 0 && S.stats[ST_T_FIRST] == 0) S.stats[ST_T_FIRST] = now();
  __syncthreads();
  const bool ok0 = S.status == 0;
  int64_t r = r_begin;
  // The last wavefront, which has no target of an allotment's joins while
  // k <= NT - 64, fetches the cost-matrix row and the most suitable center
  // of the unit PF_AHEAD iterations ahead into the caches: one word per 64
  // bytes of the row (lane 63: the center).  The words are folded into a sink
  // only PF_AHEAD iterations after their loads, so the allotments that follow
  // do not wait for them, and the rows they read are then cache hits.
  constexpr int PF_AHEAD = 2;
  const bool pf_wave = k <= NT - 64 && tid >= NT - 64;
  const int pf_lane = tid & 63;
  int32_t pf_new = 0, pf_old = 0, pf_sink = 0;
  // The allotment's bookkeeping (assignment, member list, load, objective)
  // runs on a thread of a wavefront without join targets when there is one,
  // so the joins do not wait behind its loads and stores.
  const int t_book = k <= NT - 128 ? NT - 128 : 0;
  if (ok0) {
    for (; r < r_end; ++r) {
      // phase timers: thread 0, one iteration in 8 (a timer read holds up
      // the next barrier), scaled by 8
      const bool timed = tid == 0 && (r & 7) == 0;
      const int64_t t0 = timed ? now() : 0;
      const int32_t *row = I.cm + r * k;
      int s = I.smin[r];
      if (pf_wave) {
        pf_sink += pf_old;
        pf_old = pf_new;
        pf_new = 0;
        const int64_t rp = r + PF_AHEAD;
        const int e = pf_lane * 16;
        if (rp < I.n) {
          if (pf_lane == 63) pf_new = I.smin[rp];
          else if (e < k + 15) pf_new = I.cm[rp * k + min(e, k - 1)];
        }
      }
      if (I.strict) {
        // strict-LBDD: the cheapest center with free capacity (the most
        // suitable one whenever it has room); every thread reads the load
        // before the bookkeeping thread changes it below
        const bool full = L.load[s] >= L.cap[s];
        __syncthreads();
        if (full) s = strict_center(I, L, S, row, s);
      }
      if (tid == t_book) {
        const int ld = L.load[s];
        const int vac = ld < L.cap[s];
        S.vacant = vac;
        I.assign[r] = s;
        I.members[(int64_t)s * I.n + ld] = (int32_t)r;
        I.slot[r] = ld;
        L.load[s] = ld + 1;
        S.obj += (int64_t)row[s] + (vac ? 0 : penalty_at(I, L, s, (int64_t)ld - L.cap[s] + 1));
      }
      const int ins = join_center(I, L, S, (int)r, s, (int)(r & 1));   // contains a barrier
      if ((ins & 1) && S.sink_every > 0 && tid == 0) atomicOr(&L.dirty[s >> 5], 1u << (s & 31));
      if (I.strict && L.load[s] == L.cap[s]) {
        // s has just become full: its dummy transfers are gone
        for (int v = tid; v < k; v += NT) set_w(L, k, s, v, (int64_t)s * k + v, strict_entry(I, L, s, v));
        __syncthreads();
      }
      const int64_t t1 = timed ? now() : 0;
      // Negative Cycle Refinement can only find something if the current W
      // may hold a negative cycle: the insert lowered an entry and the node
      // potentials no longer certify that W has none.
      const bool search = (ins & 1) && (!S.pot_ok || (ins & 2));
      bool labels = false;                        // LDS labels describe the current W
      if (search) labels = refine<WLDS>(I, L, S, s, 0, false, false);
      else if (tid == 0) S.stats[ST_CYC_SKIPPED] += 1;
      __syncthreads();
      const int64_t t2 = timed ? now() : 0;
      if (S.status != 0) break;
      if (!S.vacant) {
        // path searches run on the sink potentials: checked on the rows
        // changed since, or computed afresh every sink_every-th path search
        // (and whenever a check cannot repair them)
        bool use_t = false;
        if (S.sink_every > 0 && S.status == 0) {
          const bool due = !S.potT_ok || S.sink_age + 1 >= S.sink_every;   // the same in every thread
          __syncthreads();                      // read before thread 0 writes it
          if (!due) refresh_sink<WLDS>(I, L, S);
          if (due || !S.potT_ok) sink_potential<WLDS>(I, L, S);
          if (threadIdx.x == 0) S.sink_age = due ? 0 : S.sink_age + 1;
          __syncthreads();
          use_t = S.potT_ok != 0;
        }
        if (S.status == 0) refine<WLDS>(I, L, S, s, 1, labels, use_t);
      }
      __syncthreads();
      if (timed) {
        const int64_t t3 = now();
        S.stats[ST_T_ALLOT] += 8 * (t1 - t0);
        S.stats[ST_T_CYCLE] += 8 * (t2 - t1);
        S.stats[ST_T_PATH] += 8 * (t3 - t2);
      }
      if (S.status != 0) break;
    }
  }
  pf_sink += pf_old + pf_new;
  asm volatile("" : : "v"(pf_sink));          // keeps the fetches
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
    S.stats[ST_T_LAST] = now();
    for (int j = 0; j < SC_NSTATS; ++j) I.scalars[SC_STAT0 + j] = S.stats[j];
  }
}

template <bool WLDS>
__global__ __launch_bounds__(NT) void solve_kernel(InstView I, int64_t r_begin, int64_t r_end) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ Scalars S;
  solve_range<WLDS>(I, r_begin, r_end, lds, S);
}

// Many instances in one launch: every workgroup is a worker that claims the
// next instance from a device-side queue (items are ordered largest first by
// the host) and runs all its remaining iterations, then claims again.  The
// W placement and the load width are chosen per instance.
__global__ __launch_bounds__(NT) void solve_batch_kernel(const BatchItem *__restrict__ items,
                                                         int32_t m, int32_t *head,
                                                         uint32_t lds_avail) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ Scalars S;
  __shared__ int32_t claim;
  for (;;) {
    __syncthreads();                         // the previous instance is written back
    if (threadIdx.x == 0) claim = atomicAdd(head, 1);
    __syncthreads();
    const int32_t c = __builtin_amdgcn_readfirstlane(claim);   // uniform: scalar loads below
    if (c >= m) break;
    const InstView I = items[c].inst;
    const int64_t r0 = items[c].r_begin;
    const bool wlds = solve_lds_bytes(I.k, true) <= lds_avail;
    if (wlds) solve_range<true>(I, r0, I.n, lds, S);
    else solve_range<false>(I, r0, I.n, lds, S);
  }
}

}  // namespace

namespace {

__global__ void init_state_kernel(InstView I) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t0; i < I.n; i += stride) I.assign[i] = -1;
  for (int64_t i = t0; i < (int64_t)I.k * I.k; i += stride) {
    // strict-LBDD: every center with capacity starts full of dummy units
    const int u = (int)(i / I.k), v = (int)(i - (int64_t)u * I.k);
    const uint64_t w0 = (I.strict && u != v && I.cap[u] > 0) ? DUMMY_KEY : KEY_NONE;
    I.W[i] = w0;
    I.Wh[i] = (uint32_t)(w0 >> 32);
    I.WhT[(int64_t)v * I.k + u] = (uint32_t)(w0 >> 32);
    I.meta[i] = META_ALL;                       // empty center: every unit (none) held
    I.thr[i] = KEY_NONE;                        // ... so every joining unit enters
  }
  for (int64_t i = t0; i < (int64_t)I.k * I.k * BEST_M; i += stride) I.best[i] = KEY_NONE;
  for (int64_t i = t0; i < I.k; i += stride) I.load[i] = 0;
  for (int64_t i = t0; i < SC_COUNT; i += stride) I.scalars[i] = 0;
}

// out[order[r]] = assign[r]: back from processing order to the caller's
// order, with -1 for a unit at the dummy center of strict-LBDD (dummy = -1
// when there is none).
__global__ void unpermute_kernel(int64_t n, const int64_t *__restrict__ order,
                                 const int32_t *__restrict__ assign, int32_t dummy,
                                 int32_t *__restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) {
    const int32_t a = assign[r];
    out[order[r]] = (a == dummy) ? -1 : a;
  }
}

}  // namespace

hipError_t launch_init_state(const InstView &I, hipStream_t st) {
  init_state_kernel<<<1024, 256, 0, st>>>(I);
  return hipGetLastError();
}

hipError_t launch_unpermute(int64_t n, const int64_t *order, const int32_t *assign, int32_t dummy,
                            int32_t *out, hipStream_t st) {
  unpermute_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, order, assign, dummy, out);
  return hipGetLastError();
}


template <bool WLDS>
static hipError_t launch_solve_t(const InstView &I, int64_t r_begin, int64_t r_end, size_t bytes,
                                 hipStream_t st) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&solve_kernel<WLDS>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  solve_kernel<WLDS><<<1, NT, bytes, st>>>(I, r_begin, r_end);
  return hipGetLastError();
}

namespace {

// Resident worker loop of the request server.  A worker claims the oldest
// published job that nobody has claimed (compare-and-swap on a device
// counter, only ever below the published count, so no claim is lost), copies
// its descriptor from pinned host memory, solves it, and signals completion
// with a system-scope release store into pinned memory (so the host also sees
// the job's results in device memory).  A worker leaves when shutdown is
// requested or after idle_ticks of device time in which it took no job and no
// job was published; the host launches the kernel again when new work arrives
// after all workers left.
__global__ __launch_bounds__(NT) void service_kernel(ServiceCtl *ctl, const ServiceJob *ring,
                                                     int32_t ring_size, int64_t *done, ServiceDev *dev,
                                                     uint32_t lds_avail, int64_t idle_ticks) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ Scalars S;
  __shared__ int64_t claim;
  constexpr int WORDS = sizeof(InstView) / 4;
  __shared__ uint32_t job[WORDS];
  constexpr int64_t POLL_TICKS = 200;          // 2 us of the 100 MHz device timer
  for (;;) {
    __syncthreads();                           // previous job fully written back
    if (threadIdx.x == 0) {
      int64_t got = -1;
      int64_t t0 = now();
      int64_t seen = -1;
      for (;;) {
        // at most one worker every POLL_TICKS reads the host's control block
        // (a flood of reads over PCIe from idle workers would starve the
        // command processor's own fetches of queue packets) and mirrors it
        const int64_t t = now();
        int64_t last = __hip_atomic_load(&dev->polled, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (t - last > POLL_TICKS &&
            __hip_atomic_compare_exchange_strong(&dev->polled, &last, t, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)) {
          const int64_t p = __hip_atomic_load(&ctl->published, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
          const int64_t q = __hip_atomic_load(&ctl->shutdown, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          __hip_atomic_fetch_max(&dev->published, p, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          if (q) __hip_atomic_store(&dev->shutdown, q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // read-modify-writes are performed where the line is coherent for the
        // whole device; a plain load could keep hitting a stale copy in this
        // XCD's L2
        const int64_t pub = __hip_atomic_fetch_add(&dev->published, (int64_t)0, __ATOMIC_ACQUIRE,
                                                   __HIP_MEMORY_SCOPE_AGENT);
        // the idle clock restarts whenever a job is published: while requests
        // keep arriving the whole pool stays, even if others take them
        if (pub != seen) { seen = pub; t0 = now(); }
        int64_t h = __hip_atomic_fetch_add(&dev->head, (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (h < pub) {
          if (__hip_atomic_compare_exchange_strong(&dev->head, &h, h + 1, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT)) {
            got = h;
            break;
          }
          continue;                              // another worker took job h: try the next one
        }
        if (__hip_atomic_fetch_add(&dev->shutdown, (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        if (now() - t0 > idle_ticks) break;
        // ~25 us between polls: hundreds of workers polling faster hold up
        // the launch of other kernels on the device
#pragma unroll
        for (int z = 0; z < 8; ++z) __builtin_amdgcn_s_sleep(127);
      }
      claim = got;
      if (got >= 0) {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(&ring[got % ring_size].inst);
        for (int i = 0; i < WORDS; ++i)
          job[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
    __syncthreads();
    const int64_t c = claim;
    if (c < 0) break;
    InstView I;
    uint32_t *iw = reinterpret_cast<uint32_t *>(&I);
#pragma unroll
    for (int i = 0; i < WORDS; ++i) iw[i] = __builtin_amdgcn_readfirstlane(job[i]);
    const bool wlds = solve_lds_bytes(I.k, true) <= lds_avail;
    if (wlds) solve_range<true>(I, 0, I.n, lds, S);
    else solve_range<false>(I, 0, I.n, lds, S);
    __syncthreads();
    if (threadIdx.x == 0)
      __hip_atomic_store(&done[c % ring_size], c + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

}  // namespace

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
  return cus > 0 ? cus : 1;
}

hipError_t launch_service(ServiceCtl *ctl, const ServiceJob *ring, int32_t ring_size, int64_t *done,
                          ServiceDev *dev, int64_t idle_ticks, int workers, hipStream_t st) {
  const size_t lds = LDS_BUDGET;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&service_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  service_kernel<<<workers, NT, lds, st>>>(ctl, ring, ring_size, done, dev, (uint32_t)lds, idle_ticks);
  return hipGetLastError();
}

size_t batch_lds_bytes(const BatchItem *items_host, int32_t m) {
  size_t b = 0;
  for (int32_t i = 0; i < m; ++i) {
    const int k = items_host[i].inst.k;
    const size_t need = solve_lds_bytes(k, true) <= LDS_BUDGET ? solve_lds_bytes(k, true)
                                                                : solve_lds_bytes(k, false);
    b = need > b ? need : b;
  }
  return b;
}

hipError_t launch_solve_batch(const BatchItem *items_dev, int32_t m, int32_t *head, size_t lds_bytes,
                              int workers, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&solve_batch_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return e;
  solve_batch_kernel<<<workers, NT, lds_bytes, st>>>(items_dev, m, head, (uint32_t)lds_bytes);
  return hipGetLastError();
}

int batch_workers(size_t lds_bytes, int32_t m) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(&solve_batch_kernel),
                                                   NT, lds_bytes) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const int w = cus * per_cu;
  return m < w ? m : w;
}

hipError_t launch_solve(const InstView &I, int64_t r_begin, int64_t r_end, hipStream_t st) {
  if (r_end <= r_begin) return hipSuccess;
  const bool wlds = solve_lds_bytes(I.k, true) <= LDS_BUDGET;
  const size_t bytes = solve_lds_bytes(I.k, wlds);
  return wlds ? launch_solve_t<true>(I, r_begin, r_end, bytes, st)
              : launch_solve_t<false>(I, r_begin, r_end, bytes, st);
}

}  // namespace lbdd
