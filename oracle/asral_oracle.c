/*
 * asral_oracle.c -- plain, slow CPU reference of ASRAL (test infrastructure).
 *
 * THIS FILE IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg load it.  The product path (the HIP library
 * and its Python binding) never calls, links or imports anything here, and
 * this file shares no code, header or table with it.
 *
 * What it computes (paper: "Load Balanced Demand Distribution under Overload
 * Penalties", arXiv 2304.06543):
 *
 *   orc_setup            most suitable center of every unit and the MinDistance
 *                        processing order (Section 3.5, Algorithm 2 step 1).
 *   orc_best_transfers   the condensed allotment-subspace graph: for every
 *                        ordered pair of centers (u,v) the cheapest transfer of
 *                        a unit allotted to u over to v (Definition of Gamma(A),
 *                        Section 3.2), written out as the plain definition.
 *   orc_refine_search    the NegCycle / NegPath split graphs (Definitions of
 *                        NCyc and NPath, Sections 3.3-3.4) and the
 *                        Bellman-Ford shortest s*_out -> s*_in path on them.
 *   orc_solve            the ASRAL main loop (Algorithm 2) with Negative Cycle
 *                        Refinement (Algorithm 1) and Negative Path Refinement
 *                        (Appendix A), keeping Gamma in one min-heap per
 *                        ordered pair of centers ("BestTransHeap", Section 3.5).
 *   orc_solve_q          the same loop with a general penalty function per
 *                        center (Definition of the penalty function, Section
 *                        2), given as a table of the penalties of successive
 *                        units beyond capacity.
 *   orc_road_cm          the cost matrix from a road network: shortest-path
 *                        lengths from every center (Section 3.5, construction
 *                        of CM), by Dijkstra.
 *   orc_objective        the objective of Equation (1) with one constant
 *                        per-unit penalty per center.
 *
 * Readings where the paper leaves a choice (each is listed in the design notes):
 *   - vacancy of s_j is "load before adding d_i < capacity", computed from loads;
 *   - penalty q_s(j) is one constant per center for every unit beyond capacity
 *     (the paper's experiments) in orc_solve; orc_solve_q takes any
 *     non-decreasing q_s(j) as a table whose last value holds for every later j;
 *   - ties: most suitable center = smallest index among equal costs; the
 *     processing order sorts by (cheapest cost, unit id); the best transfer of a
 *     pair is the smallest transfer cost, then the smallest processing rank;
 *     Bellman-Ford runs in synchronous rounds, a label changes only on strict
 *     improvement and its predecessor is the smallest node index achieving it;
 *   - a refinement is applied only when its cost is strictly negative;
 *   - the penalty edge u -> s*_in costs (penalty the next unit at u would pay)
 *     - (penalty of the anchor's last unit beyond capacity): with a constant
 *     penalty (load[u] >= cap[u] ? pen[u] : 0) - pen[s*]; the path's penalty
 *     edge is added to the objective once;
 *   - the transfer cost sign follows the definition of Gamma (cost of moving dn
 *     from s_i to s_j is CM(dn,s_j) - CM(dn,s_i)).
 *
 * Best-transfer keys are packed as ((delta + 2^31) << 32) | rank, so that an
 * unsigned comparison orders by delta and then by rank; "no edge" is all ones.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_INVAL (-1)
#define ORC_E_NOMEM (-2)
#define ORC_E_NEGCYCLE (-5)

/* Built with -fopenmp (PARA = 1) the same code is the para-ASRAL-style CPU
 * baseline (Section 3.6): the per-heap updates of the Gamma data structure,
 * the split-graph construction and each Bellman-Ford round's targets run in
 * threads when k >= PARA_MIN_K.  Every threaded loop writes disjoint data and
 * reads only what the loop does not write, so both builds give identical
 * results.  The plain build (no -fopenmp) ignores the pragmas.              */
#ifdef _OPENMP
#define PARA 1
#else
#define PARA 0
#endif
#define PARA_MIN_K 64

#define KEY_NONE UINT64_MAX
#define DIST_NONE INT64_MAX
#define CM_LIMIT (1 << 30)

/* trace row layout (one row of ORC_TRACE_W int64 per iteration) */
#define ORC_TRACE_W 8
/* [0] vacant  [1] cycle cost applied (0 if none)  [2] cycle length (edges)
 * [3] path cost applied (0 if none, includes the penalty edge)
 * [4] path length (edges incl. penalty edge)  [5] cycle BF rounds
 * [6] path BF rounds (0 if not run)  [7] objective after the iteration */

/* stats layout */
#define ORC_STATS_N 8
/* [0] cycles applied [1] paths applied [2] units moved [3] cycle searches
 * [4] path searches [5] BF rounds total [6] heap entries pushed
 * [7] iterations run */

static inline uint64_t pack_key(int64_t delta, int64_t rank) {
    return ((uint64_t)(uint32_t)(delta + 2147483648LL) << 32) | (uint64_t)(uint32_t)rank;
}
static inline int64_t key_delta(uint64_t key) {
    return (int64_t)(key >> 32) - 2147483648LL;
}
static inline int64_t key_rank(uint64_t key) { return (int64_t)(key & 0xffffffffu); }

/* Penalty function of every center (Definition of the penalty function,
 * Section 2): the j-th unit (j >= 1) beyond the capacity of center s pays
 * val[off[s] + min(j, len_s) - 1], len_s = off[s+1] - off[s] >= 1, so the
 * last value of a center's table holds for every later unit.  A constant
 * penalty per center is a table of one value per center.                    */
typedef struct { const int64_t *off; const int32_t *val; } pen_table;

static int64_t q_at(const pen_table *P, int32_t s, int64_t j) {
    const int64_t len = P->off[s + 1] - P->off[s];
    return P->val[P->off[s] + (j < len ? j : len) - 1];
}
/* what the next unit allotted to u pays on top of its cost (0 while u has room) */
static int64_t q_next(const pen_table *P, const int32_t *load, const int32_t *cap, int32_t u) {
    return load[u] >= cap[u] ? q_at(P, u, (int64_t)load[u] - cap[u] + 1) : 0;
}
/* what the last unit beyond the anchor's capacity pays.  The anchor is
 * overloaded whenever a path search runs in the solve; a standalone search on
 * an anchor within capacity takes the first unit's penalty (with a constant
 * penalty: pen[s*] in every case).                                           */
static int64_t q_last(const pen_table *P, const int32_t *load, const int32_t *cap, int32_t u) {
    return q_at(P, u, load[u] > cap[u] ? (int64_t)load[u] - cap[u] : 1);
}

/* A table of one value per center holding pen[]; off has k + 1 entries.     */
static void flat_table(int32_t k, const int32_t *pen, int64_t *off, pen_table *P) {
    for (int32_t s = 0; s <= k; ++s) off[s] = s;
    P->off = off;
    P->val = pen;
}

/* ------------------------------------------------------------------------ */
/* Input validation: k >= 1, n >= 1, 0 <= CM < 2^30, cap >= 0, pen >= 1.     */
static int validate(int32_t k, int64_t n, const int32_t *cm, const int32_t *cap,
                    const int32_t *pen) {
    if (k < 1 || n < 1 || n >= 0xffffffffLL || !cm) return ORC_E_INVAL;
    for (int64_t i = 0; i < n * (int64_t)k; ++i)
        if (cm[i] < 0 || cm[i] >= CM_LIMIT) return ORC_E_INVAL;
    if (cap)
        for (int32_t s = 0; s < k; ++s) if (cap[s] < 0) return ORC_E_INVAL;
    if (pen)
        for (int32_t s = 0; s < k; ++s) if (pen[s] < 1 || pen[s] >= CM_LIMIT) return ORC_E_INVAL;
    return ORC_OK;
}

/* Penalty tables: off[0] = 0, at least one value per center, every value in
 * [1, 2^30), non-decreasing within a center (the definition asks for an
 * increasing function; equal successive values keep the constant penalty of
 * the experiments inside the family).                                        */
static int validate_table(int32_t k, const int64_t *off, const int32_t *val) {
    if (!off || !val || off[0] != 0) return ORC_E_INVAL;
    for (int32_t s = 0; s < k; ++s) {
        if (off[s + 1] <= off[s]) return ORC_E_INVAL;
        for (int64_t i = off[s]; i < off[s + 1]; ++i) {
            if (val[i] < 1 || val[i] >= CM_LIMIT) return ORC_E_INVAL;
            if (i > off[s] && val[i] < val[i - 1]) return ORC_E_INVAL;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Setup: "most suitable" center and MinDistance order (Algorithm 2, step 1).
 * smin[d] = smallest s minimising CM(d,s); mc[d] = CM(d, smin[d]);
 * order[r] = r-th unit by (mc, d) ascending; rank[order[r]] = r.            */
typedef struct { int32_t mc; int64_t d; } mc_item;

static int cmp_mc_item(const void *a, const void *b) {
    const mc_item *x = (const mc_item *)a, *y = (const mc_item *)b;
    if (x->mc != y->mc) return x->mc < y->mc ? -1 : 1;
    return (x->d > y->d) - (x->d < y->d);
}

int orc_setup(int32_t k, int64_t n, const int32_t *cm, int32_t *smin, int32_t *mc,
              int64_t *order, int64_t *rank) {
    int rc = validate(k, n, cm, NULL, NULL);
    if (rc) return rc;
    mc_item *items = (mc_item *)malloc(sizeof(mc_item) * (size_t)n);
    if (!items) return ORC_E_NOMEM;
    for (int64_t d = 0; d < n; ++d) {
        const int32_t *row = cm + d * (int64_t)k;
        int32_t best = 0;
        for (int32_t s = 1; s < k; ++s)
            if (row[s] < row[best]) best = s;
        smin[d] = best;
        mc[d] = row[best];
        items[d].mc = row[best];
        items[d].d = d;
    }
    qsort(items, (size_t)n, sizeof(mc_item), cmp_mc_item);
    for (int64_t r = 0; r < n; ++r) {
        order[r] = items[r].d;
        rank[items[r].d] = r;
    }
    free(items);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Condensed Gamma(A) by its definition: for u != v,
 *   W[u][v] = min over units d with a(d) = u of key(CM(d,v) - CM(d,u), rank(d));
 * W[u][u] and pairs with no unit at u are KEY_NONE.  assign[d] < 0 means d is
 * not yet allotted.                                                          */
int orc_best_transfers(int32_t k, int64_t n, const int32_t *cm, const int32_t *assign,
                       const int64_t *rank, uint64_t *W) {
    if (k < 1 || n < 0) return ORC_E_INVAL;
    for (int64_t i = 0; i < (int64_t)k * k; ++i) W[i] = KEY_NONE;
    for (int64_t d = 0; d < n; ++d) {
        int32_t u = assign[d];
        if (u < 0) continue;
        if (u >= k) return ORC_E_INVAL;
        const int32_t *row = cm + d * (int64_t)k;
        for (int32_t v = 0; v < k; ++v) {
            if (v == u) continue;
            uint64_t key = pack_key((int64_t)row[v] - row[u], rank[d]);
            if (key < W[(int64_t)u * k + v]) W[(int64_t)u * k + v] = key;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Objective, Equation (1): sum of CM over the allotment plus, for every center,
 * pen[s] times the number of units beyond its capacity.                      */
int orc_objective(int32_t k, int64_t n, const int32_t *cm, const int32_t *cap,
                  const int32_t *pen, const int32_t *assign, int64_t *out) {
    int64_t *load = (int64_t *)calloc((size_t)k, sizeof(int64_t));
    if (!load) return ORC_E_NOMEM;
    int64_t total = 0;
    for (int64_t d = 0; d < n; ++d) {
        int32_t s = assign[d];
        if (s < 0) continue;
        if (s >= k) { free(load); return ORC_E_INVAL; }
        total += cm[d * (int64_t)k + s];
        load[s] += 1;
    }
    for (int32_t s = 0; s < k; ++s)
        if (load[s] > cap[s]) total += (int64_t)pen[s] * (load[s] - cap[s]);
    free(load);
    *out = total;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Split graphs and Bellman-Ford.
 * Nodes 0..k-1 are the centers, with the anchor's node standing for s*_out;
 * node k is s*_in.  weights is (k+1) x (k+1), has_edge marks existing edges.
 *
 * NCyc (Definition in Section 3.3):
 *   u -> v  (u, v not the anchor, u != v):  W[u][v]
 *   s*_out -> v:                            W[s*][v]
 *   u -> s*_in:                             W[u][s*]
 * NPath (Definition in Section 3.4): as NCyc, but every edge into s*_in is the
 *   penalty difference q_u() - q_s*(): q_u() is what one more unit at u would
 *   pay (0 while u has room), q_s*() what the anchor's last unit beyond its
 *   capacity pays (the anchor is overloaded whenever this graph is built).
 * Pairs with no unit to transfer have no edge; there are no self loops, no
 * edges into s*_out and none out of s*_in.                                    */
static void build_split_graph(int32_t k, const uint64_t *W, int32_t anchor, int mode,
                              const int32_t *load, const int32_t *cap, const pen_table *P,
                              int64_t *wt, uint8_t *has) {
    const int32_t K1 = k + 1;
    memset(has, 0, (size_t)K1 * K1);
    #pragma omp parallel for schedule(static) if(PARA && k >= PARA_MIN_K)
    for (int32_t u = 0; u < k; ++u) {
        for (int32_t v = 0; v < k; ++v) {
            if (u == v || v == anchor) continue;       /* nothing enters s*_out */
            uint64_t key = W[(int64_t)u * k + v];
            if (key == KEY_NONE) continue;
            wt[(int64_t)u * K1 + v] = key_delta(key);
            has[(int64_t)u * K1 + v] = 1;
        }
        if (u == anchor) continue;                     /* no s*_out -> s*_in */
        if (mode == 0) {
            uint64_t key = W[(int64_t)u * k + anchor];
            if (key != KEY_NONE) {
                wt[(int64_t)u * K1 + k] = key_delta(key);
                has[(int64_t)u * K1 + k] = 1;
            }
        } else {
            wt[(int64_t)u * K1 + k] = q_next(P, load, cap, u) - q_last(P, load, cap, anchor);
            has[(int64_t)u * K1 + k] = 1;
        }
    }
}

/* Bellman-Ford in synchronous rounds from src over nodes 0..K1-1.
 * Round t: cand(v) = min over u of dist_{t-1}[u] + w(u,v), scanning u in
 * increasing order so the first (smallest) u attaining the minimum is kept;
 * dist and pred change only when cand(v) < dist_{t-1}[v].  Stops after the
 * first round without a change.  With K1 nodes a change in round K1 means a
 * negative cycle is reachable.                                                */
static int bellman_ford(int32_t K1, int32_t src, const int64_t *wt, const uint8_t *has,
                        int64_t *dist, int32_t *pred, int64_t *scratch, int32_t *rounds) {
    for (int32_t v = 0; v < K1; ++v) { dist[v] = DIST_NONE; pred[v] = -1; }
    dist[src] = 0;
    for (int32_t t = 1; t <= K1; ++t) {
        int changed = 0;
        /* each target's candidate reads only the previous round's labels */
        #pragma omp parallel for schedule(static) reduction(|:changed) if(PARA && K1 > PARA_MIN_K)
        for (int32_t v = 0; v < K1; ++v) {
            int64_t cand = DIST_NONE;
            int32_t arg = -1;
            for (int32_t u = 0; u < K1; ++u) {
                if (dist[u] == DIST_NONE || !has[(int64_t)u * K1 + v]) continue;
                int64_t c = dist[u] + wt[(int64_t)u * K1 + v];
                if (c < cand) { cand = c; arg = u; }
            }
            if (cand < dist[v]) { scratch[v] = cand; pred[v] = arg; changed = 1; }
            else scratch[v] = dist[v];
        }
        memcpy(dist, scratch, sizeof(int64_t) * (size_t)K1);
        if (!changed) { *rounds = t; return ORC_OK; }
    }
    *rounds = K1;
    return ORC_E_NEGCYCLE;
}

/* Search entry used by tests: builds the split graph for (W, anchor, mode) and
 * returns dist/pred over the k+1 nodes and the number of rounds.  The penalty
 * is a table (orc_refine_search_q) or one constant per center.                */
int orc_refine_search_q(int32_t k, const uint64_t *W, int32_t anchor, int32_t mode,
                        const int32_t *load, const int32_t *cap, const int64_t *pen_off,
                        const int32_t *pen_val, int64_t *dist, int32_t *pred, int32_t *rounds) {
    if (k < 1 || anchor < 0 || anchor >= k) return ORC_E_INVAL;
    if (validate_table(k, pen_off, pen_val)) return ORC_E_INVAL;
    const pen_table P = {pen_off, pen_val};
    const int32_t K1 = k + 1;
    int64_t *wt = (int64_t *)malloc(sizeof(int64_t) * (size_t)K1 * K1);
    uint8_t *has = (uint8_t *)malloc((size_t)K1 * K1);
    int64_t *scratch = (int64_t *)malloc(sizeof(int64_t) * (size_t)K1);
    int rc = ORC_E_NOMEM;
    if (wt && has && scratch) {
        build_split_graph(k, W, anchor, mode, load, cap, &P, wt, has);
        rc = bellman_ford(K1, anchor, wt, has, dist, pred, scratch, rounds);
    }
    free(wt); free(has); free(scratch);
    return rc;
}

int orc_refine_search(int32_t k, const uint64_t *W, int32_t anchor, int32_t mode,
                      const int32_t *load, const int32_t *cap, const int32_t *pen,
                      int64_t *dist, int32_t *pred, int32_t *rounds) {
    if (k < 1 || !pen) return ORC_E_INVAL;
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)k + 1));
    if (!off) return ORC_E_NOMEM;
    pen_table P;
    flat_table(k, pen, off, &P);
    int rc = orc_refine_search_q(k, W, anchor, mode, load, cap, off, pen, dist, pred, rounds);
    free(off);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* BestTransHeap: binary min-heap of packed keys for one ordered pair (u,v).
 * Entries are never removed when a unit leaves u; a top whose unit is no
 * longer allotted to u is discarded when it is looked at.                    */
typedef struct { uint64_t *a; int64_t size, cap; } heap_t;

static int heap_push(heap_t *h, uint64_t key) {
    if (h->size == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 8;
        uint64_t *na = (uint64_t *)realloc(h->a, sizeof(uint64_t) * (size_t)nc);
        if (!na) return ORC_E_NOMEM;
        h->a = na; h->cap = nc;
    }
    int64_t i = h->size++;
    h->a[i] = key;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h->a[p] <= h->a[i]) break;
        uint64_t t = h->a[p]; h->a[p] = h->a[i]; h->a[i] = t;
        i = p;
    }
    return ORC_OK;
}

static void heap_pop(heap_t *h) {
    h->a[0] = h->a[--h->size];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->size && h->a[l] < h->a[m]) m = l;
        if (r < h->size && h->a[r] < h->a[m]) m = r;
        if (m == i) break;
        uint64_t t = h->a[m]; h->a[m] = h->a[i]; h->a[i] = t;
        i = m;
    }
}

typedef struct {
    int32_t k;
    int64_t n;
    const int32_t *cm, *cap;
    pen_table P;            /* penalty function of every center */
    int32_t *smin, *mc, *a, *load;
    int64_t *order, *rank;
    heap_t *H;              /* k*k heaps; H[u*k+v] */
    uint64_t *W;            /* condensed view rebuilt from the heap tops */
    int64_t *wt, *dist, *scratch;
    uint8_t *has;
    int32_t *pred;
    int64_t stats[ORC_STATS_N];
    int strict;             /* strict-LBDD: dummy units fill every free slot */
} orc_state;

/* top of BestTransHeap(u,v), discarding entries whose unit has left u */
static uint64_t heap_top(orc_state *S, int32_t u, int32_t v) {
    heap_t *h = &S->H[(int64_t)u * S->k + v];
    while (h->size > 0) {
        uint64_t key = h->a[0];
        int64_t d = S->order[key_rank(key)];
        if (S->a[d] == u) return key;
        heap_pop(h);
    }
    return KEY_NONE;
}

/* unit d has just been placed at center u: add its k-1 transfer edges */
static int heaps_insert_unit(orc_state *S, int64_t d, int32_t u) {
    const int32_t *row = S->cm + d * (int64_t)S->k;
    int rc = ORC_OK;
    /* the k-1 heaps are distinct: the para-ASRAL build updates them in
     * threads (Section 3.6, updating the Gamma data structure in parallel) */
    #pragma omp parallel for schedule(static) reduction(|:rc) if(PARA && S->k >= PARA_MIN_K)
    for (int32_t v = 0; v < S->k; ++v) {
        if (v == u) continue;
        rc |= heap_push(&S->H[(int64_t)u * S->k + v], pack_key((int64_t)row[v] - row[u], S->rank[d]));
    }
    S->stats[6] += S->k - 1;
    return rc ? ORC_E_NOMEM : ORC_OK;
}

/* Key of moving one of the zero-cost dummy units of strict-LBDD (Appendix B)
 * out of a center with free capacity: transfer cost 0, ordered after every
 * real unit's key of equal cost (the rank field is beyond any real rank).  */
#define DUMMY_KEY (((uint64_t)1u << 63) | 0xFFFFFFFEu)

static void refresh_W(orc_state *S) {
    /* rows touch disjoint heaps (lazy deletion pops only H[u][.]) */
    #pragma omp parallel for schedule(static) if(PARA && S->k >= PARA_MIN_K)
    for (int32_t u = 0; u < S->k; ++u)
        for (int32_t v = 0; v < S->k; ++v) {
            uint64_t key = (u == v) ? KEY_NONE : heap_top(S, u, v);
            if (S->strict && u != v && S->load[u] < S->cap[u] && DUMMY_KEY < key) key = DUMMY_KEY;
            S->W[(int64_t)u * S->k + v] = key;
        }
}

/* One refinement (Algorithm 1 for mode 0, Appendix A for mode 1) with anchor s.
 * Returns the applied cost (< 0) in *applied, 0 if nothing was applied.      */
static int refine(orc_state *S, int32_t s, int mode, int64_t *applied, int64_t *edges,
                  int32_t *rounds) {
    const int32_t k = S->k, K1 = k + 1;
    *applied = 0; *edges = 0;
    refresh_W(S);
    build_split_graph(k, S->W, s, mode, S->load, S->cap, &S->P, S->wt, S->has);
    int rc = bellman_ford(K1, s, S->wt, S->has, S->dist, S->pred, S->scratch, rounds);
    S->stats[5] += *rounds;
    if (rc) return rc;
    if (S->dist[k] == DIST_NONE || S->dist[k] >= 0) return ORC_OK;
    /* walk the path back from s*_in; nodes are collected in reverse */
    int32_t *path = (int32_t *)malloc(sizeof(int32_t) * (size_t)(K1 + 1));
    if (!path) return ORC_E_NOMEM;
    int32_t len = 0;
    for (int32_t v = k; v != -1; v = S->pred[v]) {
        if (len > K1) { free(path); return ORC_E_NEGCYCLE; }
        path[len++] = v;
    }
    if (path[len - 1] != s) { free(path); return ORC_E_NEGCYCLE; }
    /* transfer edges: all edges for a cycle; all but the final penalty edge
     * for a path.  The moved units are read from Gamma before any move.     */
    int32_t nedges = len - 1;
    int32_t ntransfer = (mode == 0) ? nedges : nedges - 1;
    int64_t *units = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ntransfer > 0 ? ntransfer : 1));
    int32_t *from = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ntransfer > 0 ? ntransfer : 1));
    int32_t *to = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ntransfer > 0 ? ntransfer : 1));
    if (!units || !from || !to) { free(path); free(units); free(from); free(to); return ORC_E_NOMEM; }
    for (int32_t e = 0; e < ntransfer; ++e) {
        int32_t u = path[len - 1 - e];
        int32_t v = path[len - 2 - e];
        if (v == k) v = s;                      /* s*_in is the anchor itself */
        uint64_t key = S->W[(int64_t)u * k + v];
        units[e] = key == DUMMY_KEY ? -1 : S->order[key_rank(key)];   /* -1: a dummy unit */
        from[e] = u; to[e] = v;
    }
    for (int32_t e = 0; e < ntransfer; ++e) {
        if (units[e] < 0) continue;             /* a dummy moves: no real unit does */
        S->a[units[e]] = to[e];
        S->load[from[e]] -= 1;
        S->load[to[e]] += 1;
        S->stats[2]++;
    }
    int rc2 = ORC_OK;
    for (int32_t e = 0; e < ntransfer && !rc2; ++e)
        if (units[e] >= 0) rc2 = heaps_insert_unit(S, units[e], to[e]);
    *applied = S->dist[k];
    *edges = nedges;
    free(path); free(units); free(from); free(to);
    return rc2;
}

static void state_free(orc_state *S) {
    if (S->H) {
        for (int64_t i = 0; i < (int64_t)S->k * S->k; ++i) free(S->H[i].a);
        free(S->H);
    }
    free(S->smin); free(S->mc); free(S->a); free(S->load); free(S->order); free(S->rank);
    free(S->W); free(S->wt); free(S->dist); free(S->scratch); free(S->has); free(S->pred);
}

/* ASRAL (Algorithm 2) with the penalty function P, on validated inputs.
 * Runs iterations 0 .. min(n, max_iters)-1.  Outputs: assign[n] (center per
 * unit id, -1 if not yet allotted), load[k], objective, optionally W (k*k,
 * the heap tops after the last iteration), trace (ORC_TRACE_W int64 per
 * iteration) and stats (ORC_STATS_N int64).                                  */
static int solve_core(int32_t k, int64_t n, const int32_t *cm, const int32_t *cap,
                      const pen_table *P, int64_t max_iters, int32_t *assign, int32_t *load_out,
                      int64_t *objective, uint64_t *W_out, int64_t *trace, int64_t *stats) {
    int rc = ORC_OK;
    orc_state S;
    memset(&S, 0, sizeof(S));
    S.k = k; S.n = n; S.cm = cm; S.cap = cap; S.P = *P;
    const int32_t K1 = k + 1;
    S.smin = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    S.mc = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    S.a = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    S.load = (int32_t *)calloc((size_t)k, sizeof(int32_t));
    S.order = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    S.rank = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    S.H = (heap_t *)calloc((size_t)k * k, sizeof(heap_t));
    S.W = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)k * k);
    S.wt = (int64_t *)malloc(sizeof(int64_t) * (size_t)K1 * K1);
    S.has = (uint8_t *)malloc((size_t)K1 * K1);
    S.dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)K1);
    S.scratch = (int64_t *)malloc(sizeof(int64_t) * (size_t)K1);
    S.pred = (int32_t *)malloc(sizeof(int32_t) * (size_t)K1);
    if (!S.smin || !S.mc || !S.a || !S.load || !S.order || !S.rank || !S.H || !S.W ||
        !S.wt || !S.has || !S.dist || !S.scratch || !S.pred) {
        state_free(&S);
        return ORC_E_NOMEM;
    }
    rc = orc_setup(k, n, cm, S.smin, S.mc, S.order, S.rank);
    if (rc) { state_free(&S); return rc; }
    for (int64_t d = 0; d < n; ++d) S.a[d] = -1;

    int64_t delta = 0;                       /* the paper's Delta */
    int64_t iters = (max_iters < 0 || max_iters > n) ? n : max_iters;
    for (int64_t r = 0; r < iters && !rc; ++r) {
        int64_t d = S.order[r];              /* extract-min on MinDistance */
        int32_t s = S.smin[d];
        int vacant = S.load[s] < cap[s];
        /* Case (b): the unit is the (load - cap + 1)-th beyond capacity */
        int64_t q = q_next(&S.P, S.load, cap, s);
        S.a[d] = s;
        S.load[s] += 1;
        delta += (int64_t)cm[d * (int64_t)k + s] + q;
        rc = heaps_insert_unit(&S, d, s);
        if (rc) break;

        int64_t cyc_cost = 0, cyc_len = 0, path_cost = 0, path_len = 0;
        int32_t cyc_rounds = 0, path_rounds = 0;
        S.stats[3]++;
        rc = refine(&S, s, 0, &cyc_cost, &cyc_len, &cyc_rounds);
        if (rc) break;
        if (cyc_cost < 0) { delta += cyc_cost; S.stats[0]++; }
        if (!vacant) {
            S.stats[4]++;
            rc = refine(&S, s, 1, &path_cost, &path_len, &path_rounds);
            if (rc) break;
            if (path_cost < 0) { delta += path_cost; S.stats[1]++; }
        }
        if (trace) {
            int64_t *t = trace + r * ORC_TRACE_W;
            t[0] = vacant; t[1] = cyc_cost; t[2] = cyc_len; t[3] = path_cost;
            t[4] = path_len; t[5] = cyc_rounds; t[6] = path_rounds; t[7] = delta;
        }
        S.stats[7] = r + 1;
    }
    if (!rc) {
        memcpy(assign, S.a, sizeof(int32_t) * (size_t)n);
        if (load_out) memcpy(load_out, S.load, sizeof(int32_t) * (size_t)k);
        *objective = delta;
        if (W_out) { refresh_W(&S); memcpy(W_out, S.W, sizeof(uint64_t) * (size_t)k * k); }
        if (stats) memcpy(stats, S.stats, sizeof(S.stats));
    }
    state_free(&S);
    return rc;
}

/* ASRAL with one constant per-unit penalty per center, pen[k].               */
int orc_solve(int32_t k, int64_t n, const int32_t *cm, const int32_t *cap,
              const int32_t *pen, int64_t max_iters, int32_t *assign, int32_t *load_out,
              int64_t *objective, uint64_t *W_out, int64_t *trace, int64_t *stats) {
    int rc = validate(k, n, cm, cap, pen);
    if (rc) return rc;
    if (!cap || !pen || !assign || !objective) return ORC_E_INVAL;
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)k + 1));
    if (!off) return ORC_E_NOMEM;
    pen_table P;
    flat_table(k, pen, off, &P);
    rc = solve_core(k, n, cm, cap, &P, max_iters, assign, load_out, objective, W_out, trace, stats);
    free(off);
    return rc;
}

/* ASRAL with a penalty table per center: the j-th unit beyond the capacity
 * of s pays pen_val[pen_off[s] + min(j, len_s) - 1] (see pen_table).         */
int orc_solve_q(int32_t k, int64_t n, const int32_t *cm, const int32_t *cap,
                const int64_t *pen_off, const int32_t *pen_val, int64_t max_iters,
                int32_t *assign, int32_t *load_out, int64_t *objective, uint64_t *W_out,
                int64_t *trace, int64_t *stats) {
    int rc = validate(k, n, cm, cap, NULL);
    if (rc) return rc;
    if (!cap || !assign || !objective || validate_table(k, pen_off, pen_val)) return ORC_E_INVAL;
    const pen_table P = {pen_off, pen_val};
    return solve_core(k, n, cm, cap, &P, max_iters, assign, load_out, objective, W_out, trace, stats);
}

/* ------------------------------------------------------------------------ */
/* Strict-LBDD (Appendix B): no center may hold more units than its
 * capacity, and the objective is Equation (3), the plain allotment cost.
 *   Pre-processing: if the total capacity is below n, a dummy center with
 *   index k, capacity n - sum(cap) and cost max(CM) + 1 for every unit is
 *   added (it changes every complete allotment's cost by the same amount).
 *   Every center's free capacity is held by zero-cost dummy units, so Gamma
 *   has a zero-cost transfer u -> v for every v while u has free capacity.
 *   Algorithm 4: each unit, in the MinDistance order of ASRAL, goes to the
 *   cheapest center that still has free capacity (smallest index among equal
 *   costs) and Negative Cycle Refinement (Algorithm 1) runs anchored there.
 * Theorem 2: the result is an optimal allotment.
 * Readings: the processing order is ASRAL's; a dummy transfer's key follows
 * every real key of equal cost; applying a dummy transfer moves no real unit.
 * Outputs: assign[n] (-1 for units left at the dummy center), load_out[kx]
 * (kx = k or k + 1 with the dummy center, which *kx_out reports), objective
 * = sum of CM over the allotted units, W_out[kx][kx] (dummy edges included),
 * stats as orc_solve.                                                         */
int orc_solve_strict(int32_t k, int64_t n, const int32_t *cm, const int32_t *cap,
                     int64_t max_iters, int32_t *assign, int32_t *load_out, int32_t *kx_out,
                     int64_t *objective, uint64_t *W_out, int64_t *stats) {
    if (k < 1 || n < 1 || !cm || !cap || !assign || !objective || !kx_out) return ORC_E_INVAL;
    int64_t total = 0;
    int32_t maxcm = 0;
    for (int32_t s = 0; s < k; ++s) {
        if (cap[s] < 0) return ORC_E_INVAL;
        total += cap[s];
    }
    for (int64_t i = 0; i < n * (int64_t)k; ++i) {
        if (cm[i] < 0 || cm[i] >= CM_LIMIT) return ORC_E_INVAL;
        if (cm[i] > maxcm) maxcm = cm[i];
    }
    const int32_t kx = total < n ? k + 1 : k;
    int32_t *cmx = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * kx);
    int32_t *capx = (int32_t *)malloc(sizeof(int32_t) * (size_t)kx);
    int32_t *pen1 = (int32_t *)malloc(sizeof(int32_t) * (size_t)kx);
    if (!cmx || !capx || !pen1) { free(cmx); free(capx); free(pen1); return ORC_E_NOMEM; }
    for (int64_t d = 0; d < n; ++d) {
        memcpy(cmx + d * kx, cm + d * (int64_t)k, sizeof(int32_t) * (size_t)k);
        if (kx > k) cmx[d * kx + k] = maxcm + 1;
    }
    for (int32_t s = 0; s < k; ++s) capx[s] = cap[s];
    if (kx > k) capx[k] = (int32_t)(n - total);
    for (int32_t s = 0; s < kx; ++s) pen1[s] = 1;        /* no penalties in strict-LBDD */

    orc_state S;
    memset(&S, 0, sizeof(S));
    int64_t *off1 = (int64_t *)malloc(sizeof(int64_t) * ((size_t)kx + 1));
    if (!off1) { free(cmx); free(capx); free(pen1); return ORC_E_NOMEM; }
    S.k = kx; S.n = n; S.cm = cmx; S.cap = capx; S.strict = 1;
    flat_table(kx, pen1, off1, &S.P);
    const int32_t K1 = kx + 1;
    S.smin = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    S.mc = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    S.a = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    S.load = (int32_t *)calloc((size_t)kx, sizeof(int32_t));
    S.order = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    S.rank = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    S.H = (heap_t *)calloc((size_t)kx * kx, sizeof(heap_t));
    S.W = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)kx * kx);
    S.wt = (int64_t *)malloc(sizeof(int64_t) * (size_t)K1 * K1);
    S.has = (uint8_t *)malloc((size_t)K1 * K1);
    S.dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)K1);
    S.scratch = (int64_t *)malloc(sizeof(int64_t) * (size_t)K1);
    S.pred = (int32_t *)malloc(sizeof(int32_t) * (size_t)K1);
    int rc = ORC_OK;
    if (!S.smin || !S.mc || !S.a || !S.load || !S.order || !S.rank || !S.H || !S.W ||
        !S.wt || !S.has || !S.dist || !S.scratch || !S.pred)
        rc = ORC_E_NOMEM;
    if (!rc) rc = orc_setup(kx, n, cmx, S.smin, S.mc, S.order, S.rank);
    int64_t delta = 0;
    if (!rc) {
        for (int64_t d = 0; d < n; ++d) S.a[d] = -1;
        int64_t iters = (max_iters < 0 || max_iters > n) ? n : max_iters;
        for (int64_t r = 0; r < iters && !rc; ++r) {
            int64_t d = S.order[r];
            const int32_t *row = cmx + d * kx;
            int32_t s = -1;                          /* cheapest center with free capacity */
            for (int32_t t = 0; t < kx; ++t)
                if (S.load[t] < capx[t] && (s < 0 || row[t] < row[s])) s = t;
            S.a[d] = s;
            S.load[s] += 1;
            delta += row[s];
            rc = heaps_insert_unit(&S, d, s);
            if (rc) break;
            int64_t gain = 0, len = 0;
            int32_t rounds = 0;
            S.stats[3]++;
            rc = refine(&S, s, 0, &gain, &len, &rounds);
            if (rc) break;
            if (gain < 0) { delta += gain; S.stats[0]++; }
            S.stats[7] = r + 1;
        }
    }
    if (!rc) {
        int64_t at_dummy = 0;
        for (int64_t d = 0; d < n; ++d) {
            int32_t c = S.a[d];
            if (kx > k && c == k) { ++at_dummy; c = -1; }
            assign[d] = c;
        }
        *objective = delta - at_dummy * ((int64_t)maxcm + 1);
        *kx_out = kx;
        if (load_out) memcpy(load_out, S.load, sizeof(int32_t) * (size_t)kx);
        if (W_out) { refresh_W(&S); memcpy(W_out, S.W, sizeof(uint64_t) * (size_t)kx * kx); }
        if (stats) memcpy(stats, S.stats, sizeof(S.stats));
    }
    state_free(&S);
    free(cmx); free(capx); free(pen1); free(off1);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Cost matrix from a road network (construction of CM, Section 3.5; Datasets,
 * Section 5): CM(d, s) is the length of a shortest path from the vertex of
 * center s to the vertex of unit d.  Dijkstra from every center with a binary
 * min-heap of (distance, vertex) pairs and lazy deletion (a popped pair whose
 * distance is above the vertex's label is stale and skipped).
 *   graph     CSR over V vertices: arcs row_ptr[u] .. row_ptr[u+1]-1 leave u,
 *             arc i goes to col[i] with length len[i] >= 0 (a two-way road is
 *             two arcs)
 *   centers   [k] vertex of each center; units [n] vertex of each unit
 *   cm        [n][k] output
 * Fails with ORC_E_INVAL on bad indices or lengths, and when some unit's
 * vertex cannot be reached from some center or lies 2^30 or more away.      */
typedef struct { int64_t d; int32_t v; } dv_pair;

static int dv_less(dv_pair a, dv_pair b) { return a.d < b.d || (a.d == b.d && a.v < b.v); }

static void dv_push(dv_pair *h, int64_t *size, dv_pair x) {
    int64_t i = (*size)++;
    h[i] = x;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!dv_less(h[i], h[p])) break;
        dv_pair t = h[p]; h[p] = h[i]; h[i] = t;
        i = p;
    }
}

static dv_pair dv_pop(dv_pair *h, int64_t *size) {
    dv_pair top = h[0];
    h[0] = h[--(*size)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < *size && dv_less(h[l], h[m])) m = l;
        if (r < *size && dv_less(h[r], h[m])) m = r;
        if (m == i) break;
        dv_pair t = h[m]; h[m] = h[i]; h[i] = t;
        i = m;
    }
    return top;
}

int orc_road_cm(int32_t V, const int64_t *row_ptr, const int32_t *col, const int32_t *len,
                int32_t k, const int32_t *centers, int64_t n, const int32_t *units, int32_t *cm) {
    if (V < 1 || k < 1 || n < 1 || !row_ptr || !col || !len || !centers || !units || !cm)
        return ORC_E_INVAL;
    if (row_ptr[0] != 0) return ORC_E_INVAL;
    for (int32_t u = 0; u < V; ++u)
        if (row_ptr[u + 1] < row_ptr[u]) return ORC_E_INVAL;
    const int64_t E = row_ptr[V];
    for (int64_t i = 0; i < E; ++i)
        if (col[i] < 0 || col[i] >= V || len[i] < 0 || len[i] >= CM_LIMIT) return ORC_E_INVAL;
    for (int32_t s = 0; s < k; ++s) if (centers[s] < 0 || centers[s] >= V) return ORC_E_INVAL;
    for (int64_t d = 0; d < n; ++d) if (units[d] < 0 || units[d] >= V) return ORC_E_INVAL;
    int64_t *dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)V);
    dv_pair *heap = (dv_pair *)malloc(sizeof(dv_pair) * (size_t)(E + 1));
    if (!dist || !heap) { free(dist); free(heap); return ORC_E_NOMEM; }
    int rc = ORC_OK;
    for (int32_t s = 0; s < k && !rc; ++s) {
        for (int32_t v = 0; v < V; ++v) dist[v] = DIST_NONE;
        int64_t size = 0;
        dist[centers[s]] = 0;
        dv_pair start = {0, centers[s]};
        dv_push(heap, &size, start);
        while (size > 0) {
            dv_pair x = dv_pop(heap, &size);
            if (x.d > dist[x.v]) continue;            /* stale entry */
            for (int64_t i = row_ptr[x.v]; i < row_ptr[x.v + 1]; ++i) {
                int64_t c = x.d + len[i];
                if (c < dist[col[i]]) {
                    dist[col[i]] = c;
                    dv_pair y = {c, col[i]};
                    dv_push(heap, &size, y);          /* at most one push per arc */
                }
            }
        }
        for (int64_t d = 0; d < n; ++d) {
            int64_t c = dist[units[d]];
            if (c == DIST_NONE || c >= CM_LIMIT) { rc = ORC_E_INVAL; break; }
            cm[d * (int64_t)k + s] = (int32_t)c;
        }
    }
    free(dist); free(heap);
    return rc;
}
