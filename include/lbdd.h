/*
 * lbdd.h -- C ABI of the MI355X (gfx950) ASRAL solver for Load Balanced Demand
 * Distribution under overload penalties (arXiv 2304.06543).
 *
 * Problem (Section 2.1, the problem statement): given k service centers S, n
 * demand units D, an integer cost matrix CM(d,s), a capacity c_s and a
 * penalty for every unit a center takes beyond its capacity, find a complete
 * allotment (every unit to exactly one center) with a small value of the
 * objective of Equation (1): the sum of CM over the allotment plus the total
 * overload penalty.  The solver runs ASRAL (Algorithm 2): units are allotted
 * one at a time in ascending order of their cheapest cost, each allotment is
 * followed by Negative Cycle Refinement (Algorithm 1) and, when the receiving
 * center was already full, by Negative Path Refinement (Appendix A).
 *
 * Conventions for every function:
 *   - Return LBDD_OK (0) or a negative LBDD_E_* code; nothing aborts.  The
 *     calling thread's last failure is described by lbdd_last_error().
 *   - All integers are host-endian.  CM is int32, row-major [n][k]:
 *     CM(d_i, s_j) = cm[i * k + j], with 0 <= CM < 2^30.
 *   - Capacities are int32 >= 0; penalties are int32 in [1, 2^30): the penalty
 *     is one constant per center, charged for every unit beyond capacity
 *     (the paper's experiments, Section 5; Definition of the penalty function
 *     in Section 2 allows a monotone function, of which this is a special case).
 *   - The objective is int64.
 *   - Work is enqueued on the instance's HIP stream (hipStream_t passed as
 *     void*; NULL means the default stream).  Calls that return results
 *     synchronise with that stream.
 *   - A handle is not thread-safe; distinct handles are independent.
 *
 * Ties (the paper leaves them open; this library fixes them):
 *   - a unit's most suitable center is the smallest index among its cheapest;
 *   - units are processed by (cheapest cost, unit index) ascending;
 *   - the best transfer of a center pair is the smallest transfer cost, then
 *     the earliest-processed unit;
 *   - Bellman-Ford runs in synchronous rounds, labels change only on strict
 *     improvement, and a label's predecessor is the smallest node index that
 *     attains it; a refinement is applied only if its cost is < 0.
 */
#ifndef LBDD_H
#define LBDD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBDD_OK = 0,
    LBDD_E_INVAL = -1,    /* bad argument or input value out of range */
    LBDD_E_NOMEM = -2,    /* device or host allocation failed */
    LBDD_E_DEVICE = -3,   /* a HIP runtime call failed */
    LBDD_E_STATE = -4,    /* call not valid in the handle's current state */
    LBDD_E_INTERNAL = -5, /* an invariant failed (e.g. Bellman-Ford found a
                             negative cycle that Lemmas 1-2 rule out) */
    LBDD_E_CANCELLED = -6,/* a server job was cancelled before it started */
    LBDD_E_TIMEOUT = -7   /* a server job waited longer than the queue timeout */
};

#define LBDD_MAX_K 2048                /* centers per instance */
#define LBDD_MAX_N 0x7fffffffLL        /* units per instance */

/* lbdd_create flags */
#define LBDD_CM_DEVICE 0x1u   /* cm is a device pointer; it is read during
                                 lbdd_create only and never freed */
/* lbdd_assignment flags */
#define LBDD_OUT_DEVICE 0x1u  /* out is a device pointer */

typedef struct lbdd_instance lbdd_instance;

/* Create an instance and run the setup step of Algorithm 2 (step 1): each
 * unit's most suitable center and the MinDistance processing order.
 *   k, n        numbers of centers and units (1 <= k <= LBDD_MAX_K,
 *               1 <= n <= LBDD_MAX_N)
 *   cm          [n][k] int32 cost matrix, host memory unless LBDD_CM_DEVICE
 *   capacity    [k] int32 host array, copied
 *   penalty     [k] int32 host array, copied
 *   hip_stream  stream all of this instance's work is enqueued on
 *   out         receives the handle (owned by the caller; lbdd_destroy frees)
 * The library keeps its own device copy of CM, rows permuted into processing
 * order; the caller's buffer may be reused once this call returns.
 * Errors: LBDD_E_INVAL (ranges above, NULL pointers, any CM entry outside
 * [0, 2^30) -- checked on the device, so this call synchronises),
 * LBDD_E_NOMEM, LBDD_E_DEVICE. */
int lbdd_create(int32_t k, int64_t n, const int32_t *cm, const int32_t *capacity,
                const int32_t *penalty, uint32_t flags, void *hip_stream,
                lbdd_instance **out);

/* Create an instance whose penalty is a general function of the overload
 * (Definition of the penalty function, Section 2: the j-th unit beyond the
 * capacity of s pays q_s(j) > 0, non-decreasing in j), given as one table
 * per center: q_s(j) = pen_val[pen_off[s] + min(j, len_s) - 1] with
 * len_s = pen_off[s + 1] - pen_off[s] >= 1, so a table's last value holds for
 * every later unit (a table of one value is the constant penalty of
 * lbdd_create).  The objective is then Equation (2): CM over the allotment
 * plus, for every center, q_s(1) + ... + q_s(load - capacity).  The
 * allotment to a full center adds q_s(load - capacity + 1); the path search's
 * edge u -> s*_in costs what one more unit at u would pay minus what the
 * anchor's last unit beyond capacity pays.
 *   k, n, cm, capacity, flags, hip_stream, out   as lbdd_create
 *   pen_off     [k + 1] int64 host array, pen_off[0] = 0, strictly increasing
 *   pen_val     [pen_off[k]] int32 host array, values in [1, 2^30),
 *               non-decreasing within each center; both copied
 * Errors: as lbdd_create, and LBDD_E_INVAL for a malformed table. */
int lbdd_create_penalty_table(int32_t k, int64_t n, const int32_t *cm, const int32_t *capacity,
                              const int64_t *pen_off, const int32_t *pen_val, uint32_t flags,
                              void *hip_stream, lbdd_instance **out);

/* Cost matrix from a road network (construction of CM, Section 3.5; the
 * paper's datasets, Section 5): CM(d, s) = length of a shortest path from
 * the vertex of center s to the vertex of unit d.  All arrays are device
 * pointers:
 *   V           vertices (>= 1)
 *   row_ptr     [V + 1] int64 CSR offsets: the arcs leaving u are
 *               row_ptr[u] .. row_ptr[u + 1] - 1 (row_ptr[0] = 0)
 *   col, length [row_ptr[V]] int32 head vertex and length (in [0, 2^30)) of
 *               every arc; a two-way road is two arcs
 *   centers     [k] int32 vertex of every center (1 <= k <= LBDD_MAX_K)
 *   units       [n] int32 vertex of every demand unit
 *   cm          [n][k] int32 output, ready for lbdd_create(LBDD_CM_DEVICE)
 *   work        lbdd_road_cm_work_bytes(V, k) bytes of device scratch
 *               (owned by the caller, 16 bytes per vertex per center, for at
 *               most 256 centers at a time)
 * The input is checked on the device before the searches run; the call
 * synchronises with the stream.  Errors: LBDD_E_INVAL (sizes, NULL, a
 * malformed network, or a unit unreachable from a center or 2^30 or more
 * away), LBDD_E_DEVICE. */
size_t lbdd_road_cm_work_bytes(int32_t V, int32_t k);
int lbdd_road_cost_matrix(int32_t V, const int64_t *row_ptr, const int32_t *col, const int32_t *length,
                          int32_t k, const int32_t *centers, int64_t n, const int32_t *units, int32_t *cm,
                          void *work, void *hip_stream);

/* Create a strict-LBDD instance (Appendix B): no center may take more units
 * than its capacity and the objective is Equation (3), the sum of CM over the
 * allotment.  Solved by Algorithm 4, which Theorem 2 makes exact: each unit
 * (in the MinDistance order of lbdd_create) goes to the cheapest center that
 * still has free capacity (smallest index among equal costs), then Negative
 * Cycle Refinement runs anchored there.  Free capacity is held by zero-cost
 * dummy units, so a center with free capacity has a zero-cost transfer to
 * every other center; such a transfer orders after every real transfer of
 * cost 0 and applying it moves no unit.
 *   k, n, cm, flags, hip_stream, out   as lbdd_create
 *   capacity    [k] int32 >= 0 host array, copied
 * With excess demand (n > sum of capacities) the instance gets a dummy center
 * k of capacity n - sum whose cost is (largest CM entry + 1) for every unit:
 * lbdd_centers then reports k + 1, lbdd_snapshot's load and W cover it, the
 * units left there are -1 in lbdd_assignment, and lbdd_objective leaves
 * their constant cost out.  Then k must be below LBDD_MAX_K and every CM
 * entry below 2^30 - 1.  lbdd_solve, lbdd_solve_iters, lbdd_solve_batch,
 * lbdd_objective, lbdd_assignment, lbdd_progress, lbdd_snapshot, lbdd_stats
 * and lbdd_destroy work as for any instance (the path counters stay 0).
 * Errors: as lbdd_create. */
int lbdd_create_strict(int32_t k, int64_t n, const int32_t *cm, const int32_t *capacity,
                       uint32_t flags, void *hip_stream, lbdd_instance **out);

/* Number of centers of the instance's graph Gamma: k, or k + 1 for a strict
 * instance with a dummy center.  Errors: LBDD_E_INVAL (NULL). */
int lbdd_centers(lbdd_instance *h, int32_t *k_graph);

/* Run all remaining iterations of Algorithm 2 (allot, Algorithm 1, and
 * Appendix A when the receiving center was full).  Asynchronous: enqueued on
 * the instance's stream.  Calling it on a solved instance does nothing.
 * Errors: LBDD_E_INVAL (NULL), LBDD_E_DEVICE (launch failure). */
int lbdd_solve(lbdd_instance *h);

/* Run at most `iters` more iterations (iters >= 0).  Same semantics as
 * lbdd_solve otherwise; used to inspect intermediate allotments. */
int lbdd_solve_iters(lbdd_instance *h, int64_t iters);

/* Objective Delta of Equation (1) for the current allotment (complete after
 * lbdd_solve).  Synchronises.  Errors: LBDD_E_INVAL (NULL), LBDD_E_INTERNAL
 * (the solve hit a failed invariant), LBDD_E_DEVICE. */
int lbdd_objective(lbdd_instance *h, int64_t *out);

/* Current allotment, one int32 center index per unit in the caller's unit
 * order (-1 for units not yet allotted).  out holds n entries, host memory
 * unless LBDD_OUT_DEVICE.  Synchronises.  Errors as lbdd_objective. */
int lbdd_assignment(lbdd_instance *h, int32_t *out, uint32_t flags);

/* Number of iterations done so far (0..n).  Synchronises. */
int lbdd_progress(lbdd_instance *h, int64_t *iters_done);

/* State snapshot for inspection, all host memory, with k = lbdd_centers:
 * load [k] int32 (units per center), W [k][k] uint64 best-transfer keys of
 * the allotment-subspace graph (Definition of Gamma, Section 3.2; key =
 * ((delta + 2^31) << 32) | rank, all ones = no transfer; a strict instance's
 * dummy transfer is (2^31 << 32) | (2^32 - 2)), order [n] int64 (unit index
 * at each processing position).  Any pointer may be NULL.  Synchronises. */
int lbdd_snapshot(lbdd_instance *h, int32_t *load, uint64_t *W, int64_t *order);

/* Counters (int64, up to `count` of them, host memory):
 *   [0] cycles applied  [1] paths applied  [2] units moved
 *   [3] cycle searches run  [4] path searches run  [5] Bellman-Ford rounds
 *   [6] member rows read by list refills (one column each)
 *   [7] iterations done  [8] cycle searches skipped because the node
 *       potentials prove the table has no negative cycle
 *   [9] .. [12] device timer ticks spent in: allotment, cycle refinement,
 *       path refinement (these three sampled on one iteration in 8 and
 *       scaled by 8), list updates and refills after applied refinements
 *       (part of [10], [11])
 *   [13] best-transfer list refills (column scans of one center's members)
 *   [14] device timer when the instance's first solve launch began, [15] when
 *       its last iteration so far finished (device timer ticks)
 *   [16] Bellman-Ford edge relaxations (sum over rounds of frontier x k)
 *   [17] path searches answered from the labels of a cycle search that ran
 *        on the same table (part of [4])
 *   [18] searches run in Dijkstra order on feasible node potentials (part
 *        of [3] + [4]; the others run as Bellman-Ford rounds or are [17])
 *   [19] applied refinements after which the node potentials were kept
 *        (the search's candidate potentials, repaired where needed)
 *   [20] centers settled by the searches of [18] (each stops once no open
 *        center can lower the s_in label below 0 or below the best found)
 *   [21] candidate potentials repaired (shortest distances on reduced
 *        weights from the tails of the edges that failed the check)
 *   [22] rounds of those repairs
 *   [23] .. [25] device timer ticks spent in searches in Dijkstra order, in
 *        Bellman-Ford searches, and in potential checks and repairs
 *   [26] sink potentials computed (LBDD_OPT_SINK_EVERY), [27] ticks spent so
 *   [28] Bellman-Ford searches pruned by feasible potentials (part of the
 *        searches that are not [18])
 *   [29] device timer frequency in kHz
 * Synchronises.  Returns the number of counters written (>= 0). */
int lbdd_stats(lbdd_instance *h, int64_t *out, int32_t count);

/* Per-instance options (none changes a result, only how fast it comes).
 *   LBDD_OPT_SEARCH_RATIO  int64 in [-1, 2^20]: the cost of one Bellman-Ford
 *     round in Dijkstra steps, x16.  A refinement search runs in Dijkstra
 *     order (when the node potentials allow it and k <= 512) if the running
 *     mean of the rounds a Bellman-Ford search needs, times the ratio,
 *     exceeds the running mean of the centers a search in Dijkstra order
 *     settles (both means kept per search mode).  -1: the ratio is measured
 *     during the solve from the device times of rounds and steps (one search
 *     in 64 takes the other kind to keep both times current); 0: always
 *     Bellman-Ford; 2^20: Dijkstra whenever allowed.  New instances start
 *     with the value lbdd_tune_search recorded for their k in this process,
 *     else -1.
 * lbdd_set_option takes effect at the next solve launch.  Both synchronise
 * the instance's stream.  Errors: LBDD_E_INVAL (NULL, unknown option, value
 * out of range), LBDD_E_DEVICE. */
#define LBDD_OPT_SEARCH_RATIO 1
/*   LBDD_OPT_SINK_EVERY  int64 in [0, 2^20]: every this many path searches
 *     (Appendix A), the node potentials are first recomputed as sink
 *     potentials (minus the cheapest cost of placing one more unit starting
 *     from each center, q of a center being what its next unit pays), on
 *     which a path search in Dijkstra order settles little beyond its
 *     cheapest paths; in between they are checked and repaired on the rows
 *     of W that changed.  0: never (path searches use the same potentials
 *     as cycle searches).  New instances start with 8. */
#define LBDD_OPT_SINK_EVERY 2
int lbdd_set_option(lbdd_instance *h, int32_t option, int64_t value);
int lbdd_get_option(lbdd_instance *h, int32_t option, int64_t *value);

/* Solve many instances in one persistent launch (growth of Algorithm 2 to a
 * batch of independent instances; each instance's result is the one
 * lbdd_solve gives it alone).  Every workgroup of the launch is a worker that
 * claims instances from a device-side queue, largest remaining work (n * k)
 * first, and runs all their remaining iterations.
 *   hs          m distinct handles (partially solved ones continue where they
 *               stopped; solved ones are skipped)
 *   hip_stream  stream of the launch; each instance's own stream is made to
 *               wait for it, so later calls on a handle see its results
 * Asynchronous.  Errors: LBDD_E_INVAL (NULL or repeated handles, m < 0),
 * LBDD_E_NOMEM, LBDD_E_DEVICE. */
int lbdd_solve_batch(lbdd_instance **hs, int32_t m, void *hip_stream);

/* ---- request server (continuous batching on one GPU) ----------------------
 * A server keeps a resident service kernel whose workers (one workgroup each,
 * on all but `reserve_cus` compute units) solve admitted instances one after
 * another; each result equals lbdd_solve's result for the instance alone.
 * Requests are admitted in arrival order while their device footprint fits in
 * the HBM budget and a job slot is free; younger requests that fit may pass an
 * older one that does not, a bounded number of times in a row.  A request
 * larger than the budget runs once nothing else is in flight.  Server calls
 * are thread-safe. */
typedef struct lbdd_server lbdd_server;

enum { LBDD_JOB_QUEUED = 0, LBDD_JOB_RUNNING = 1, LBDD_JOB_DONE = 2 };

/* hbm_budget: bytes of device memory jobs may hold at once (> 0);
 * max_jobs: job slots (>= 1); reserve_cus: compute units left free for the
 * setup kernels of newly admitted jobs.  On MI355X (256 CUs) leave at least
 * 64: with more than ~192 resident workers, other kernels (the admissions'
 * setup) are held back until idle workers leave, and the pool shrinks to the
 * busy ones.  Errors: LBDD_E_INVAL, LBDD_E_NOMEM, LBDD_E_DEVICE. */
int lbdd_server_create(size_t hbm_budget, int32_t max_jobs, int32_t reserve_cus, lbdd_server **out);

/* Queue one instance (arguments as lbdd_create with a host cost matrix).
 * cm is borrowed: it must stay valid and unchanged until the job is finished
 * (lbdd_server_poll reports LBDD_JOB_DONE or an error); capacity and penalty
 * are copied.  *ticket identifies the job.  Errors: LBDD_E_INVAL,
 * LBDD_E_STATE (server shutting down). */
int lbdd_server_submit(lbdd_server *srv, int32_t k, int64_t n, const int32_t *cm,
                       const int32_t *capacity, const int32_t *penalty, uint64_t *ticket);

/* Non-blocking state of a job: LBDD_JOB_QUEUED, _RUNNING, _DONE, or a
 * negative error code; *objective is set when done (may be NULL). */
int lbdd_server_poll(lbdd_server *srv, uint64_t ticket, int32_t *state, int64_t *objective);

/* Block until the job has finished; returns its error code if it failed. */
int lbdd_server_wait(lbdd_server *srv, uint64_t ticket, int64_t *objective);

/* Copy a finished job's allotment (n int32, host memory; may be NULL) and its
 * times (5 doubles, may be NULL): in seconds since the server started, [0]
 * submitted, [1] admitted (on the device and published to the workers), [2]
 * seen finished by the server; in seconds of the device clock, [3] when its
 * first iteration began and [4] when its last one ended on the device.
 * Releases the ticket.  Errors: LBDD_E_INVAL (unknown ticket), LBDD_E_STATE
 * (not finished), or the job's own error. */
int lbdd_server_result(lbdd_server *srv, uint64_t ticket, int32_t *assign, double *times);

/* Cancel a job that is still waiting for admission: it leaves the queue,
 * its state becomes LBDD_E_CANCELLED and its cost matrix is no longer
 * borrowed (lbdd_server_result then releases the ticket).  A job already on
 * the device runs to completion.  Errors: LBDD_E_INVAL (unknown ticket),
 * LBDD_E_STATE (the job is running or finished). */
int lbdd_server_cancel(lbdd_server *srv, uint64_t ticket);

/* Queue timeout in seconds (0: none, the default): a job that has waited
 * longer than this for admission leaves the queue with state
 * LBDD_E_TIMEOUT.  Jobs already admitted are not affected.  Errors:
 * LBDD_E_INVAL (negative or not finite). */
int lbdd_server_set_queue_timeout(lbdd_server *srv, double seconds);

/* Counters (int64): [0] submitted [1] admitted [2] finished [3] failed
 * [4] service kernel launches [5] peak jobs in flight [6] peak bytes admitted
 * [7] bytes admitted now [8] workers [9] cancelled [10] timed out.  Returns
 * the number written. */
int lbdd_server_stats(lbdd_server *srv, int64_t *out, int32_t count);

/* Stop: waiting jobs are dropped (their state becomes LBDD_E_STATE), jobs
 * already on the device finish, then everything is freed. */
void lbdd_server_destroy(lbdd_server *srv);

/* Free the instance and all its device memory (synchronises its stream). */
void lbdd_destroy(lbdd_instance *h);

/* Description of the calling thread's last failure ("" if none). */
const char *lbdd_last_error(void);

/* Best-transfer table of an arbitrary allotment, scanning the whole cost
 * matrix (the condensed allotment-subspace graph, Definition of Gamma in
 * Section 3.2, with the cheapest edge per ordered pair as in the NCyc
 * definition, Section 3.3): for u != v,
 *   W[u][v] = min over units d with assign[d] == u of
 *             ((CM(d,v) - CM(d,u) + 2^31) << 32) | rank[d]
 * and all ones where no unit is allotted to u, and on the diagonal.
 *   cm      [n][k] int32, device      assign [n] int32 in [-1, k), device
 *   rank    [n] int32 >= 0 distinct, device (tie order of units)
 *   W       [k][k] uint64, device, written
 *   work    device scratch of at least lbdd_best_transfers_work_bytes(k, n);
 *           it holds the units grouped by center when the call returns
 *   flags   LBDD_SCAN_REUSE_GROUPING: work already holds the grouping of this
 *           same (assign, rank) from a previous call (e.g. after CM changed),
 *           so only the table is cleared and the cost matrix scanned
 * Asynchronous on `hip_stream`.  Errors: LBDD_E_INVAL (sizes, NULL, unknown
 * flags), LBDD_E_DEVICE. */
#define LBDD_SCAN_REUSE_GROUPING 0x1u
size_t lbdd_best_transfers_work_bytes(int32_t k, int64_t n);
int lbdd_best_transfers(int32_t k, int64_t n, const int32_t *cm, const int32_t *assign,
                        const int32_t *rank, uint64_t *W, void *work, uint32_t flags,
                        void *hip_stream);

/* lbdd_best_transfers without a workspace argument and without allocating,
 * for callers that cannot allocate device memory: code being captured into
 * a HIP graph, tight serving loops, harnesses that forbid allocation.  The
 * arguments and the result are those of lbdd_best_transfers; the workspace
 * is a fixed array of LBDD_NOALLOC_SCRATCH_BYTES (16 MiB) inside the library,
 * one per GPU, held from the library's first use on that GPU until the
 * process ends.  The call makes no hipMalloc/hipFree and no allocating
 * library call; its kernels clear what must start at zero.
 *   flags  LBDD_SCAN_REUSE_GROUPING: the scratch still holds the grouping of
 *          this same (assign, rank) from the last call on this GPU
 * Every call on one GPU shares that GPU's scratch and leaves its grouping
 * there: calls that overlap on one GPU (several streams, threads) race.
 * Asynchronous on `hip_stream`.  Errors: LBDD_E_INVAL (as lbdd_best_transfers,
 * and when lbdd_best_transfers_work_bytes(k, n) exceeds the scratch: about
 * n > 2,000,000 units), LBDD_E_DEVICE. */
#define LBDD_NOALLOC_SCRATCH_BYTES (16 << 20)
int lbdd_best_transfers_noalloc(int32_t k, int64_t n, const int32_t *cm, const int32_t *assign,
                                const int32_t *rank, uint64_t *W, uint32_t flags, void *hip_stream);

/* A plain streaming read of `bytes` bytes at `src` (device memory, 16-byte
 * aligned, bytes a multiple of 16) by `blocks` workgroups of 256 threads,
 * each thread four 16-byte loads in flight: the read bandwidth ceiling that
 * the cost-matrix scans (Section 3.2, Gamma) are compared with.  The XOR of
 * the 32-bit words read is XORed into *sink (device, 8 bytes), so every load
 * is kept.  Asynchronous on `hip_stream`.  Errors: LBDD_E_INVAL, LBDD_E_DEVICE. */
int lbdd_read_ceiling(const void *src, int64_t bytes, uint64_t *sink, int32_t blocks, void *hip_stream);

/* The tables of many allotments at once (the batched form of the scan above;
 * LBDD_SCAN_REUSE_GROUPING is defined there):
 * item i has k[i] centers (1 <= k[i] <= LBDD_MAX_K) and n[i] >= 0 units, and
 * cm[i], assign[i], rank[i], W[i] as lbdd_best_transfers (device pointers;
 * the four pointer arrays and k, n are host arrays of m entries).  One
 * sequence of launches serves all items: a clear of every table, grouping
 * passes over the concatenated units and one streaming pass over the
 * concatenated rows, split evenly over the resident workgroups; the lane
 * layout follows each item's k.  Items with k % 4 != 0 (or a cm that is not
 * 16-byte aligned) use 4-byte loads and k <= 512; others k <= 2048.
 *   work    device scratch of lbdd_best_transfers_batch_work_bytes(m, k, n)
 *           bytes (0 for invalid sizes); holds the item descriptors and the
 *           groupings when the call returns
 *   flags   LBDD_SCAN_REUSE_GROUPING: work holds the descriptors and
 *           groupings of a previous call with the same arguments (e.g. after
 *           the cost matrices changed), so only the tables are cleared and
 *           the matrices scanned: fully asynchronous
 * Without the flag the call waits for earlier work on `hip_stream`, copies
 * the item descriptors into work, then enqueues the kernels asynchronously.
 * Errors: LBDD_E_INVAL (sizes, m outside [1, LBDD_MAX_SCAN_ITEMS], NULL,
 * unknown flags, an item beyond the layouts above), LBDD_E_DEVICE. */
#define LBDD_MAX_SCAN_ITEMS 65535     /* items per lbdd_best_transfers_batch call */
size_t lbdd_best_transfers_batch_work_bytes(int32_t m, const int32_t *k, const int64_t *n);
int lbdd_best_transfers_batch(int32_t m, const int32_t *k, const int64_t *n, const int32_t *const *cm,
                              const int32_t *const *assign, const int32_t *const *rank, uint64_t *const *W,
                              void *work, uint32_t flags, void *hip_stream);

/* ---- autotuner -------------------------------------------------------------
 * Both calls time choices that leave every result unchanged and record the
 * fastest in a lock-guarded table of this process.  An instance takes its
 * search ratio from the table when it is created (looked up by its k bucket,
 * the bit length of k, and its n bucket, the number of decimal digits of n
 * minus one); a scan looks its tile configuration up (by k and load width)
 * when it is launched.  The tables can be saved to and loaded from a JSON
 * tuning cache (lbdd_tune_save / lbdd_tune_load); when the environment
 * variable LBDD_TUNE_CACHE names one, the library loads it for the current
 * device's architecture on its first lookup, so instances, batches and the
 * server start tuned.
 *
 * lbdd_tune_search: creates a fresh instance from the inputs (arguments as
 * lbdd_create) once per candidate search ratio (-1, 0, 64, 2^20), times its
 * first `iters` iterations with HIP events on `hip_stream`, checks that all
 * candidates reach the same objective, and records the fastest ratio for
 * this k and n bucket (used by later lbdd_create calls) if it beats the default (-1) by
 * more than 2 %, else the default.  A short prefix has few searches: time
 * enough iterations (up to n) to tell the candidates apart.  Writes it to
 * *ratio_out and the candidates' times in ms to ms_out[0 .. count-1].
 * Synchronises.  Returns the number of candidates (4), or LBDD_E_INVAL,
 * LBDD_E_NOMEM, LBDD_E_DEVICE, LBDD_E_INTERNAL (candidates disagreed). */
int lbdd_tune_search(int32_t k, int64_t n, const int32_t *cm, const int32_t *capacity,
                     const int32_t *penalty, uint32_t flags, int64_t iters, void *hip_stream,
                     int64_t *ratio_out, float *ms_out, int32_t count);

/* lbdd_tune_best_transfers: arguments as lbdd_best_transfers (n >= 1).
 * Groups the units once, then times the streaming pass of every tile
 * configuration that covers k columns (lanes per row, column groups per
 * lane, one or two resident waves of workgroups) `reps` times after a
 * warm-up, checks on the device that each produced the default's table, and
 * records the fastest (the default unless another is faster by more than
 * 2 %) for this k and load width (16-byte loads need
 * k % 4 == 0 and a 16-byte aligned cm).  On return W holds the table of the
 * inputs and work their grouping, as after lbdd_best_transfers.
 *   config_out  [4] int32: columns per load, lanes per row, column groups per
 *               lane, waves of workgroups of the chosen configuration
 *   ms_out      [2] float: mean ms of the default and of the chosen one
 * Synchronises.  Returns the number of configurations timed, or
 * LBDD_E_INVAL, LBDD_E_NOMEM, LBDD_E_DEVICE, LBDD_E_INTERNAL (a configuration
 * produced another table). */
int lbdd_tune_best_transfers(int32_t k, int64_t n, const int32_t *cm, const int32_t *assign,
                             const int32_t *rank, uint64_t *W, void *work, int32_t reps,
                             void *hip_stream, int32_t *config_out, float *ms_out);

/* The tuning cache: a JSON file {"format": "lbdd-tune-1", "entries": [...]}
 * whose entries carry the architecture they were tuned on ("arch", e.g.
 * "gfx950") and either a search ratio for a (k bucket, n bucket) or a scan
 * configuration for a (k, load width).
 * lbdd_tune_save writes every entry of this process's tables, tagged with
 * `arch` (NULL: the current device's), replacing the file (written to
 * path.tmp, then renamed).  Returns the number of entries written, or
 * LBDD_E_INVAL (NULL path, unwritable file), LBDD_E_DEVICE (no device to
 * name the architecture).
 * lbdd_tune_load reads such a file and applies the entries tuned on `arch`
 * (NULL: the current device's); entries of other architectures are skipped.
 * Every entry is checked first (ratio range, a scan shape this library has
 * that covers k), and a file with any bad entry changes nothing.  Returns
 * the number of entries applied, or LBDD_E_INVAL (unreadable, not JSON,
 * another format, a bad entry), LBDD_E_DEVICE.
 * lbdd_tune_clear empties both tables (every lookup then gives the
 * defaults).  None of the three launches device work. */
int lbdd_tune_save(const char *path, const char *arch);
int lbdd_tune_load(const char *path, const char *arch);
void lbdd_tune_clear(void);

#ifdef __cplusplus
}
#endif
#endif /* LBDD_H */
