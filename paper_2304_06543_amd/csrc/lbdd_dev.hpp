// lbdd_dev.hpp -- device-side types and helpers shared by the HIP kernels of
// the MI355X ASRAL solver.  gfx950 only: wave64, 160 KB LDS per CU.
#pragma once

#include <vector>

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbdd {

constexpr uint64_t KEY_NONE = ~0ull;          // "no transfer" in the best-transfer table
constexpr int64_t DIST_NONE = INT64_MAX;      // unreachable Bellman-Ford label
constexpr int32_t CM_LIMIT = 1 << 30;         // costs and penalties lie in [0, 2^30)

// Best-transfer key of moving the unit at processing rank `rank` between two
// centers with transfer cost `delta` (Definition of Gamma, Section 3.2):
// unsigned order = (delta, rank) lexicographic, so a plain integer min picks
// the cheapest transfer and, among equal costs, the earliest-processed unit.
// (The bias is added in unsigned arithmetic: delta + 2^31 in int32 would
// overflow for every negative delta.)
__device__ __host__ inline uint64_t pack_key(int32_t delta, uint32_t rank) {
  return (uint64_t)((uint32_t)delta ^ 0x80000000u) << 32 | rank;
}
__device__ __host__ inline int32_t key_delta(uint64_t key) {
  return (int32_t)((uint32_t)(key >> 32) - 0x80000000u);
}
__device__ __host__ inline uint32_t key_rank(uint64_t key) { return (uint32_t)key; }

// Key of a zero-cost dummy-unit transfer of strict-LBDD (Appendix B): a
// center with free capacity holds dummy units that can move to any other
// center at no cost.  Its rank field lies beyond every real row, so it
// orders after every real key of cost 0; moving it moves no real unit.
constexpr uint64_t DUMMY_KEY = (uint64_t)0x80000000u << 32 | 0xfffffffeu;

// Bias that makes a search label (a sum of at most LBDD_MAX_K+1 edges of
// magnitude < 2^31) non-negative, so labels order as unsigned integers.
constexpr int64_t DIST_BIAS = 1ll << 46;

// Device view of one instance.  Rows of `cm` are in processing order: row r is
// the unit processed in iteration r, so a best-transfer key's rank is the row.
struct InstView {
  int32_t k;
  int32_t strict;          // strict-LBDD: W[u][v] includes the dummy transfer
                           // while u has free capacity; allotment goes to the
                           // cheapest center with free capacity
  int64_t n;
  const int32_t *cm;       // [n][k] permuted cost matrix
  const int32_t *smin;     // [n] most suitable center of row r
  const int32_t *cap;      // [k]
  const int32_t *pen;      // [k]
  int32_t *assign;         // [n] center of row r, -1 before its iteration
  int32_t *load;           // [k] units per center
  int32_t *members;        // [k][n] rows allotted to each center (first load[u])
  int32_t *slot;           // [n] index of row r in its center's member list
  uint64_t *W;             // [k][k] best-transfer table (heads of the lists below)
  uint32_t *Wh;            // [k][k] high words of W (delta + 2^31, all ones = no
                           // transfer): what a search reads, at half the bytes,
                           // while W is in global memory
  uint32_t *WhT;           // [k][k] the same high words transposed (WhT[v][u] is
                           // W[u][v]'s), kept in every launch: read by the
                           // searches toward the penalty sink
  uint64_t *best;          // [k][k][BEST_M] smallest transfer keys of each pair
  uint8_t *meta;           // [k][k] keys held (low 4 bits), every unit held (META_ALL)
  uint64_t *thr;           // [k][k] a joining unit's key changes the list (or its
                           // flags) only if it is below this threshold
  int64_t *scalars;        // [SC_COUNT] objective, progress, status, counters
  // penalty function per center as a table (null: the constant pen[s]): the
  // j-th unit beyond the capacity of s pays pval[poff[s] + min(j, len) - 1],
  // len = poff[s + 1] - poff[s] >= 1
  const int64_t *poff;     // [k + 1]
  const int32_t *pval;     // [poff[k]]
};

// Bounded best-transfer lists (the paper's BestTransHeap of an ordered center
// pair, truncated): the list of (u, w) holds the c <= BEST_M smallest keys
// among the units now allotted to u, sorted, unused slots all ones.
constexpr int BEST_M = 8;
constexpr uint8_t META_ALL = 16;   // the list holds every unit of the center

// layout of InstView::scalars
enum : int {
  SC_OBJECTIVE = 0,
  SC_DONE = 1,          // iterations completed
  SC_STATUS = 2,        // 0 ok, else an LBDD_E_* code
  SC_STAT0 = 3,         // first of the counters reported by lbdd_stats
  SC_NSTATS = 29,
  SC_RATIO = SC_STAT0 + SC_NSTATS,   // search-choice ratio (x16, see refine in solve.hip)
  SC_SINK_EVERY,                     // path searches per sink-potential computation
  SC_COUNT
};
// Cost of a Bellman-Ford round in Dijkstra steps (x16), or AUTO: the ratio
// of the measured times of a round and of a step (the default unless tuned).
constexpr int64_t SEARCH_RATIO_AUTO = -1;
constexpr int64_t DEFAULT_SEARCH_RATIO = SEARCH_RATIO_AUTO;
constexpr int64_t MAX_SEARCH_RATIO = 1 << 20;   // Dijkstra whenever it applies
constexpr int64_t MAX_SINK_EVERY = 1 << 20;
// Path searches per sink-potential computation unless set per instance.
constexpr int64_t DEFAULT_SINK_EVERY = 8;
enum : int {
  ST_CYCLES = 0, ST_PATHS, ST_MOVES, ST_CYC_SEARCH, ST_PATH_SEARCH, ST_BF_ROUNDS,
  ST_ROWS_SCANNED, ST_ITERS, ST_CYC_SKIPPED,
  // device wall-clock ticks spent in each phase (thread 0's view)
  ST_T_ALLOT, ST_T_CYCLE, ST_T_PATH, ST_T_RESCAN,
  ST_REFILLS,           // list refills (column rescans)
  ST_T_FIRST,           // device timer when the instance's first launch began
  ST_T_LAST,            // device timer when its last iteration finished
  ST_RELAX,             // Bellman-Ford edge relaxations (frontier size x targets)
  ST_PATH_DERIVED,      // path searches answered from the cycle search's labels
  ST_DIJKSTRA,          // searches run in Dijkstra order on feasible potentials
  ST_POT_KEPT,          // applied refinements whose labels stayed feasible potentials
  ST_DJ_SETTLED,        // centers settled by searches in Dijkstra order
  ST_POT_REPAIRS,       // candidate potentials repaired after a failed check
  ST_REPAIR_ROUNDS,     // rounds of those repairs
  // device timer ticks spent in (thread 0's view): searches in Dijkstra
  // order, Bellman-Ford searches, potential checks and repairs
  ST_T_DIJKSTRA, ST_T_BF, ST_T_POT,
  ST_SINK,              // sink potentials computed (see sink_potential in solve.hip)
  ST_T_SINK,            // device timer ticks spent computing them
  ST_BF_PRUNED          // Bellman-Ford searches pruned by feasible potentials
};

// one workgroup solves one instance
constexpr int SOLVE_THREADS = 1024;
// W is kept in LDS when the whole per-instance LDS image fits (160 KB per CU
// on gfx950, a margin left for static LDS)
constexpr size_t LDS_BUDGET = 156 * 1024;
__host__ __device__ size_t solve_lds_bytes(int k, bool wlds);

// one instance of a batched launch
struct BatchItem {
  InstView inst;
  int64_t r_begin;          // first iteration still to run
};

// Request server: control block and job ring in pinned host memory, shared
// by the host server thread and the resident service kernel.
struct ServiceCtl {
  int64_t published;        // jobs published so far (host writes, release)
  int64_t shutdown;         // nonzero: workers leave once no job is waiting
};
// Device-memory side of the service kernel: the claim counter and mirrors of
// the host's control block.  Idle workers poll these (in L2) instead of host
// memory; one worker at a time refreshes the mirrors from host memory.
struct ServiceDev {
  int64_t head;             // jobs claimed so far
  int64_t published;        // mirror of ServiceCtl::published
  int64_t shutdown;         // mirror of ServiceCtl::shutdown
  int64_t polled;           // device timer of the last refresh from host memory
};
struct ServiceJob {
  InstView inst;            // device state of the job's instance
};

// ---- host launchers (return hipError_t) ----
// setup.hip: most suitable center, processing order, row permutation
size_t setup_work_bytes(int32_t k, int64_t n);
hipError_t launch_setup(int32_t k, int64_t n, const int32_t *cm_in, int32_t *cm_perm,
                        int32_t *smin_perm, int64_t *order, int32_t *bad_flag, void *work,
                        hipStream_t st);
// solve.hip: iterations [r_begin, r_end) of the main loop
hipError_t launch_init_state(const InstView &I, hipStream_t st);
hipError_t launch_solve(const InstView &I, int64_t r_begin, int64_t r_end, hipStream_t st);
hipError_t launch_unpermute(int64_t n, const int64_t *order, const int32_t *assign, int32_t dummy,
                            int32_t *out, hipStream_t st);
// setup.hip: the cost matrix of a strict-LBDD instance with excess demand,
// extended by a dummy center whose column holds (largest entry + 1); *mx
// receives the largest entry (it must hold 0 before the call)
hipError_t launch_extend_dummy(int32_t k, int64_t n, const int32_t *cm, int32_t *cm_ext, int32_t *mx,
                               hipStream_t st);
size_t batch_lds_bytes(const BatchItem *items_host, int32_t m);
int batch_workers(size_t lds_bytes, int32_t m);
hipError_t launch_solve_batch(const BatchItem *items_dev, int32_t m, int32_t *head, size_t lds_bytes,
                              int workers, hipStream_t st);
int device_cus();
hipError_t launch_service(ServiceCtl *ctl, const ServiceJob *ring, int32_t ring_size, int64_t *done,
                          ServiceDev *dev, int64_t idle_ticks, int workers, hipStream_t st);
// tune.hip: values chosen by the autotuner for this process (or loaded from
// a tuning cache), looked up by the k bucket (bit length of k) and the n
// bucket (decimal digits of n minus one)
int64_t tuned_search_ratio(int32_t k, int64_t n);
int tune_bucket_k(int32_t k);
int tune_bucket_n(int64_t n);
void tune_cache_autoload();
// scan.hip: whole-matrix best-transfer table.  A tile configuration: VEC
// columns per load, LPR lanes per row, NP column groups per lane, MULT
// resident waves of workgroups.
struct ScanCfg {
  int32_t vec, lpr, np, mult;
};
bool scan_cfg_valid(int32_t k, const ScanCfg &c);
ScanCfg scan_default_cfg(int32_t k, bool vec4);
int scan_candidates(int32_t k, bool vec4, ScanCfg *out, int max);
void scan_set_tuned(int32_t k, bool vec4, const ScanCfg &c);
struct ScanTuned {
  int32_t k;
  bool vec4;
  ScanCfg cfg;
};
std::vector<ScanTuned> scan_tuned_list();
void scan_clear_tuned();
hipError_t launch_scan_group(int32_t k, int64_t n, const int32_t *assign, const int32_t *rank,
                             uint64_t *W, void *work, bool regroup, hipStream_t st);
hipError_t launch_scan_only(int32_t k, const int32_t *cm, void *work, const ScanCfg &c,
                            uint64_t *W, hipStream_t st);
bool scan_vec4_ok(int32_t k, const int32_t *cm);
hipError_t launch_differ(const uint64_t *a, const uint64_t *b, int64_t count, int32_t *flag,
                         hipStream_t st);
size_t scan_work_bytes(int32_t k, int64_t n);
hipError_t launch_full_scan(int32_t k, int64_t n, const int32_t *cm, const int32_t *assign,
                            const int32_t *rank, uint64_t *W, void *work, bool reuse_grouping,
                            hipStream_t st);

}  // namespace lbdd
