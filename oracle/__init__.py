"""ctypes binding of the plain C ASRAL oracle (test infrastructure).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import it.  The product path never does;
it shares no code with the HIP library.

``build()`` compiles ``asral_oracle.c`` with gcc into ``_asral_oracle.so``
beside it, and ``build_para()`` the same source with OpenMP into
``_asral_para.so``: the para-ASRAL-style CPU baseline (Section 3.6), whose
results are identical.  Every function below cites the passage of the paper it
follows in the C source's header.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "asral_oracle.c")
LIB = os.path.join(_HERE, "_asral_oracle.so")
PARA_LIB = os.path.join(_HERE, "_asral_para.so")

TRACE_W = 8
STATS_N = 8
KEY_NONE = np.uint64(0xFFFFFFFFFFFFFFFF)
DIST_NONE = np.iinfo(np.int64).max

E_INVAL, E_NOMEM, E_NEGCYCLE = -1, -2, -5


def build(src: str = SRC, out: str = LIB, extra=()) -> str:
    """Compile the oracle with gcc (-O2, strict IEEE irrelevant: integer only)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-Wno-unknown-pragmas", "-fPIC", "-shared",
           *extra, "-o", out, src]
    subprocess.run(cmd, check=True)
    return out


def build_para(out: str = PARA_LIB) -> str:
    """The para-ASRAL-style build: the same source with OpenMP threads."""
    return build(out=out, extra=("-fopenmp",))


_lib = None
_para = None


def load_para():
    """The threaded build (thread count from OMP_NUM_THREADS)."""
    global _para
    if _para is None:
        if not os.path.exists(PARA_LIB):
            build_para()
        _para = _load(PARA_LIB)
    return _para


def _load(path: str = LIB):
    global _lib
    if path == LIB and _lib is not None:
        return _lib
    if not os.path.exists(path):
        build(out=path)
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.orc_setup.argtypes = [C.c_int32, C.c_int64, P, P, P, P, P]
    lib.orc_best_transfers.argtypes = [C.c_int32, C.c_int64, P, P, P, P]
    lib.orc_objective.argtypes = [C.c_int32, C.c_int64, P, P, P, P, P]
    lib.orc_refine_search.argtypes = [C.c_int32, P, C.c_int32, C.c_int32, P, P, P, P, P, P]
    lib.orc_solve.argtypes = [C.c_int32, C.c_int64, P, P, P, C.c_int64, P, P, P, P, P, P]
    lib.orc_solve_strict.argtypes = [C.c_int32, C.c_int64, P, P, C.c_int64, P, P, P, P, P, P]
    lib.orc_solve_q.argtypes = [C.c_int32, C.c_int64, P, P, P, P, C.c_int64, P, P, P, P, P, P]
    lib.orc_refine_search_q.argtypes = [C.c_int32, P, C.c_int32, C.c_int32, P, P, P, P, P, P, P]
    lib.orc_road_cm.argtypes = [C.c_int32, P, P, P, C.c_int32, P, C.c_int64, P, P]
    for f in (lib.orc_setup, lib.orc_best_transfers, lib.orc_objective,
              lib.orc_refine_search, lib.orc_solve, lib.orc_solve_strict, lib.orc_solve_q,
              lib.orc_refine_search_q, lib.orc_road_cm):
        f.restype = C.c_int
    if path == LIB:
        _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class OracleError(RuntimeError):
    def __init__(self, rc: int, what: str):
        super().__init__(f"{what} failed with code {rc}")
        self.rc = rc


def setup(cm: np.ndarray, lib=None):
    """(smin, mc, order, rank) -- Algorithm 2 step 1."""
    lib = lib or _load()
    cm = _i32(cm)
    n, k = cm.shape
    smin = np.empty(n, np.int32); mc = np.empty(n, np.int32)
    order = np.empty(n, np.int64); rank = np.empty(n, np.int64)
    rc = lib.orc_setup(k, n, _p(cm), _p(smin), _p(mc), _p(order), _p(rank))
    if rc:
        raise OracleError(rc, "orc_setup")
    return smin, mc, order, rank


def best_transfers(cm: np.ndarray, assign: np.ndarray, rank: np.ndarray, lib=None) -> np.ndarray:
    """Condensed Gamma(A) as packed uint64 keys [k][k] (definition of Gamma)."""
    lib = lib or _load()
    cm = _i32(cm)
    n, k = cm.shape
    W = np.empty((k, k), np.uint64)
    rc = lib.orc_best_transfers(k, n, _p(cm), _p(_i32(assign)),
                                _p(np.ascontiguousarray(rank, dtype=np.int64)), _p(W))
    if rc:
        raise OracleError(rc, "orc_best_transfers")
    return W


def objective(cm, cap, pen, assign, lib=None) -> int:
    """Equation (1) with constant per-unit penalties."""
    lib = lib or _load()
    cm = _i32(cm)
    n, k = cm.shape
    out = np.zeros(1, np.int64)
    rc = lib.orc_objective(k, n, _p(cm), _p(_i32(cap)), _p(_i32(pen)), _p(_i32(assign)), _p(out))
    if rc:
        raise OracleError(rc, "orc_objective")
    return int(out[0])


def refine_search(W: np.ndarray, anchor: int, mode: int, load, cap, pen, lib=None):
    """Shortest s*_out -> s*_in path on NCyc (mode 0) or NPath (mode 1).

    Returns (dist[k+1], pred[k+1], rounds)."""
    lib = lib or _load()
    W = np.ascontiguousarray(W, dtype=np.uint64)
    k = W.shape[0]
    dist = np.empty(k + 1, np.int64); pred = np.empty(k + 1, np.int32)
    rounds = np.zeros(1, np.int32)
    rc = lib.orc_refine_search(k, _p(W), anchor, mode, _p(_i32(load)), _p(_i32(cap)),
                               _p(_i32(pen)), _p(dist), _p(pred), _p(rounds))
    if rc:
        raise OracleError(rc, "orc_refine_search")
    return dist, pred, int(rounds[0])


def refine_search_q(W: np.ndarray, anchor: int, mode: int, load, cap, pen_off, pen_val, lib=None):
    """refine_search with a penalty table per center (see solve_q)."""
    lib = lib or _load()
    W = np.ascontiguousarray(W, dtype=np.uint64)
    k = W.shape[0]
    dist = np.empty(k + 1, np.int64); pred = np.empty(k + 1, np.int32)
    rounds = np.zeros(1, np.int32)
    off = np.ascontiguousarray(pen_off, dtype=np.int64)
    rc = lib.orc_refine_search_q(k, _p(W), anchor, mode, _p(_i32(load)), _p(_i32(cap)),
                                 _p(off), _p(_i32(pen_val)), _p(dist), _p(pred), _p(rounds))
    if rc:
        raise OracleError(rc, "orc_refine_search_q")
    return dist, pred, int(rounds[0])


@dataclass
class Result:
    assign: np.ndarray      # int32 [n], center per unit id (-1: not allotted)
    load: np.ndarray        # int32 [k]
    objective: int          # Delta, int64
    W: np.ndarray | None    # uint64 [k][k] heap tops after the last iteration
    trace: np.ndarray | None  # int64 [iters][TRACE_W]
    stats: np.ndarray       # int64 [STATS_N]


def solve(cm, cap, pen, max_iters: int = -1, want_W: bool = False, want_trace: bool = False,
          lib=None) -> Result:
    """ASRAL, Algorithm 2, run for min(n, max_iters) iterations."""
    lib = lib or _load()
    cm = _i32(cm)
    n, k = cm.shape
    iters = n if (max_iters < 0 or max_iters > n) else max_iters
    assign = np.empty(n, np.int32); load = np.empty(k, np.int32)
    obj = np.zeros(1, np.int64)
    W = np.empty((k, k), np.uint64) if want_W else None
    trace = np.zeros((max(iters, 1), TRACE_W), np.int64) if want_trace else None
    stats = np.zeros(STATS_N, np.int64)
    rc = lib.orc_solve(k, n, _p(cm), _p(_i32(cap)), _p(_i32(pen)), iters, _p(assign), _p(load),
                       _p(obj), _p(W) if W is not None else None,
                       _p(trace) if trace is not None else None, _p(stats))
    if rc:
        raise OracleError(rc, "orc_solve")
    return Result(assign, load, int(obj[0]), W, trace[:iters] if trace is not None else None, stats)


@dataclass
class StrictResult:
    assign: np.ndarray        # [n] center per unit id, -1 if left at the dummy center
    load: np.ndarray          # [kx] units per center (dummy center last when added)
    kx: int                   # k, or k + 1 with the dummy center of excess demand
    objective: int            # Equation (3): sum of CM over allotted units
    W: np.ndarray | None      # [kx][kx] best-transfer keys with dummy transfers
    stats: np.ndarray


DUMMY_KEY = np.uint64((1 << 63) | 0xFFFFFFFE)


def solve_strict(cm, cap, max_iters: int = -1, want_W: bool = False, lib=None) -> StrictResult:
    """Strict-LBDD, Algorithm 4 (Appendix B), run for min(n, max_iters) iterations."""
    lib = lib or _load()
    cm = _i32(cm)
    n, k = cm.shape
    iters = n if (max_iters < 0 or max_iters > n) else max_iters
    assign = np.empty(n, np.int32); load = np.zeros(k + 1, np.int32)
    kx = np.zeros(1, np.int32); obj = np.zeros(1, np.int64)
    W = np.empty((k + 1) * (k + 1), np.uint64) if want_W else None
    stats = np.zeros(STATS_N, np.int64)
    rc = lib.orc_solve_strict(k, n, _p(cm), _p(_i32(cap)), iters, _p(assign), _p(load), _p(kx),
                              _p(obj), _p(W) if W is not None else None, _p(stats))
    if rc:
        raise OracleError(rc, "orc_solve_strict")
    m = int(kx[0])
    return StrictResult(assign, load[:m], m, int(obj[0]),
                        W[:m * m].reshape(m, m) if W is not None else None, stats)


# -- key packing (the interface format of best-transfer keys) --------------
def key_delta(W: np.ndarray) -> np.ndarray:
    return (W >> np.uint64(32)).astype(np.int64) - 2**31


def key_rank(W: np.ndarray) -> np.ndarray:
    return (W & np.uint64(0xFFFFFFFF)).astype(np.int64)


def solve_q(cm, cap, pen_off, pen_val, max_iters: int = -1, want_W: bool = False,
            want_trace: bool = False, lib=None) -> Result:
    """ASRAL with a general penalty function (Definition of the penalty
    function, Section 2): the j-th unit beyond the capacity of center s pays
    pen_val[pen_off[s] + min(j, len_s) - 1], len_s = pen_off[s+1] - pen_off[s]
    >= 1 (the last value of a center's table holds for every later unit)."""
    lib = lib or _load()
    cm = _i32(cm)
    n, k = cm.shape
    iters = n if (max_iters < 0 or max_iters > n) else max_iters
    assign = np.empty(n, np.int32); load = np.empty(k, np.int32)
    obj = np.zeros(1, np.int64)
    W = np.empty((k, k), np.uint64) if want_W else None
    trace = np.zeros((max(iters, 1), TRACE_W), np.int64) if want_trace else None
    stats = np.zeros(STATS_N, np.int64)
    off = np.ascontiguousarray(pen_off, dtype=np.int64)
    rc = lib.orc_solve_q(k, n, _p(cm), _p(_i32(cap)), _p(off), _p(_i32(pen_val)), iters,
                         _p(assign), _p(load), _p(obj), _p(W) if W is not None else None,
                         _p(trace) if trace is not None else None, _p(stats))
    if rc:
        raise OracleError(rc, "orc_solve_q")
    return Result(assign, load, int(obj[0]), W, trace[:iters] if trace is not None else None, stats)


def road_cm(row_ptr, col, length, centers, units, lib=None) -> np.ndarray:
    """Cost matrix [n][k] int32 from a road network: the shortest-path length
    from the vertex of each center to the vertex of each unit (Dijkstra from
    every center).  The graph is CSR: arcs row_ptr[u]..row_ptr[u+1]-1 leave u."""
    lib = lib or _load()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    V = len(rp) - 1
    centers = _i32(centers); units = _i32(units)
    k, n = len(centers), len(units)
    cm = np.empty((n, k), np.int32)
    rc = lib.orc_road_cm(V, _p(rp), _p(_i32(col)), _p(_i32(length)), k, _p(centers), n,
                         _p(units), _p(cm))
    if rc:
        raise OracleError(rc, "orc_road_cm")
    return cm
