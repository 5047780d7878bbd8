"""Python binding of liblbdd.so (argument marshalling only).

Every step of the solve runs in the HIP library; this module only converts
arguments.  torch is used for device memory and streams.  There is no CPU
fallback: if the built library is missing, loading raises.

    inst = Instance(cm, capacity, penalty)     # cm: torch int32 (cuda) or numpy
    inst.solve()
    inst.objective(), inst.assignment()
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbdd.so")

OK, E_INVAL, E_NOMEM, E_DEVICE, E_STATE, E_INTERNAL, E_CANCELLED, E_TIMEOUT = 0, -1, -2, -3, -4, -5, -6, -7
CM_DEVICE = 0x1
OUT_DEVICE = 0x1
MAX_K = 2048
STATS = ("cycles", "paths", "moves", "cycle_searches", "path_searches", "bf_rounds",
         "rows_scanned", "iterations", "cycle_searches_skipped",
         "ticks_allot", "ticks_cycle", "ticks_path", "ticks_rescan", "refills",
         "tick_first", "tick_last", "relaxations", "paths_derived", "dijkstra",
         "potentials_kept", "dijkstra_settled", "potential_repairs", "repair_rounds",
         "ticks_dijkstra", "ticks_bf", "ticks_potentials", "sink_potentials", "ticks_sink",
         "bf_pruned", "timer_khz")

# search ratios lbdd_tune_search times, in order: measured during the solve,
# always Bellman-Ford, a fixed 4 steps per round, Dijkstra whenever allowed
SEARCH_AUTO = -1
SEARCH_CANDIDATES = (SEARCH_AUTO, 0, 64, 1 << 20)

# every symbol include/lbdd.h declares
EXPORTS = ("lbdd_create", "lbdd_solve", "lbdd_solve_iters", "lbdd_solve_batch", "lbdd_objective",
           "lbdd_assignment", "lbdd_progress", "lbdd_snapshot", "lbdd_stats",
           "lbdd_destroy", "lbdd_last_error", "lbdd_best_transfers_work_bytes",
           "lbdd_best_transfers", "lbdd_server_create", "lbdd_server_submit",
           "lbdd_server_poll", "lbdd_server_wait", "lbdd_server_result", "lbdd_server_stats",
           "lbdd_server_destroy", "lbdd_set_option", "lbdd_get_option", "lbdd_tune_search",
           "lbdd_tune_best_transfers", "lbdd_create_strict", "lbdd_centers",
           "lbdd_create_penalty_table", "lbdd_road_cm_work_bytes", "lbdd_road_cost_matrix",
           "lbdd_best_transfers_batch_work_bytes", "lbdd_best_transfers_batch",
           "lbdd_best_transfers_noalloc", "lbdd_read_ceiling", "lbdd_server_cancel",
           "lbdd_server_set_queue_timeout", "lbdd_tune_save", "lbdd_tune_load", "lbdd_tune_clear")
JOB_QUEUED, JOB_RUNNING, JOB_DONE = 0, 1, 2
SERVER_STATS = ("submitted", "admitted", "finished", "failed", "kernel_launches",
                "peak_jobs", "peak_bytes", "bytes_now", "workers", "cancelled", "timed_out")

_lib = None


class LbddError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbdd error {code}: {msg}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2304_06543_amd.build`")
    lib = C.CDLL(path)
    P, I32, I64, U32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32
    sig = {
        "lbdd_create": ([I32, I64, P, P, P, U32, P, C.POINTER(P)], C.c_int),
        "lbdd_solve": ([P], C.c_int),
        "lbdd_solve_iters": ([P, I64], C.c_int),
        "lbdd_solve_batch": ([C.POINTER(P), I32, P], C.c_int),
        "lbdd_objective": ([P, C.POINTER(I64)], C.c_int),
        "lbdd_assignment": ([P, P, U32], C.c_int),
        "lbdd_progress": ([P, C.POINTER(I64)], C.c_int),
        "lbdd_snapshot": ([P, P, P, P], C.c_int),
        "lbdd_stats": ([P, P, I32], C.c_int),
        "lbdd_destroy": ([P], None),
        "lbdd_last_error": ([], C.c_char_p),
        "lbdd_best_transfers_work_bytes": ([I32, I64], C.c_size_t),
        "lbdd_best_transfers": ([I32, I64, P, P, P, P, P, U32, P], C.c_int),
        "lbdd_server_create": ([C.c_size_t, I32, I32, C.POINTER(P)], C.c_int),
        "lbdd_server_submit": ([P, I32, I64, P, P, P, C.POINTER(C.c_uint64)], C.c_int),
        "lbdd_server_poll": ([P, C.c_uint64, C.POINTER(I32), C.POINTER(I64)], C.c_int),
        "lbdd_server_wait": ([P, C.c_uint64, C.POINTER(I64)], C.c_int),
        "lbdd_server_result": ([P, C.c_uint64, P, P], C.c_int),
        "lbdd_server_stats": ([P, P, I32], C.c_int),
        "lbdd_server_destroy": ([P], None),
        "lbdd_server_cancel": ([P, C.c_uint64], C.c_int),
        "lbdd_tune_save": ([C.c_char_p, C.c_char_p], C.c_int),
        "lbdd_tune_load": ([C.c_char_p, C.c_char_p], C.c_int),
        "lbdd_tune_clear": ([], None),
        "lbdd_server_set_queue_timeout": ([P, C.c_double], C.c_int),
        "lbdd_set_option": ([P, I32, I64], C.c_int),
        "lbdd_get_option": ([P, I32, C.POINTER(I64)], C.c_int),
        "lbdd_tune_search": ([I32, I64, P, P, P, U32, I64, P, C.POINTER(I64), P, I32], C.c_int),
        "lbdd_tune_best_transfers": ([I32, I64, P, P, P, P, P, I32, P, P, P], C.c_int),
        "lbdd_create_strict": ([I32, I64, P, P, U32, P, C.POINTER(P)], C.c_int),
        "lbdd_centers": ([P, C.POINTER(I32)], C.c_int),
        "lbdd_create_penalty_table": ([I32, I64, P, P, P, P, U32, P, C.POINTER(P)], C.c_int),
        "lbdd_road_cm_work_bytes": ([I32, I32], C.c_size_t),
        "lbdd_road_cost_matrix": ([I32, P, P, P, I32, P, I64, P, P, P, P], C.c_int),
        "lbdd_best_transfers_batch_work_bytes": ([I32, P, P], C.c_size_t),
        "lbdd_best_transfers_batch": ([I32, P, P, P, P, P, P, P, U32, P], C.c_int),
        "lbdd_best_transfers_noalloc": ([I32, I64, P, P, P, P, U32, P], C.c_int),
        "lbdd_read_ceiling": ([P, I64, P, I32, P], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc < 0:
        raise LbddError(rc, load().lbdd_last_error().decode())
    return rc


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _host_i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.int32)


OPT_SEARCH_RATIO = 1
OPT_SINK_EVERY = 2


def _create_args(cm, capacity, penalty):
    """(k, n, cm pointer, flags, capacity, penalty, buffer to keep alive) for
    lbdd_create from a torch cuda tensor or a host array."""
    cap = _host_i32(capacity)
    pen = _host_i32(penalty)
    if hasattr(cm, "is_cuda") and cm.is_cuda:
        import torch
        if cm.dtype != torch.int32 or not cm.is_contiguous() or cm.dim() != 2:
            raise ValueError("cm must be a contiguous 2-D int32 tensor")
        n, k = cm.shape
        ptr, flags, keep = C.c_void_p(cm.data_ptr()), CM_DEVICE, cm
    else:
        cmh = _host_i32(cm)
        if cmh.ndim != 2:
            raise ValueError("cm must be 2-D [n][k]")
        n, k = cmh.shape
        ptr, flags, keep = cmh.ctypes.data_as(C.c_void_p), 0, cmh
    if cap.shape != (k,) or pen.shape != (k,):
        raise ValueError("capacity and penalty need k entries")
    return int(k), int(n), ptr, flags, cap, pen, keep


class Instance:
    """One LBDD instance living on the GPU (lbdd_create ... lbdd_destroy)."""

    def __init__(self, cm, capacity, penalty=None, stream=None, strict: bool = False,
                 pen_table=None):
        """penalty (one constant per center) is required unless strict
        (strict-LBDD, lbdd_create_strict, which takes none) or pen_table =
        (offsets[k+1], values) gives a penalty function per center
        (lbdd_create_penalty_table)."""
        lib = load()
        self._lib = lib
        self._h = C.c_void_p()
        if strict or pen_table is not None:
            if penalty is not None or (strict and pen_table is not None):
                raise ValueError("give one of penalty, pen_table, strict")
            k, n, ptr, flags, cap, _, keep = _create_args(cm, capacity, capacity)
        else:
            if penalty is None:
                raise ValueError("penalty is required")
            k, n, ptr, flags, cap, pen, keep = _create_args(cm, capacity, penalty)
        self.k, self.n, self.strict = k, n, strict
        self._stream = _stream_ptr(stream)
        if strict:
            _check(lib.lbdd_create_strict(k, n, ptr, cap.ctypes.data_as(C.c_void_p), flags,
                                          self._stream, C.byref(self._h)))
        elif pen_table is not None:
            off = np.ascontiguousarray(pen_table[0], dtype=np.int64)
            val = _host_i32(pen_table[1])
            if off.shape != (k + 1,) or val.shape != (int(off[-1]),):
                raise ValueError("pen_table needs k + 1 offsets and offsets[k] values")
            _check(lib.lbdd_create_penalty_table(k, n, ptr, cap.ctypes.data_as(C.c_void_p),
                                                 off.ctypes.data_as(C.c_void_p),
                                                 val.ctypes.data_as(C.c_void_p), flags,
                                                 self._stream, C.byref(self._h)))
        else:
            _check(lib.lbdd_create(k, n, ptr, cap.ctypes.data_as(C.c_void_p),
                                   pen.ctypes.data_as(C.c_void_p), flags, self._stream,
                                   C.byref(self._h)))
        del keep
        kg = C.c_int32()
        _check(lib.lbdd_centers(self._h, C.byref(kg)))
        self.k_graph = int(kg.value)    # k, or k + 1 with strict-LBDD's dummy center

    def set_option(self, option: int, value: int):
        _check(self._lib.lbdd_set_option(self._h, int(option), int(value)))
        return self

    def get_option(self, option: int) -> int:
        out = C.c_int64()
        _check(self._lib.lbdd_get_option(self._h, int(option), C.byref(out)))
        return out.value

    def solve(self):
        _check(self._lib.lbdd_solve(self._h))
        return self

    def solve_iters(self, iters: int):
        _check(self._lib.lbdd_solve_iters(self._h, int(iters)))
        return self

    def objective(self) -> int:
        out = C.c_int64()
        _check(self._lib.lbdd_objective(self._h, C.byref(out)))
        return int(out.value)

    def progress(self) -> int:
        out = C.c_int64()
        _check(self._lib.lbdd_progress(self._h, C.byref(out)))
        return int(out.value)

    def assignment(self, device: bool = False):
        """int32 center per unit (-1 if not yet allotted): numpy, or a torch
        cuda tensor with device=True."""
        if device:
            import torch
            out = torch.empty(self.n, dtype=torch.int32, device="cuda")
            _check(self._lib.lbdd_assignment(self._h, C.c_void_p(out.data_ptr()), OUT_DEVICE))
            return out
        out = np.empty(self.n, np.int32)
        _check(self._lib.lbdd_assignment(self._h, out.ctypes.data_as(C.c_void_p), 0))
        return out

    def snapshot(self):
        """(load[kg], W[kg][kg] uint64 keys, order[n]) with kg = k_graph."""
        load_ = np.empty(self.k_graph, np.int32)
        W = np.empty((self.k_graph, self.k_graph), np.uint64)
        order = np.empty(self.n, np.int64)
        _check(self._lib.lbdd_snapshot(self._h, load_.ctypes.data_as(C.c_void_p),
                                       W.ctypes.data_as(C.c_void_p),
                                       order.ctypes.data_as(C.c_void_p)))
        return load_, W, order

    def stats(self) -> dict:
        out = np.zeros(len(STATS), np.int64)
        m = _check(self._lib.lbdd_stats(self._h, out.ctypes.data_as(C.c_void_p), len(STATS)))
        return {name: int(out[i]) for i, name in enumerate(STATS[:m])}

    def close(self):
        if self._h:
            self._lib.lbdd_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def solve(cm, capacity, penalty, stream=None):
    """Solve one instance; returns (objective, assignment as numpy int32)."""
    with Instance(cm, capacity, penalty, stream) as inst:
        inst.solve()
        return inst.objective(), inst.assignment()


def road_cost_matrix(row_ptr, col, length, centers, units, work=None, stream=None):
    """Cost matrix [n][k] int32 (a torch cuda tensor) from a road network given
    as torch cuda tensors: row_ptr int64 [V+1], col and length int32 [E],
    centers int32 [k], units int32 [n] (lbdd_road_cost_matrix)."""
    import torch
    lib = load()
    for name, t, dt in (("row_ptr", row_ptr, torch.int64), ("col", col, torch.int32),
                        ("length", length, torch.int32), ("centers", centers, torch.int32),
                        ("units", units, torch.int32)):
        if not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous cuda tensor of {dt}")
    V, k, n = row_ptr.numel() - 1, centers.numel(), units.numel()
    if work is None:
        work = torch.empty(lib.lbdd_road_cm_work_bytes(V, k), dtype=torch.uint8, device=row_ptr.device)
    cm = torch.empty((n, k), dtype=torch.int32, device=row_ptr.device)
    _check(lib.lbdd_road_cost_matrix(V, row_ptr.data_ptr(), col.data_ptr(), length.data_ptr(), k,
                                     centers.data_ptr(), n, units.data_ptr(), cm.data_ptr(),
                                     work.data_ptr(), _stream_ptr(stream)))
    return cm


def solve_strict(cm, capacity, stream=None):
    """Solve one strict-LBDD instance (Appendix B); returns (objective of
    Equation (3), assignment as numpy int32 with -1 for units no center can
    hold)."""
    with Instance(cm, capacity, stream=stream, strict=True) as inst:
        inst.solve()
        return inst.objective(), inst.assignment()


def solve_batch(instances, stream=None):
    """Solve a list of Instances in one persistent launch (lbdd_solve_batch)."""
    lib = load()
    arr = (C.c_void_p * len(instances))(*[i._h.value for i in instances])
    _check(lib.lbdd_solve_batch(arr, len(instances), _stream_ptr(stream)))
    return instances


def best_transfers_work_bytes(k: int, n: int) -> int:
    return int(load().lbdd_best_transfers_work_bytes(int(k), int(n)))


SCAN_REUSE_GROUPING = 0x1


def best_transfers(cm, assign, rank, W=None, work=None, stream=None, reuse_grouping=False):
    """Best-transfer table of an allotment over the whole cost matrix.

    cm [n][k] int32, assign [n] int32, rank [n] int32: torch cuda tensors.
    Returns W as a torch int64 tensor [k][k] holding the uint64 key bits.
    reuse_grouping: `work` holds the grouping of the same assign/rank from a
    previous call; only the scan runs."""
    import torch
    n, k = cm.shape
    for t in (cm, assign, rank):
        if not (t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()):
            raise ValueError("cm, assign and rank must be contiguous int32 cuda tensors")
    if W is None:
        W = torch.empty((k, k), dtype=torch.int64, device=cm.device)
    if work is None:
        work = torch.empty(best_transfers_work_bytes(k, n), dtype=torch.uint8, device=cm.device)
    _check(load().lbdd_best_transfers(int(k), int(n), C.c_void_p(cm.data_ptr()),
                                      C.c_void_p(assign.data_ptr()), C.c_void_p(rank.data_ptr()),
                                      C.c_void_p(W.data_ptr()), C.c_void_p(work.data_ptr()),
                                      SCAN_REUSE_GROUPING if reuse_grouping else 0,
                                      _stream_ptr(stream)))
    return W


def read_ceiling(buf, sink, blocks: int, stream=None):
    """lbdd_read_ceiling over the bytes of the contiguous cuda tensor `buf`;
    sink is an 8-byte cuda tensor the fold is XORed into."""
    _check(load().lbdd_read_ceiling(C.c_void_p(buf.data_ptr()), int(buf.numel() * buf.element_size()),
                                    C.c_void_p(sink.data_ptr()), int(blocks), _stream_ptr(stream)))


NOALLOC_SCRATCH_BYTES = 16 << 20


def best_transfers_noalloc(cm, assign, rank, W, stream=None, reuse_grouping=False):
    """best_transfers through lbdd_best_transfers_noalloc: the workspace is
    the library's fixed per-GPU scratch and nothing is allocated (W, [k][k]
    int64 on the device, is the caller's).  reuse_grouping: the scratch holds
    the grouping of the same assign/rank from the last call on this GPU."""
    import torch
    n, k = cm.shape
    for t in (cm, assign, rank):
        if not (t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()):
            raise ValueError("cm, assign and rank must be contiguous int32 cuda tensors")
    if not (W.is_cuda and W.dtype == torch.int64 and W.is_contiguous() and W.numel() == k * k):
        raise ValueError("W must be a contiguous int64 cuda tensor of k*k entries")
    _check(load().lbdd_best_transfers_noalloc(int(k), int(n), C.c_void_p(cm.data_ptr()),
                                              C.c_void_p(assign.data_ptr()), C.c_void_p(rank.data_ptr()),
                                              C.c_void_p(W.data_ptr()),
                                              SCAN_REUSE_GROUPING if reuse_grouping else 0,
                                              _stream_ptr(stream)))
    return W


def best_transfers_batch_work_bytes(cms) -> int:
    ks = np.array([c.shape[1] for c in cms], np.int32)
    ns = np.array([c.shape[0] for c in cms], np.int64)
    return int(load().lbdd_best_transfers_batch_work_bytes(len(cms), ks.ctypes.data_as(C.c_void_p),
                                                           ns.ctypes.data_as(C.c_void_p)))


def best_transfers_batch(cms, assigns, ranks, Ws=None, work=None, stream=None, reuse_grouping=False):
    """Best-transfer tables of many allotments in one sequence of launches
    (lbdd_best_transfers_batch).  cms[i] [n_i][k_i], assigns[i], ranks[i] [n_i]:
    contiguous int32 torch cuda tensors.  Returns the list of tables (torch
    int64 [k_i][k_i] holding the uint64 key bits).  reuse_grouping: `work`
    holds the descriptors and groupings of a previous call with the same
    arguments; only the tables are cleared and the matrices scanned."""
    import torch
    m = len(cms)
    if not (m == len(assigns) == len(ranks)) or m == 0:
        raise ValueError("need the same positive number of cms, assigns and ranks")
    for t in (*cms, *assigns, *ranks):
        if not (t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()):
            raise ValueError("cm, assign and rank must be contiguous int32 cuda tensors")
    ks = np.array([c.shape[1] for c in cms], np.int32)
    ns = np.array([c.shape[0] for c in cms], np.int64)
    if reuse_grouping and (Ws is None or work is None):
        raise ValueError("reuse_grouping needs the tables and the work buffer of the earlier call")
    if Ws is None:
        Ws = [torch.empty((int(k), int(k)), dtype=torch.int64, device=cms[0].device) for k in ks]
    lib = load()
    if work is None:
        work = torch.empty(max(best_transfers_batch_work_bytes(cms), 1), dtype=torch.uint8,
                           device=cms[0].device)
    ptrs = [(C.c_void_p * m)(*[t.data_ptr() for t in ts]) for ts in (cms, assigns, ranks, Ws)]
    _check(lib.lbdd_best_transfers_batch(m, ks.ctypes.data_as(C.c_void_p), ns.ctypes.data_as(C.c_void_p),
                                         *[C.cast(p, C.c_void_p) for p in ptrs],
                                         C.c_void_p(work.data_ptr()),
                                         SCAN_REUSE_GROUPING if reuse_grouping else 0,
                                         _stream_ptr(stream)))
    return Ws


def tune_search(cm, capacity, penalty, iters: int, stream=None):
    """Autotune the search choice for this k on a prefix of `iters`
    iterations (lbdd_tune_search).  Returns (ratio, [ms per candidate]), the
    candidates being SEARCH_CANDIDATES."""
    k, n, ptr, flags, cap, pen, keep = _create_args(cm, capacity, penalty)
    ratio = C.c_int64()
    ms = (C.c_float * 8)()
    m = _check(load().lbdd_tune_search(k, n, ptr, cap.ctypes.data_as(C.c_void_p),
                                       pen.ctypes.data_as(C.c_void_p), flags, int(iters),
                                       _stream_ptr(stream), C.byref(ratio),
                                       C.cast(ms, C.c_void_p), 8))
    del keep
    return ratio.value, [float(ms[i]) for i in range(m)]


def tune_save(path: str, arch: str = None) -> int:
    """lbdd_tune_save: write this process's tuned choices to a JSON tuning
    cache, tagged with arch (None: the current device's)."""
    return _check(load().lbdd_tune_save(os.fsencode(path), arch.encode() if arch else None))


def tune_load(path: str, arch: str = None) -> int:
    """lbdd_tune_load: apply the cache's entries tuned on arch (None: the
    current device's); returns how many were applied."""
    return _check(load().lbdd_tune_load(os.fsencode(path), arch.encode() if arch else None))


def tune_clear():
    """lbdd_tune_clear: forget every tuned choice of this process."""
    load().lbdd_tune_clear()


def tune_best_transfers(cm, assign, rank, reps: int = 5, W=None, work=None, stream=None):
    """Autotune the whole-matrix scan's tiles for this k (lbdd_tune_best_transfers).
    Returns (W, (vec, lanes_per_row, groups_per_lane, waves), (default_ms, tuned_ms), count)."""
    import torch
    n, k = cm.shape
    for t in (cm, assign, rank):
        if not (t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()):
            raise ValueError("cm, assign and rank must be contiguous int32 cuda tensors")
    if W is None:
        W = torch.empty((k, k), dtype=torch.int64, device=cm.device)
    if work is None:
        work = torch.empty(best_transfers_work_bytes(k, n), dtype=torch.uint8, device=cm.device)
    cfg = (C.c_int32 * 4)()
    ms = (C.c_float * 2)()
    m = _check(load().lbdd_tune_best_transfers(int(k), int(n), C.c_void_p(cm.data_ptr()),
                                               C.c_void_p(assign.data_ptr()),
                                               C.c_void_p(rank.data_ptr()), C.c_void_p(W.data_ptr()),
                                               C.c_void_p(work.data_ptr()), int(reps),
                                               _stream_ptr(stream), C.cast(cfg, C.c_void_p),
                                               C.cast(ms, C.c_void_p)))
    return W, tuple(int(x) for x in cfg), (float(ms[0]), float(ms[1])), m


class Server:
    """Request server with continuous batching (lbdd_server_*).

    submit() keeps a reference to the cost matrix until the job's result has
    been taken with result()."""

    def __init__(self, hbm_budget: int = 64 << 30, max_jobs: int = 1024, reserve_cus: int = 64):
        self._lib = load()
        self._s = C.c_void_p()
        _check(self._lib.lbdd_server_create(int(hbm_budget), int(max_jobs), int(reserve_cus),
                                            C.byref(self._s)))
        self._keep = {}

    def submit(self, cm, capacity, penalty) -> int:
        cmh = _host_i32(cm)
        n, k = cmh.shape
        cap, pen = _host_i32(capacity), _host_i32(penalty)
        if cap.shape != (k,) or pen.shape != (k,):
            raise ValueError("capacity and penalty need k entries")
        t = C.c_uint64()
        _check(self._lib.lbdd_server_submit(self._s, int(k), int(n), cmh.ctypes.data_as(C.c_void_p),
                                            cap.ctypes.data_as(C.c_void_p),
                                            pen.ctypes.data_as(C.c_void_p), C.byref(t)))
        self._keep[t.value] = (cmh, n)
        return t.value

    def poll(self, ticket: int):
        st, obj = C.c_int32(), C.c_int64()
        _check(self._lib.lbdd_server_poll(self._s, int(ticket), C.byref(st), C.byref(obj)))
        return st.value, (obj.value if st.value == JOB_DONE else None)

    def wait(self, ticket: int) -> int:
        obj = C.c_int64()
        _check(self._lib.lbdd_server_wait(self._s, int(ticket), C.byref(obj)))
        return obj.value

    def result(self, ticket: int):
        """(allotment int32[n], times): submitted, admitted, finished in s since
        the server started; device clock at the first and the last iteration."""
        _, n = self._keep[ticket]
        a = np.empty(n, np.int32)
        times = np.zeros(5, np.float64)
        try:
            _check(self._lib.lbdd_server_result(self._s, int(ticket), a.ctypes.data_as(C.c_void_p),
                                                times.ctypes.data_as(C.c_void_p)))
        finally:
            self._keep.pop(ticket, None)
        return a, tuple(times)

    def cancel(self, ticket: int):
        """Take a job that is still waiting out of the queue (its state
        becomes E_CANCELLED); a running or finished job raises (E_STATE)."""
        _check(self._lib.lbdd_server_cancel(self._s, int(ticket)))

    def set_queue_timeout(self, seconds: float):
        """Jobs that wait longer than this for admission fail with E_TIMEOUT
        (0: no limit)."""
        _check(self._lib.lbdd_server_set_queue_timeout(self._s, float(seconds)))

    def stats(self) -> dict:
        out = np.zeros(len(SERVER_STATS), np.int64)
        m = _check(self._lib.lbdd_server_stats(self._s, out.ctypes.data_as(C.c_void_p), len(SERVER_STATS)))
        return {name: int(out[i]) for i, name in enumerate(SERVER_STATS[:m])}

    def close(self):
        if self._s:
            self._lib.lbdd_server_destroy(self._s)
            self._s = C.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
