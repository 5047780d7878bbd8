"""Write the stored oracle results used by the GPU parity tests.

    python -m tests.golden.make_golden                 # C1, C2, strict, tables
    python -m tests.golden.make_golden C4 C5 C3        # the large workloads

Calls only the CPU oracle (oracle/) and the input generators (lbdd_inputs).
For each workload it records the input hash, the objective, a sha256 of the
int32 allotment (one center per unit, little-endian) and the oracle's counters.
The large workloads (the k=500, n=1,000,000 instance, instances of the batched
and of the serving workload) run on the OpenMP build of the same source, whose
results are identical to the plain build's; for the k=500 instance a prefix of
300,000 iterations is stored too, with its loads and a sha256 of its
best-transfer table (uint64 [k][k], little-endian).  Results are merged into
oracle_results.json by name, so groups can be written by separate runs.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

import lbdd_inputs as L
import oracle

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_results.json")
STAT_NAMES = ["cycles", "paths", "moves", "cycle_searches", "path_searches",
              "bf_rounds", "heap_pushes", "iterations"]

# instances of the batched workload (index into batch_specs()) and of the
# serving trace (index into serving_trace()) whose results are stored: k from
# 8 to 462, n up to 5.3e5, the largest k whose table stays in LDS (135) and
# the smallest beyond it (136), several more with the table in global memory,
# and the largest request among the first 40 of the trace (28)
BATCH_IDS = (7, 0, 3, 17, 28, 49, 53, 233)
SERVE_IDS = (2, 9, 14, 37, 28, 32, 29, 36)
C3_PREFIX = 300_000


def assignment_hash(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()


def table_hash(W: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(W, dtype="<u8").tobytes()).hexdigest()


def _save(name, entry):
    res = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            res = json.load(f)
    res[name] = entry
    with open(OUT + ".tmp", "w") as f:
        json.dump(res, f, indent=1)
    os.replace(OUT + ".tmp", OUT)


def _plain_entry(inst, r, dt, lib_name):
    return dict(k=inst.k, n=inst.n, input_sha256=L.input_hash(inst), objective=r.objective,
                assignment_sha256=assignment_hash(r.assign),
                assignment_head=r.assign[:16].tolist(),
                load=r.load.tolist() if inst.k <= 128 else None,
                stats=dict(zip(STAT_NAMES, r.stats.tolist())),
                oracle_seconds=round(dt, 2), oracle_build=lib_name)


def base():
    for name in ("C1", "C2"):
        inst = L.make_config(name)
        t = time.time()
        r = oracle.solve(*inst.arrays())
        dt = time.time() - t
        _save(name, _plain_entry(inst, r, dt, "plain"))
        print(name, r.objective, dt, flush=True)
    # strict-LBDD (Appendix B) on the same capacities: excess demand, so the
    # dummy center takes n - sum(capacity) units
    for name in ("C1", "C2"):
        inst = L.make_config(name)
        t = time.time()
        r = oracle.solve_strict(inst.cm, inst.cap)
        dt = time.time() - t
        _save(name + "_strict", dict(
            k=inst.k, n=inst.n, input_sha256=L.input_hash(inst), objective=r.objective,
            assignment_sha256=assignment_hash(r.assign), kx=r.kx,
            unallotted=int((r.assign < 0).sum()),
            load=r.load.tolist() if r.kx <= 129 else None,
            stats=dict(zip(STAT_NAMES, r.stats.tolist())),
            oracle_seconds=round(dt, 2)))
        print(name + "_strict", r.objective, dt, flush=True)
    # general penalty functions (the definition in Section 2, Equation (2)) on
    # C2: tables that start at the constant penalties and rise by U{0..20} per
    # further unit beyond capacity, 2,000 values per center
    inst = L.make_config("C2")
    off, val = L.rising_penalties(inst, length=2000, seed=2)
    t = time.time()
    r = oracle.solve_q(inst.cm, inst.cap, off, val)
    dt = time.time() - t
    _save("C2_table", dict(
        k=inst.k, n=inst.n, input_sha256=L.input_hash(inst), table_length=2000, table_seed=2,
        objective=r.objective, assignment_sha256=assignment_hash(r.assign),
        stats=dict(zip(STAT_NAMES, r.stats.tolist())),
        oracle_seconds=round(dt, 2)))
    print("C2_table", r.objective, dt, flush=True)


def _solve_para(inst, name, **kw):
    lib = oracle.load_para()
    t = time.time()
    r = oracle.solve(*inst.arrays(), lib=lib, **kw)
    dt = time.time() - t
    print(name, inst.k, inst.n, r.objective, round(dt, 1), flush=True)
    return r, dt


def batch():
    specs = L.batch_specs()
    for j in BATCH_IDS:
        inst = L.make_batch_instance(specs[j])
        r, dt = _solve_para(inst, f"C4_{j}")
        e = _plain_entry(inst, r, dt, "openmp")
        e["spec"] = list(specs[j])
        _save(f"C4_{j}", e)


def serve():
    trace = L.serving_trace()
    for j in SERVE_IDS:
        spec = trace[j][1]
        inst = L.make_batch_instance(spec)
        r, dt = _solve_para(inst, f"C5_{j}")
        e = _plain_entry(inst, r, dt, "openmp")
        e["spec"] = list(spec)
        _save(f"C5_{j}", e)


def c3():
    inst = L.make_config("C3")
    r, dt = _solve_para(inst, "C3_prefix", max_iters=C3_PREFIX, want_W=True)
    e = _plain_entry(inst, r, dt, "openmp")
    e.update(iterations=C3_PREFIX, load=r.load.tolist(), table_sha256=table_hash(r.W))
    _save("C3_prefix", e)
    r, dt = _solve_para(inst, "C3")
    e = _plain_entry(inst, r, dt, "openmp")
    e["load"] = r.load.tolist()
    _save("C3", e)


GROUPS = {"base": base, "C4": batch, "C5": serve, "C3": c3}


def main(argv):
    for g in (argv or ["base"]):
        GROUPS[g]()


if __name__ == "__main__":
    main(sys.argv[1:])
