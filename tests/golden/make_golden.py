"""Write the stored oracle results used by the GPU parity tests.

    python -m tests.golden.make_golden

Calls only the CPU oracle (oracle/) and the input generators (lbdd_inputs).
For each workload it records the input hash, the objective, a sha256 of the
int32 allotment (one center per unit, little-endian) and the oracle's counters.
"""
import hashlib
import json
import os
import time

import numpy as np

import lbdd_inputs as L
import oracle

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_results.json")


def assignment_hash(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()


def main():
    res = {}
    for name in ("C1", "C2"):
        inst = L.make_config(name)
        t = time.time()
        r = oracle.solve(*inst.arrays())
        dt = time.time() - t
        res[name] = dict(
            k=inst.k, n=inst.n, input_sha256=L.input_hash(inst), objective=r.objective,
            assignment_sha256=assignment_hash(r.assign),
            assignment_head=r.assign[:16].tolist(),
            load=r.load.tolist() if inst.k <= 128 else None,
            stats=dict(zip(["cycles", "paths", "moves", "cycle_searches", "path_searches",
                            "bf_rounds", "heap_pushes", "iterations"], r.stats.tolist())),
            oracle_seconds=round(dt, 2))
        print(name, res[name]["objective"], dt, flush=True)
    # strict-LBDD (Appendix B) on the same capacities: excess demand, so the
    # dummy center takes n - sum(capacity) units
    for name in ("C1", "C2"):
        inst = L.make_config(name)
        t = time.time()
        r = oracle.solve_strict(inst.cm, inst.cap)
        dt = time.time() - t
        res[name + "_strict"] = dict(
            k=inst.k, n=inst.n, input_sha256=L.input_hash(inst), objective=r.objective,
            assignment_sha256=assignment_hash(r.assign), kx=r.kx,
            unallotted=int((r.assign < 0).sum()),
            load=r.load.tolist() if r.kx <= 129 else None,
            stats=dict(zip(["cycles", "paths", "moves", "cycle_searches", "path_searches",
                            "bf_rounds", "heap_pushes", "iterations"], r.stats.tolist())),
            oracle_seconds=round(dt, 2))
        print(name + "_strict", r.objective, dt, flush=True)
    # general penalty functions (the definition in Section 2, Equation (2)) on
    # C2: tables that start at the constant penalties and rise by U{0..20} per
    # further unit beyond capacity, 2,000 values per center
    inst = L.make_config("C2")
    off, val = L.rising_penalties(inst, length=2000, seed=2)
    t = time.time()
    r = oracle.solve_q(inst.cm, inst.cap, off, val)
    dt = time.time() - t
    res["C2_table"] = dict(
        k=inst.k, n=inst.n, input_sha256=L.input_hash(inst), table_length=2000, table_seed=2,
        objective=r.objective, assignment_sha256=assignment_hash(r.assign),
        stats=dict(zip(["cycles", "paths", "moves", "cycle_searches", "path_searches",
                        "bf_rounds", "heap_pushes", "iterations"], r.stats.tolist())),
        oracle_seconds=round(dt, 2))
    print("C2_table", r.objective, dt, flush=True)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
