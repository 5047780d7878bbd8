#!/usr/bin/env python3
"""Benchmark: whole ASRAL solves of one LBDD instance on one MI355X.

One step = one complete solve of the plain single-instance workload
(k=100 centers, n=100,000 units, Gaussian-mixture demand, CM = Manhattan
distance + noise, capacities ~ local density with total 0.95 n, penalties
U{100..1000}): setup (most suitable centers, processing order, row
permutation) and all n iterations of allot / cycle refinement / path
refinement / rescans, then the objective read back.  The cost matrix is
resident in HBM (a torch tensor) before timing starts.

Prints one JSON line.  Extra objects:
  roofline      the solve kernel's cost-matrix bytes per second against HBM
                peak, timed with HIP events on the stream it runs on
  scan          the whole-matrix best-transfer scan at k=500, n=1,000,000
                (2 GB of costs) against HBM peak
  cpu_baseline  the CPU oracle timed on this host for one whole solve
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def solve_bytes(k: int, iters: int, rows_scanned: int) -> int:
    """Algorithmic cost-matrix bytes of one solve: one CM row per allotment
    plus, per rescanned member row, the row and its member-list entry."""
    return iters * 4 * k + rows_scanned * (4 * k + 4)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-scan", action="store_true")
    ap.add_argument("--scan-reps", type=int, default=10)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              f"(independent instances would be placed on separate GPUs with no exchange)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import lbdd_inputs as L
    from paper_2304_06543_amd import lbdd

    lbdd.load()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    inst = L.make_config("C2")
    cm = torch.from_numpy(inst.cm).to(dev)
    torch.cuda.synchronize()
    with open(os.path.join(ROOT, "tests", "golden", "oracle_results.json")) as f:
        gold = json.load(f)["C2"]

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)

    def step():
        inst_h = lbdd.Instance(cm, inst.cap, inst.pen, stream=stream)
        ev0.record(stream)
        inst_h.solve()
        ev1.record(stream)
        obj = inst_h.objective()
        st = inst_h.stats()
        inst_h.close()
        return obj, st, ev0.elapsed_time(ev1)

    log(f"bench: C2 k={inst.k} n={inst.n}: warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    solve_ms, objs, stats = [], [], None
    log(f"bench: timing {args.steps} steps")
    t0 = time.perf_counter()
    for i in range(args.steps):
        obj, stats, ms = step()
        objs.append(obj)
        solve_ms.append(ms)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    parity = all(o == gold["objective"] for o in objs)
    log(f"bench: {ms_per_step:.1f} ms/step, solve kernel {np.mean(solve_ms):.1f} ms, "
        f"objective parity {parity}, stats {stats}")

    nbytes = solve_bytes(inst.k, stats["iterations"], stats["rows_scanned"])
    kern_s = float(np.mean(solve_ms)) / 1e3
    achieved = nbytes / kern_s / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                "kernel": "solve_kernel", "bytes_per_launch": nbytes,
                "launch_ms": round(kern_s * 1e3, 3)}

    scan = None
    if not args.no_scan:
        log("bench: whole-matrix scan at k=500, n=1,000,000")
        big = L.make_config("C3")
        cmb = torch.from_numpy(big.cm).to(dev)
        # allotment: every unit at its cheapest center; rank: unit index
        assign = torch.argmin(cmb, dim=1).to(torch.int32).contiguous()
        rank = torch.arange(big.n, dtype=torch.int32, device=dev)
        W = torch.empty((big.k, big.k), dtype=torch.int64, device=dev)
        work = torch.empty(lbdd.best_transfers_work_bytes(big.k, big.n), dtype=torch.uint8,
                           device=dev)
        lbdd.best_transfers(cmb, assign, rank, W, work, stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.scan_reps):
            lbdd.best_transfers(cmb, assign, rank, W, work, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.scan_reps
        sbytes = big.n * (4 * big.k + 8 + 4 + 4) + big.k * big.k * 8
        scan = {"workload": "k=500 n=1000000 whole-matrix best-transfer scan",
                "ms": round(ms, 4), "bytes": sbytes,
                "achieved": round(sbytes / (ms / 1e3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(sbytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"bench: scan {ms:.3f} ms -> {scan['achieved']} GB/s")
        del cmb, W, work

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log("bench: CPU oracle, one whole solve of the same instance (single thread)")
        tc = time.perf_counter()
        r = oracle.solve(*inst.arrays())
        dt = time.perf_counter() - tc
        cpu = {"value": round(1.0 / dt, 5), "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": f"one whole solve of the k=100 n=100000 instance ({dt:.1f} s); "
                         f"objective {'matches' if r.objective == gold['objective'] else 'DIFFERS'}"}
        log(f"bench: oracle {dt:.1f} s")

    out = {
        "metric": "cost-matrix GB/s (% HBM peak); LBDD solves/sec and p99 latency, batched vs plain",
        "value": round(args.steps / (t1 - t0), 4),
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": "plain single-instance ASRAL solve, k=100 centers, n=100000 units "
                               "(Gaussian-mixture demand, Manhattan CM + U{0..50}, density "
                               "capacities total 0.95n, penalties U{100..1000})",
                   "k": inst.k, "n": inst.n, "parallelism": "one instance per GPU"},
        "parity": {"objective_matches_oracle": parity, "objective": objs[-1]},
        "stats": stats,
        "roofline": roofline,
        "scan": scan,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
