#!/usr/bin/env python3
"""Benchmark: ASRAL solves of LBDD instances on one MI355X.

One step = one complete solve of the plain single-instance workload (k=100
centers, n=100,000 units, Gaussian-mixture demand, CM = Manhattan distance +
U{0..50}, capacities ~ local density with total 0.95 n, penalties
U{100..1000}): instance creation from the device-resident cost matrix (setup:
most suitable centers, processing order, row permutation), all n iterations
of allot / cycle refinement / path refinement / list updates, and the
objective and allotment read back.  The cost matrix is in HBM before timing.

Prints one JSON line.  Besides the contract's fields:
  parity        every timed step's objective and allotment hash against the
                stored oracle result
  roofline      the solve kernel (the step's dominant kernel): cost-matrix
                bytes per second against HBM peak, timed with HIP events on
                the stream it runs on; it is bound by dependent latency in one
                workgroup, not by bandwidth (bound "latency")
  c3            k=500, n=1,000,000 (2 GB of costs): one whole solve (--c3
                prefix: its first 300,000 iterations), timed with HIP events,
                allotment, loads and objective (and, for the prefix, the
                table) against the stored oracle result, and a bounded oracle
                sample beside it
  scan          the whole-matrix best-transfer scan at k=500, n=1,000,000
                with its own roofline (HBM-bound), next to a hand-written
                read-only streaming kernel and a torch copy as ceilings; the
                same scan on the two cache-resident plain workloads
                (effective rates)
  batch         the batched workload (256 instances) in one persistent launch
                vs plain solves one after another, with completion latencies
                and an instance-parallel oracle sample
  serve         the first requests of the serving trace (k log-uniform in
                [8, 500], n log-uniform in [2e3, 1e6], Poisson 50/s) through
                the request server vs plain FIFO solves
  cpu_baseline  the CPU oracle timed on this host for one whole solve of the
                step's instance
Optional sections (--extras): strict-LBDD, penalty tables, the road-network
workload, the threaded oracle and the search autotuner.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu() -> str:
    """The host's CPU model and logical core count."""
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} logical cores"


def host_workers() -> int:
    """Processes for instance-parallel oracle runs: the host's cores, at most
    16 (one GPU's share of a shared box)."""
    return max(1, min(16, os.cpu_count() or 1))


def recorded_traffic(kernel: str):
    """HBM bytes per launch of `kernel` on this benchmark's workload, from the
    committed counter summary (rocprofv3 FETCH_SIZE and WRITE_SIZE, scaled by
    the factors a plain elementwise kernel of known size gave), or None when
    the kernel's sources changed since the counters were taken."""
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
            rec = json.load(f)[kernel]
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
    except (OSError, KeyError, ValueError):
        return None
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return int(rec["fetch_bytes"]) + int(rec["write_bytes"])


def solve_bytes(k: int, stats: dict) -> int:
    """Algorithmic cost-matrix bytes of one solve: one CM row per allotment,
    the moved unit's row twice per move (it leaves one center's lists and
    joins another's), and per member row read by a list refill its list entry,
    its cost at the center and its cost at the refilled column."""
    return stats["iterations"] * 4 * k + stats["moves"] * 8 * k + stats["rows_scanned"] * 12


def sha_i32(a) -> str:
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()


def eq1(cm, cap, pen, a) -> int:
    """Equation (1) recomputed from an allotment (host, int64)."""
    import numpy as np
    ok = a >= 0
    total = int(cm[np.nonzero(ok)[0], a[ok]].astype(np.int64).sum())
    load = np.bincount(a[ok], minlength=cm.shape[1])
    return total + int((np.maximum(0, load - cap.astype(np.int64)) * pen.astype(np.int64)).sum())


def wait_event(ev, what, every=30.0):
    """Wait for a recorded event, logging every `every` seconds (a long solve
    is one launch; the log shows it is running)."""
    t0 = time.perf_counter()
    nxt = every
    while not ev.query():
        time.sleep(0.05)
        el = time.perf_counter() - t0
        if el >= nxt:
            log(f"bench: {what}: still running, {el:.0f} s")
            nxt += every


def pct(x, q):
    import numpy as np
    return round(float(np.percentile(np.asarray(x, dtype=np.float64), q)), 4)


# ------------------------------------------------------------ oracle samples
def _oracle_solve(args):
    """Worker of the instance-parallel CPU baseline: one whole oracle solve."""
    import oracle
    cm, cap, pen = args
    t = time.perf_counter()
    r = oracle.solve(cm, cap, pen)
    return r.objective, sha_i32(r.assign), time.perf_counter() - t


def oracle_parallel(insts):
    """The oracle on these instances, one per host process (instance-parallel:
    independent instances on the host's cores)."""
    import multiprocessing as mp
    cores = min(host_workers(), len(insts))
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = []
        for j, r in enumerate(pool.imap(_oracle_solve, [i.arrays() for i in insts])):
            res.append(r)
            log(f"bench: oracle sample: {j + 1}/{len(insts)} solved, {time.perf_counter() - t0:.1f} s")
    return res, time.perf_counter() - t0, cores


# ----------------------------------------------------------------- sections
def run_c3(mode, lbdd, L, torch, dev, stream, gold, prefix_sample, no_cpu):
    """The k=500, n=1,000,000 workload: one whole solve (mode "whole") or its
    first 300,000 iterations (mode "prefix"), timed with HIP events and
    checked against the stored oracle result."""
    t0 = time.perf_counter()
    inst = L.make_config("C3")
    cm = torch.from_numpy(inst.cm).to(dev)
    torch.cuda.synchronize()
    log(f"bench: c3 instance generated and copied in {time.perf_counter() - t0:.1f} s")
    gp = gold.get("C3_prefix")
    iters = inst.n if mode == "whole" else (gp["iterations"] if gp else 300_000)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    tw = time.perf_counter()
    h = lbdd.Instance(cm, inst.cap, inst.pen, stream=stream)
    e0.record(stream)
    h.solve_iters(iters)
    e1.record(stream)
    wait_event(e1, f"c3 {mode}")
    obj = h.objective()
    a = h.assignment()
    wall = time.perf_counter() - tw
    st = h.stats()
    load, W, _ = h.snapshot()
    h.close()
    solve_s = e0.elapsed_time(e1) / 1e3
    log(f"bench: c3 {iters} iterations {solve_s:.1f} s (wall {wall:.1f} s), objective {obj}")
    out = {"workload": "plain single instance k=500, n=1000000 (2 GB CM; Gaussian-mixture demand, "
                       "Manhattan CM + U{0..50}, capacities 0.9n with 10% of centers at half share, "
                       "penalties U{100..2000})",
           "iterations": iters, "whole_solve": iters == inst.n,
           "solve_s": round(solve_s, 3), "end_to_end_s": round(wall, 3),
           "iterations_per_s": round(iters / solve_s, 1),
           "solves_per_s": round(1.0 / solve_s, 5) if iters == inst.n else None,
           "objective": obj, "objective_is_equation_1": obj == eq1(inst.cm, inst.cap, inst.pen, a),
           "stats": st}
    g = gold.get("C3") if iters == inst.n else gp
    if g is not None:
        out["objective_matches_oracle"] = obj == g["objective"]
        out["assignment_matches_oracle"] = sha_i32(a) == g["assignment_sha256"]
        out["loads_match_oracle"] = load.tolist() == g["load"]
        if "table_sha256" in g:
            out["table_matches_oracle"] = hashlib.sha256(
                W.astype("<u8").tobytes()).hexdigest() == g["table_sha256"]
        out["oracle_s"] = g.get("oracle_seconds")
        out["oracle_build"] = g.get("oracle_build")
    else:
        out["objective_matches_oracle"] = None
    if not no_cpu:
        import oracle
        # bounded sample: the first `prefix_sample` iterations, on the oracle
        # (one thread) and on the GPU
        hs = lbdd.Instance(cm, inst.cap, inst.pen, stream=stream)
        e0.record(stream)
        hs.solve_iters(prefix_sample)
        e1.record(stream)
        g_obj = hs.objective()
        g_ms = e0.elapsed_time(e1)
        hs.close()
        tc = time.perf_counter()
        r = oracle.solve(*inst.arrays(), max_iters=prefix_sample)
        dt = time.perf_counter() - tc
        out["cpu_baseline"] = {
            "value": round(prefix_sample / dt, 1), "unit": "iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {prefix_sample} iterations of the same instance, setup included "
                      f"({dt:.1f} s); the GPU ran the same prefix at {prefix_sample / (g_ms / 1e3):.0f} "
                      f"iterations/s; objectives {'match' if r.objective == g_obj else 'DIFFER'}",
            "host": host_cpu()}
        log(f"bench: c3 oracle sample {dt:.1f} s for {prefix_sample} iterations")
    del cm
    return out


def run_scan(lbdd, L, torch, dev, stream, reps, tune):
    """The whole-matrix best-transfer scan at k=500, n=1,000,000 and its
    bandwidth ceilings."""
    log("bench: whole-matrix scan at k=500, n=1,000,000")
    big = L.make_config("C3")
    cmb = torch.from_numpy(big.cm).to(dev)
    # allotment: every unit at its cheapest center; rank: unit index
    assign = torch.argmin(cmb, dim=1).to(torch.int32).contiguous()
    rank = torch.arange(big.n, dtype=torch.int32, device=dev)
    W = torch.empty((big.k, big.k), dtype=torch.int64, device=dev)
    work = torch.empty(lbdd.best_transfers_work_bytes(big.k, big.n), dtype=torch.uint8, device=dev)
    lbdd.best_transfers(cmb, assign, rank, W, work, stream)
    torch.cuda.synchronize()
    tuned = None
    if tune:
        _, cfg, tms, ncfg = lbdd.tune_best_transfers(cmb, assign, rank, reps=3, W=W, work=work, stream=stream)
        tuned = {"configs_timed": ncfg, "chosen": {"cols_per_load": cfg[0], "lanes_per_row": cfg[1],
                                                   "groups_per_lane": cfg[2], "waves": cfg[3]},
                 "default_kernel_ms": round(tms[0], 4), "tuned_kernel_ms": round(tms[1], 4)}
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        lbdd.best_transfers(cmb, assign, rank, W, work, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    # the scan kernel alone (grouping of the same allotment reused): the
    # table clear plus one streaming pass over the cost matrix
    e0.record(stream)
    for _ in range(reps):
        lbdd.best_transfers(cmb, assign, rank, W, work, stream, reuse_grouping=True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_k = e0.elapsed_time(e1) / reps
    sbytes = big.n * (4 * big.k + 8 + 4 + 4) + big.k * big.k * 8
    kbytes = big.n * (4 * big.k + 8) + big.k * big.k * 8
    k_gbs = kbytes / (ms_k / 1e3) / 1e9
    out = {"workload": "k=500 n=1000000 whole-matrix best-transfer scan, every unit at its cheapest center",
           "ms": round(ms, 4), "bytes": sbytes, "achieved": round(sbytes / (ms / 1e3) / 1e9, 1),
           "unit": "GB/s", "kernel_ms": round(ms_k, 4), "kernel_bytes": kbytes,
           "roofline": {"bound": "hbm", "achieved": round(k_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(k_gbs / HBM_PEAK_GBS, 4), "traffic": recorded_traffic("scan_kernel"),
                        "kernel": "scan_kernel", "bytes_per_launch": kbytes,
                        "launch_ms": round(ms_k, 4)},
           "tune": tuned}
    log(f"bench: scan call {ms:.3f} ms; scan kernel {ms_k:.3f} ms -> {k_gbs:.0f} GB/s")
    del W, work, assign, rank
    # ceilings on the same 2 GB: a hand-written read-only streaming kernel
    # (lbdd_read_ceiling) and a torch device-to-device copy
    sink = torch.zeros(1, dtype=torch.int64, device=dev)
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    best = None
    for mult in (1, 2, 4, 8, 16):
        lbdd.read_ceiling(cmb, sink, cus * mult, stream)
        e0.record(stream)
        for _ in range(reps):
            lbdd.read_ceiling(cmb, sink, cus * mult, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        rms = e0.elapsed_time(e1) / reps
        if best is None or rms < best[1]:
            best = (mult, rms)
    nb = cmb.numel() * 4
    rgbs = nb / (best[1] / 1e3) / 1e9
    out["read_ceiling"] = {"kernel": "lbdd_read_ceiling: 16-byte nontemporal loads, eight in flight per "
                                     f"thread, one contiguous share per workgroup, {best[0]} workgroups "
                                     "of 256 per CU",
                           "bytes": nb, "ms": round(best[1], 4), "achieved": round(rgbs, 1),
                           "frac_of_peak": round(rgbs / HBM_PEAK_GBS, 4)}
    out["kernel_frac_of_read_ceiling"] = round(k_gbs / rgbs, 4)
    src = cmb.view(-1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    cms_ = e0.elapsed_time(e1) / reps
    copy_gbs = 2 * nb / (cms_ / 1e3) / 1e9
    out["copy_ceiling"] = {"kernel": "torch device-to-device copy of 2 GB (2 GB read + 2 GB written)",
                           "ms": round(cms_, 4), "achieved": round(copy_gbs, 1),
                           "frac_of_peak": round(copy_gbs / HBM_PEAK_GBS, 4)}
    log(f"bench: read ceiling {rgbs:.0f} GB/s, copy {copy_gbs:.0f} GB/s")
    del src, dst, cmb
    return out


def run_scan_cached(lbdd, L, torch, dev, stream, reps):
    """The whole-matrix scan on the two small plain workloads (k=8, n=2,000:
    64 KB of costs; k=100, n=100,000: 40 MB).  Their matrices fit in the L2
    or the last-level cache, so the rate is an effective one, not an HBM
    figure."""
    out = {}
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    for name in ("C1", "C2"):
        inst = L.make_config(name)
        cm = torch.from_numpy(inst.cm).to(dev)
        assign = torch.argmin(cm, dim=1).to(torch.int32).contiguous()
        rank = torch.arange(inst.n, dtype=torch.int32, device=dev)
        W = torch.empty((inst.k, inst.k), dtype=torch.int64, device=dev)
        work = torch.empty(lbdd.best_transfers_work_bytes(inst.k, inst.n), dtype=torch.uint8, device=dev)
        lbdd.best_transfers(cm, assign, rank, W, work, stream)
        e0.record(stream)
        for _ in range(reps):
            lbdd.best_transfers(cm, assign, rank, W, work, stream, reuse_grouping=True)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        kb = inst.n * (4 * inst.k + 8) + inst.k * inst.k * 8
        out[name] = {"k": inst.k, "n": inst.n, "bytes": kb, "kernel_ms": round(ms, 4),
                     "effective_gbs": round(kb / (ms / 1e3) / 1e9, 1),
                     "note": "cache-resident: effective rate, not HBM bandwidth"}
        log(f"bench: scan {name} (k={inst.k}, n={inst.n}): {ms:.4f} ms, effective {kb / (ms / 1e3) / 1e9:.0f} GB/s")
        del cm, assign, rank, W, work
    return out


def run_scan_batch(m, reps, lbdd, L, torch, dev, stream):
    """The batched scan over the first m instances of the batched workload
    (every unit at its cheapest center, rank = unit index)."""
    log(f"bench: batched scan over the first {m} instances of the batched workload")
    insts, cms = [], []
    for sp in L.batch_specs()[:m]:
        insts.append(L.make_batch_instance(sp))
        cms.append(torch.from_numpy(insts[-1].cm).to(dev))
        insts[-1].cm = None                            # the device copy is enough
    asg = [torch.argmin(c, dim=1).to(torch.int32).contiguous() for c in cms]
    rks = [torch.arange(i.n, dtype=torch.int32, device=dev) for i in insts]
    work = torch.empty(lbdd.best_transfers_batch_work_bytes(cms), dtype=torch.uint8, device=dev)
    Ws = lbdd.best_transfers_batch(cms, asg, rks, work=work, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        lbdd.best_transfers_batch(cms, asg, rks, Ws=Ws, work=work, stream=stream, reuse_grouping=True)
    e1.record(stream)
    torch.cuda.synchronize()
    kern_ms = e0.elapsed_time(e1) / reps
    kbytes = sum(i.n * (4 * i.k + 8) + 8 * i.k * i.k for i in insts)
    same = True
    for j in (0, m - 1):                              # spot check against the single scan
        W1 = lbdd.best_transfers(cms[j], asg[j], rks[j], stream=stream)
        same = same and bool(torch.equal(W1, Ws[j]))
    gbs = kbytes / (kern_ms / 1e3) / 1e9
    log(f"bench: batched scan streaming pass {kern_ms:.3f} ms -> {gbs:.0f} GB/s")
    return {"workload": f"first {m} instances of the batched workload, every unit at its cheapest center",
            "instances": m, "instances_with_16B_rows": sum(1 for i in insts if i.k % 4 == 0),
            "kernel_ms": round(kern_ms, 4), "kernel_bytes": kbytes, "kernel_achieved": round(gbs, 1),
            "kernel_frac": round(gbs / HBM_PEAK_GBS, 4),
            "kernel_traffic": recorded_traffic("bscan_kernel") if m == 16 else None,
            "tables_equal_single_scans": same}


def run_batch(m, m_plain, m_cpu, lbdd, L, torch, dev, gold, no_cpu):
    """The first m instances of the batched workload (k ~ U{16..256}, n
    log-uniform in [1e4, 2e5]): one lbdd_solve_batch launch against plain
    solves one after another (the first m_plain instances), on the same GPU
    and the same device inputs."""
    specs = L.batch_specs()[:m]
    t0 = time.perf_counter()
    insts, cms = [], []
    for sp in specs:
        insts.append(L.make_batch_instance(sp))
        cms.append(torch.from_numpy(insts[-1].cm).to(dev))
    torch.cuda.synchronize()
    log(f"bench: batch: {m} instances generated and copied in {time.perf_counter() - t0:.1f} s")
    # batched launch
    hs = [lbdd.Instance(c, i.cap, i.pen) for c, i in zip(cms, insts)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lbdd.solve_batch(hs)
    done = torch.cuda.Event()
    done.record(torch.cuda.current_stream(dev))
    wait_event(done, "batched launch")
    objs = [h.objective() for h in hs]
    bat_s = time.perf_counter() - t0
    shas = [sha_i32(h.assignment()) for h in hs]
    st = [h.stats() for h in hs]
    khz = st[0]["timer_khz"]
    first = min(x["tick_first"] for x in st)
    lat = [(x["tick_last"] - first) / (khz * 1e3) for x in st]
    own = [(x["tick_last"] - x["tick_first"]) / (khz * 1e3) for x in st]
    for h in hs:
        h.close()
    log(f"bench: batch: one launch {bat_s:.2f} s")
    # plain solves one after another
    t0 = time.perf_counter()
    plain_ok = True
    plain_s = []
    for j in range(m_plain):
        tj = time.perf_counter()
        with lbdd.Instance(cms[j], insts[j].cap, insts[j].pen) as h:
            h.solve()
            o = h.objective()
            plain_ok = plain_ok and o == objs[j] and sha_i32(h.assignment()) == shas[j]
        plain_s.append(time.perf_counter() - tj)
        if (j + 1) % 32 == 0:
            log(f"bench: batch: {j + 1} plain solves, {time.perf_counter() - t0:.1f} s")
    seq_s = time.perf_counter() - t0
    stored = {}
    for name, e in gold.items():
        if name.startswith("C4_") and "spec" in e and tuple(e["spec"]) in specs:
            j = specs.index(tuple(e["spec"]))
            stored[name] = objs[j] == e["objective"] and shas[j] == e["assignment_sha256"]
    out = {"workload": f"{m} instances of the batched workload (k~U{{16..256}}, n log-uniform [1e4,2e5])",
           "instances": m, "sum_nk": int(sum(i.n * i.k for i in insts)),
           "batched_s": round(bat_s, 3), "batched_solves_per_s": round(m / bat_s, 3),
           "batched_latency_from_launch_p50_s": pct(lat, 50),
           "batched_latency_from_launch_p99_s": pct(lat, 99),
           "largest_instance_own_s": round(max(own), 3),
           "plain_instances": m_plain, "plain_sequential_s": round(seq_s, 3),
           "plain_solves_per_s": round(m_plain / seq_s, 3),
           "plain_latency_p50_s": pct(plain_s, 50), "plain_latency_p99_s": pct(plain_s, 99),
           "speedup": round((m / bat_s) / (m_plain / seq_s), 2),
           "batched_equal_plain": plain_ok,
           "stored_oracle_instances_equal": stored}
    log(f"bench: batch {bat_s:.2f} s for {m} vs plain {seq_s:.2f} s for {m_plain}")
    if not no_cpu and m_cpu > 0:
        # bounded sample: the m_cpu instances of least n * k
        order = sorted(range(m), key=lambda j: insts[j].n * insts[j].k)[:m_cpu]
        res, wall, cores = oracle_parallel([insts[j] for j in order])
        ok = all(o == objs[j] and s == shas[j] for (o, s, _), j in zip(res, order))
        gpu_s = sum(plain_s[j] for j in order if j < m_plain)
        out["cpu_baseline"] = {
            "value": round(len(order) / wall, 4), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"the {len(order)} instances of least n*k, whole solves, one per process "
                      f"({wall:.1f} s wall, {sum(t for _, _, t in res):.1f} s of CPU); the GPU's "
                      f"plain solves of the same instances took {gpu_s:.2f} s in all",
            "results_equal_gpu": ok, "host": host_cpu()}
    del cms
    return out


def run_serve(count, m_cpu, lbdd, L, gold, no_cpu):
    """The first `count` requests of the serving trace (Poisson, mean gap
    20 ms; k log-uniform [8, 500], n log-uniform [2e3, 1e6]) replayed through
    the request server (continuous batching) and through plain FIFO solves,
    one at a time as they arrive; latency runs from arrival to result ready."""
    trace = L.serving_trace()[:count]
    t0 = time.perf_counter()
    insts = [L.make_batch_instance(sp) for _, sp in trace]
    log(f"bench: serve: {count} requests generated in {time.perf_counter() - t0:.1f} s")
    arr = [a for a, _ in trace]
    with lbdd.Server(hbm_budget=96 << 30, max_jobs=1024) as srv:
        t0 = time.perf_counter()
        tickets = []
        for a, inst in zip(arr, insts):
            d = a - (time.perf_counter() - t0)
            if d > 0:
                time.sleep(d)
            tickets.append(srv.submit(*inst.arrays()))
        lat, objs, shas = [], [], []
        for j, tk in enumerate(tickets):
            objs.append(srv.wait(tk))
            log(f"bench: serve: request {j + 1}/{count} served at {time.perf_counter() - t0:.1f} s")
            a, times = srv.result(tk)
            shas.append(sha_i32(a))
            lat.append(times[2] - times[0])
        span = time.perf_counter() - t0
        sst = srv.stats()
    log(f"bench: serve: served in {span:.1f} s; plain FIFO replay")
    t0 = time.perf_counter()
    flat, fok = [], True
    for j, (a, inst) in enumerate(zip(arr, insts)):
        d = a - (time.perf_counter() - t0)
        if d > 0:
            time.sleep(d)
        with lbdd.Instance(inst.cm, inst.cap, inst.pen) as h:
            h.solve()
            fok = fok and h.objective() == objs[j] and sha_i32(h.assignment()) == shas[j]
        flat.append((time.perf_counter() - t0) - a)
        log(f"bench: serve: FIFO request {j + 1}/{count} (k={inst.k}, n={inst.n}) done at "
            f"{time.perf_counter() - t0:.1f} s")
    fspan = time.perf_counter() - t0
    stored = {}
    specs = [sp for _, sp in trace]
    for name, e in gold.items():
        if name.startswith("C5_") and "spec" in e and tuple(e["spec"]) in specs:
            j = specs.index(tuple(e["spec"]))
            stored[name] = objs[j] == e["objective"] and shas[j] == e["assignment_sha256"]
    big = max(insts, key=lambda i: i.n * i.k)
    out = {"workload": f"first {count} requests of the serving trace: Poisson arrivals at 50/s, "
                       f"k log-uniform [8,500], n log-uniform [2000,1000000]",
           "requests": count, "largest_request": {"k": big.k, "n": big.n},
           "served_solves_per_s": round(count / span, 3),
           "served_latency_p50_s": pct(lat, 50), "served_latency_p99_s": pct(lat, 99),
           "fifo_solves_per_s": round(count / fspan, 3),
           "fifo_latency_p50_s": pct(flat, 50), "fifo_latency_p99_s": pct(flat, 99),
           "peak_jobs_on_device": sst["peak_jobs"], "served_equal_plain": fok,
           "stored_oracle_requests_equal": stored}
    log(f"bench: serve {span:.1f} s vs FIFO {fspan:.1f} s")
    if not no_cpu and m_cpu > 0:
        order = sorted(range(count), key=lambda j: insts[j].n * insts[j].k)[:m_cpu]
        res, wall, cores = oracle_parallel([insts[j] for j in order])
        ok = all(o == objs[j] and s == shas[j] for (o, s, _), j in zip(res, order))
        out["cpu_baseline"] = {
            "value": round(len(order) / wall, 4), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"the {len(order)} requests of least n*k, whole solves, one per process "
                      f"({wall:.1f} s wall, {sum(t for _, _, t in res):.1f} s of CPU)",
            "results_equal_gpu": ok, "host": host_cpu()}
    return out


def run_extras(args, lbdd, L, torch, dev, stream, cm, inst, gold):
    """Context sections: strict-LBDD, penalty tables and the road workload on
    the GPU, each checked against the oracle, and the threaded oracle."""
    import numpy as np
    import oracle
    out = {}
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)

    def timed(**kw):
        h = lbdd.Instance(cm, inst.cap, stream=stream, **kw)
        ev0.record(stream)
        h.solve()
        ev1.record(stream)
        o = h.objective()
        h.close()
        return o, ev0.elapsed_time(ev1)

    timed(strict=True)
    o, ms = timed(strict=True)
    tc = time.perf_counter()
    rs = oracle.solve_strict(inst.cm, inst.cap)
    dts = time.perf_counter() - tc
    out["strict"] = {"workload": "strict-LBDD (Appendix B, Algorithm 4) on the step's instance",
                     "solve_ms": round(ms, 3), "objective": o,
                     "objective_matches_oracle": o == gold["C2_strict"]["objective"] == rs.objective,
                     "cpu_baseline": {"value": round(1.0 / dts, 5), "unit": "solves/s", "cores": 1,
                                      "kind": "oracle", "sample": f"one whole solve ({dts:.1f} s)"}}
    g = gold["C2_table"]
    off, val = L.rising_penalties(inst, length=g["table_length"], seed=g["table_seed"])
    timed(pen_table=(off, val))
    o, ms = timed(pen_table=(off, val))
    out["penalty_table"] = {"workload": "the step's instance with rising penalty tables (Section 2, Equation (2))",
                            "solve_ms": round(ms, 3), "objective": o,
                            "objective_matches_oracle": o == g["objective"]}
    net = L.make_road_config("R1")
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)
    g_rp, g_col, g_len = t(net.row_ptr, np.int64), t(net.col, np.int32), t(net.length, np.int32)
    g_cen, g_units = t(net.centers, np.int32), t(net.units, np.int32)
    rwork = torch.empty(lbdd.load().lbdd_road_cm_work_bytes(net.V, net.k), dtype=torch.uint8, device=dev)
    rcm = lbdd.road_cost_matrix(g_rp, g_col, g_len, g_cen, g_units, work=rwork, stream=stream)
    torch.cuda.synchronize()
    tc = time.perf_counter()
    for _ in range(5):
        rcm = lbdd.road_cost_matrix(g_rp, g_col, g_len, g_cen, g_units, work=rwork, stream=stream)
    torch.cuda.synchronize()
    cm_ms = (time.perf_counter() - tc) * 1e3 / 5
    h = lbdd.Instance(rcm, net.cap, net.pen, stream=stream)
    ev0.record(stream)
    h.solve()
    ev1.record(stream)
    robj = h.objective()
    rms = ev0.elapsed_time(ev1)
    h.close()
    cm_ref = oracle.road_cm(net.row_ptr, net.col, net.length, net.centers, net.units)
    out["road"] = {"workload": "R1: road-like network of 65,902 vertices, 131 centers, a unit on every "
                               "other vertex, total capacity 0.7n, penalties U{1..200}",
                   "cost_matrix_ms": round(cm_ms, 3), "solve_ms": round(rms, 3), "objective": robj,
                   "cost_matrix_matches_oracle": bool(np.array_equal(rcm.cpu().numpy(), cm_ref)),
                   "objective_matches_oracle": oracle.solve(cm_ref, net.cap, net.pen).objective == robj}
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    tc = time.perf_counter()
    rp = oracle.solve(*inst.arrays(), lib=oracle.load_para())
    dtp = time.perf_counter() - tc
    out["para_oracle"] = {"value": round(1.0 / dtp, 5), "unit": "solves/s", "cores": threads,
                          "kind": "para-ASRAL-style threaded oracle (OpenMP, same results)",
                          "objective_matches": rp.objective == gold["C2"]["objective"]}
    if args.tune:
        ratio, cand_ms = lbdd.tune_search(cm, inst.cap, inst.pen, iters=inst.n, stream=stream)
        out["tune_search"] = {"k": inst.k, "chosen_ratio_x16": ratio,
                              "candidates_ratio_x16": list(lbdd.SEARCH_CANDIDATES),
                              "candidates_ms": [round(x, 3) for x in cand_ms]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip every oracle timing")
    ap.add_argument("--c3", choices=("whole", "prefix", "skip"), default="whole",
                    help="k=500, n=1,000,000: one whole solve, or its first 300,000 iterations")
    ap.add_argument("--c3-cpu-iters", type=int, default=5000,
                    help="iterations of the k=500 instance in the bounded oracle sample")
    ap.add_argument("--no-scan", action="store_true")
    ap.add_argument("--scan-reps", type=int, default=10)
    ap.add_argument("--scan-batch", type=int, default=16,
                    help="instances of the batched workload scanned together by the batched scan (0: skip)")
    ap.add_argument("--batch", type=int, default=256,
                    help="instances of the batched workload solved in one launch (0: skip)")
    ap.add_argument("--batch-plain", type=int, default=64,
                    help="of those, how many (the first) are also solved plainly one after another")
    ap.add_argument("--batch-cpu", type=int, default=16,
                    help="instances (least n*k) in the instance-parallel oracle sample")
    ap.add_argument("--serve", type=int, default=40,
                    help="requests of the serving trace to serve vs plain FIFO (0: skip)")
    ap.add_argument("--serve-cpu", type=int, default=16,
                    help="requests (least n*k) in the instance-parallel oracle sample")
    ap.add_argument("--extras", action="store_true",
                    help="also strict-LBDD, penalty tables, the road workload and the threaded oracle")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the scan's tiles (and, with --extras, the search choice)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one 1 GiB elementwise kernel (HBM counter calibration)")
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
        gold = json.load(f)
    g2 = gold["C2"]

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)

    def step():
        h = lbdd.Instance(cm, inst.cap, inst.pen, stream=stream)
        ev0.record(stream)
        h.solve()
        ev1.record(stream)
        obj = h.objective()
        a = h.assignment()
        st = h.stats()
        h.close()
        return obj, a, st, ev0.elapsed_time(ev1)

    log(f"bench: k={inst.k} n={inst.n}: warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    solve_ms, results, stats = [], [], None
    log(f"bench: timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        obj, a, stats, ms = step()
        results.append((obj, a))
        solve_ms.append(ms)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    obj_ok = all(o == g2["objective"] for o, _ in results)
    sha_ok = all(sha_i32(a) == g2["assignment_sha256"] for _, a in results)
    log(f"bench: {ms_per_step:.1f} ms/step, solve kernel median {np.median(solve_ms):.1f} ms, "
        f"parity objective {obj_ok} allotment {sha_ok}")
    # end to end from a host cost matrix (PCIe copy included): context only
    tc = time.perf_counter()
    h = lbdd.Instance(inst.cm, inst.cap, inst.pen, stream=stream)
    h.solve()
    e2e_obj = h.objective()
    h.assignment()
    h.close()
    e2e_ms = (time.perf_counter() - tc) * 1e3

    nbytes = solve_bytes(inst.k, stats)
    kern_s = float(np.median(solve_ms)) / 1e3
    achieved = nbytes / kern_s / 1e9
    roofline = {"bound": "latency", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
                "traffic": recorded_traffic("solve_kernel"),
                "kernel": "solve_kernel", "bytes_per_launch": nbytes,
                "launch_ms": round(kern_s * 1e3, 3),
                "limited_by": "dependent latency: one persistent workgroup runs the n iterations "
                              "(barriers, LDS and L2 round trips of the searches); the HBM figure "
                              "is given for reference, the HBM-bound kernel is the scan (scan.roofline)"}

    c3 = (run_c3(args.c3, lbdd, L, torch, dev, stream, gold, args.c3_cpu_iters, args.no_cpu_baseline)
          if args.c3 != "skip" else None)
    scan = None
    if not args.no_scan:
        scan = run_scan(lbdd, L, torch, dev, stream, args.scan_reps, args.tune)
        scan["cache_resident"] = run_scan_cached(lbdd, L, torch, dev, stream, args.scan_reps)
        if args.scan_batch > 0:
            scan["batch"] = run_scan_batch(args.scan_batch, args.scan_reps, lbdd, L, torch, dev, stream)
    if args.copy_calib:
        # plain elementwise kernel of known traffic: reads 1 GiB, writes 1 GiB
        src = torch.empty(1 << 28, dtype=torch.int32, device=dev)
        src.fill_(1)
        torch.cuda.synchronize()
        dst = src + 1
        torch.cuda.synchronize()
        log("bench: 1 GiB read + 1 GiB write kernel done (counter calibration)")
        del src, dst
    batch = (run_batch(args.batch, min(args.batch_plain, args.batch), args.batch_cpu, lbdd, L, torch, dev,
                       gold, args.no_cpu_baseline) if args.batch > 0 else None)
    serve = run_serve(args.serve, args.serve_cpu, lbdd, L, gold, args.no_cpu_baseline) if args.serve > 0 else None
    extras = run_extras(args, lbdd, L, torch, dev, stream, cm, inst, gold) if args.extras else None

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log("bench: CPU oracle, one whole solve of the step's instance (single thread)")
        tc = time.perf_counter()
        r = oracle.solve(*inst.arrays())
        dt = time.perf_counter() - tc
        cpu = {"value": round(1.0 / dt, 5), "unit": "solves/s", "cores": 1, "kind": "oracle",
               "sample": f"one whole solve of the k=100 n=100000 instance ({dt:.1f} s); "
                         f"objective {'matches' if r.objective == g2['objective'] else 'DIFFERS'}",
               "host": host_cpu()}
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
        "parity": {"objective_matches_oracle": obj_ok, "assignment_matches_oracle": sha_ok,
                   "steps_checked": args.steps, "objective": results[-1][0]},
        "solve_ms_median": round(float(np.median(solve_ms)), 3),
        "end_to_end_host_cm": {"ms": round(e2e_ms, 3), "objective_matches_oracle": e2e_obj == g2["objective"],
                               "what": "create from a host CM (PCIe copy) + setup + solve + objective "
                                       "and allotment read back"},
        "stats": stats,
        "roofline": roofline,
        "c3": c3,
        "scan": scan,
        "batch": batch,
        "serve": serve,
        "extras": extras,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
