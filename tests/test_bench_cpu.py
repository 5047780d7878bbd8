"""Host-side checks of bench.py that need no GPU: it measures one GPU only,
and its recorded HBM traffic follows the kernels' sources."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in p.stderr


def test_recorded_traffic_follows_sources():
    """Every kernel in profiles/traffic.json has its counter summary, and
    bench.py reports its recorded traffic exactly when the kernel's sources
    still hash to those the counters were taken from (else null)."""
    import hashlib
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        rec = json.load(f)
    for kernel in ("solve_kernel", "scan_kernel", "bscan_kernel"):
        assert kernel in rec
        assert os.path.exists(os.path.join(ROOT, rec[kernel]["summary"]))
        h = hashlib.sha256()
        for src in rec[kernel]["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        fresh = h.hexdigest() == rec[kernel]["sources_sha256"]
        expect = rec[kernel]["fetch_bytes"] + rec[kernel]["write_bytes"] if fresh else None
        assert bench.recorded_traffic(kernel) == expect


def test_recorded_traffic_is_null_for_changed_sources(tmp_path, monkeypatch):
    """A kernel whose source no longer matches gets no traffic figure."""
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        rec = json.load(f)
    rec["solve_kernel"]["sources_sha256"] = "0" * 64
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic.json").write_text(json.dumps(rec))
    for src in rec["solve_kernel"]["sources"]:
        d = tmp_path / os.path.dirname(src)
        d.mkdir(parents=True, exist_ok=True)
        (tmp_path / src).write_bytes(open(os.path.join(ROOT, src), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic("solve_kernel") is None


def test_stored_results_hold_what_the_bench_checks():
    """Every objective bench.py compares against is stored, with the table
    parameters the penalty-table step rebuilds its inputs from."""
    with open(os.path.join(ROOT, "tests", "golden", "oracle_results.json")) as f:
        gold = json.load(f)
    for name in ("C2", "C2_strict", "C2_table"):
        assert isinstance(gold[name]["objective"], int)
    assert gold["C2_table"]["table_length"] > 0 and "table_seed" in gold["C2_table"]
    assert gold["C2_table"]["input_sha256"] == gold["C2"]["input_sha256"]
