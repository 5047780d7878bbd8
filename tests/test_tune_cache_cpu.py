"""The tuning cache (lbdd_tune_save / lbdd_tune_load / lbdd_tune_clear) on the
CPU: these calls launch no device work when the architecture is named, so
the round trip, the architecture filter and the rejection of bad files are
checked here; that a loaded choice leaves results unchanged is a GPU test."""
import json
import os

import pytest

from paper_2304_06543_amd import lbdd

GOOD = {"format": "lbdd-tune-1", "entries": [
    {"arch": "gfx950", "kind": "search", "k_bucket": 7, "n_bucket": 5, "ratio": 0},
    {"arch": "gfx950", "kind": "search", "k_bucket": 9, "n_bucket": 6, "ratio": -1},
    {"arch": "gfx950", "kind": "scan", "k": 500, "vec4": 1, "config": [4, 64, 2, 2]},
    {"arch": "gfx942", "kind": "search", "k_bucket": 7, "n_bucket": 5, "ratio": 1048576},
    {"arch": "gfx942", "kind": "scan", "k": 100, "vec4": 0, "config": [1, 64, 2, 1]},
]}


@pytest.fixture
def lib(tmp_path):
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2304_06543_amd", "liblbdd.so")
    if not os.path.exists(path):
        pytest.skip("library not built")
    lbdd.load()
    lbdd.tune_clear()
    yield lbdd
    lbdd.tune_clear()


def _write(tmp_path, obj, name="cache.json"):
    p = tmp_path / name
    p.write_text(obj if isinstance(obj, str) else json.dumps(obj))
    return str(p)


def _entries(path):
    with open(path) as f:
        d = json.load(f)
    assert d["format"] == "lbdd-tune-1"
    return sorted(json.dumps(e, sort_keys=True) for e in d["entries"])


def test_round_trip_keeps_the_entries_of_one_architecture(lib, tmp_path):
    src = _write(tmp_path, GOOD)
    assert lib.tune_load(src, "gfx950") == 3
    out = str(tmp_path / "out.json")
    assert lib.tune_save(out, "gfx950") == 3
    want = sorted(json.dumps(e, sort_keys=True) for e in GOOD["entries"] if e["arch"] == "gfx950")
    assert _entries(out) == want
    assert not os.path.exists(out + ".tmp")
    # the other architecture's entries, alone
    lib.tune_clear()
    assert lib.tune_load(src, "gfx942") == 2
    assert lib.tune_save(out, "gfx942") == 2
    assert len(_entries(out)) == 2


def test_clear_forgets_everything(lib, tmp_path):
    lib.tune_load(_write(tmp_path, GOOD), "gfx950")
    lib.tune_clear()
    out = str(tmp_path / "empty.json")
    assert lib.tune_save(out, "gfx950") == 0
    assert _entries(out) == []
    assert lib.tune_load(out, "gfx950") == 0


@pytest.mark.parametrize("bad", [
    "not json",
    "{\"format\": \"lbdd-tune-1\", \"entries\": []} trailing",
    {"format": "other", "entries": []},
    {"format": "lbdd-tune-1"},
    {"format": "lbdd-tune-1", "entries": [{"arch": "gfx950", "kind": "search", "k_bucket": 13,
                                           "n_bucket": 5, "ratio": 0}]},
    {"format": "lbdd-tune-1", "entries": [{"arch": "gfx950", "kind": "search", "k_bucket": 7,
                                           "n_bucket": 5, "ratio": 1.5}]},
    {"format": "lbdd-tune-1", "entries": [{"arch": "gfx950", "kind": "search", "k_bucket": 7,
                                           "n_bucket": 5, "ratio": -2}]},
    {"format": "lbdd-tune-1", "entries": [{"arch": "gfx950", "kind": "scan", "k": 500, "vec4": 1,
                                           "config": [4, 16, 1, 1]}]},        # 64 columns < k
    {"format": "lbdd-tune-1", "entries": [{"arch": "gfx950", "kind": "scan", "k": 100, "vec4": 1,
                                           "config": [1, 64, 2, 1]}]},        # width mismatch
    {"format": "lbdd-tune-1", "entries": [{"arch": "gfx950", "kind": "scan", "k": 100, "vec4": 0,
                                           "config": [1, 64, 3, 1]}]},        # no such shape
    {"format": "lbdd-tune-1", "entries": [{"arch": "gfx950", "kind": "other"}]},
    {"format": "lbdd-tune-1", "entries": [{"kind": "search"}]},
])
def test_bad_files_change_nothing(lib, tmp_path, bad):
    good = GOOD["entries"][0]
    lib.tune_load(_write(tmp_path, {"format": "lbdd-tune-1", "entries": [good]}, "g.json"), "gfx950")
    # a valid entry for the same bucket ahead of the bad one: not applied either
    other = {**good, "ratio": 64}
    if not isinstance(bad, str) and "entries" in bad:
        bad = {**bad, "entries": [other] + bad["entries"]}
    with pytest.raises(lbdd.LbddError) as e:
        lib.tune_load(_write(tmp_path, bad), "gfx950")
    assert e.value.code == lbdd.E_INVAL
    out = str(tmp_path / "after.json")
    assert lib.tune_save(out, "gfx950") == 1               # only the good entry, from before
    assert _entries(out) == [json.dumps(good, sort_keys=True)]


def test_missing_file_and_null_path(lib, tmp_path):
    with pytest.raises(lbdd.LbddError):
        lib.tune_load(str(tmp_path / "none.json"), "gfx950")
    with pytest.raises(lbdd.LbddError):
        lib.tune_save(str(tmp_path / "no_dir" / "x.json"), "gfx950")


def test_json_reader_under_sanitizers(tmp_path):
    """The cache's JSON reader, built on its own with the address and
    undefined-behaviour sanitizers: values, refusals, and random damage."""
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = str(tmp_path / "tune_cache_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-o", exe,
                    os.path.join(root, "tests", "tune_cache_check.cpp")], check=True)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "ok" in p.stdout
