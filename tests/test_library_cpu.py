"""CPU-side checks of the product library: it builds, loads without a GPU and
exports every function include/lbdd.h declares (no compute calls here)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "lbdd.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(lbdd_\w+)\s*\(", src, re.M)))


def test_header_declares_the_core_calls():
    names = declared_functions()
    for n in ("lbdd_create", "lbdd_solve", "lbdd_objective", "lbdd_assignment", "lbdd_destroy",
              "lbdd_last_error", "lbdd_best_transfers"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2304_06543_amd import lbdd
    lib = lbdd.load()
    names = declared_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(lbdd.EXPORTS) == names


def test_no_error_before_any_call():
    from paper_2304_06543_amd import lbdd
    assert lbdd.load().lbdd_last_error() == b""


def test_product_does_not_reference_the_oracle():
    """The product path (package and kernels) never names the oracle."""
    pkg = os.path.join(ROOT, "paper_2304_06543_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                with open(os.path.join(dirpath, fn)) as f:
                    txt = f.read()
                assert "import oracle" not in txt and "asral_oracle" not in txt, fn


def test_missing_library_fails_loudly(tmp_path):
    from paper_2304_06543_amd import lbdd
    saved = lbdd._lib
    lbdd._lib = None
    try:
        with pytest.raises(RuntimeError):
            lbdd.load(str(tmp_path / "nope.so"))
    finally:
        lbdd._lib = saved
