"""CPU checks of the C-ABI library: it loads and exports every declared symbol.

No compute call is made (there is no GPU here)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lrx.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lrx_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("lrx_create", "lrx_set_structure", "lrx_set_tensors", "lrx_evaluate", "lrx_destroy",
                 "lrx_last_error", "lrx_evaluate_batch"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2412_11081_amd import lrx

    if not os.path.exists(lrx.LIB_PATH):
        pytest.fail("liblrx.so not built (run __graft_entry__.build())")
    out = subprocess.run(["nm", "-D", "--defined-only", lrx.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (lrx_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    lib = lrx.load()
    for n in declared():
        assert hasattr(lib, n)


def test_binding_exports_match_header():
    from paper_2412_11081_amd import lrx

    assert sorted(lrx.EXPORTS) == declared()


def test_product_path_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_2412_11081_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "lrx_oracle" not in src and "orc_" not in src, f
