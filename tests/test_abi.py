"""CPU checks of the C-ABI library: it loads and exports every function that
include/hmlik.h declares, and the Python binding names the same set.
No compute call is made (there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hmlik.h")
LIB = os.path.join(ROOT, "paper_1709_04419_amd", "libhmlik.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hm_[a-z_]+)\s*\(", text)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_header():
    from paper_1709_04419_amd import hmlik
    assert set(hmlik.EXPORTED) == set(declared_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_status_strings():
    from paper_1709_04419_amd import hmlik
    assert hmlik.hm_status_string(0) == "ok"
    assert "pivot" in hmlik.hm_status_string(hmlik.HM_ERR_NOT_SPD)
    assert hmlik.hm_status_string(99) == "unknown status"
