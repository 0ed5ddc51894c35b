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


def _c_struct_fields(name):
    """(type, field) pairs of a typedef struct in the header, comments removed."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + r"\s*;", text).group(1)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        typ, names = decl.split(None, 1)
        out += [(typ, v.strip()) for v in names.split(",")]
    return out


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
@pytest.mark.parametrize("name", ["hm_theta", "hm_tree_opts", "hm_approx", "hm_result", "hm_server_opts",
                                  "hm_request_stats"])
def test_binding_structs_match_header(name):
    """Every ctypes structure of the binding has the header's fields, in order,
    with the header's types (so offsets and sizes agree)."""
    from paper_1709_04419_amd import hmlik
    ctype = {"double": ctypes.c_double, "int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64}
    py = getattr(hmlik, name)._fields_
    hdr = _c_struct_fields(name)
    assert [f for f, _ in py] == [f for _, f in hdr]
    assert [t for _, t in py] == [ctype[t] for t, _ in hdr]


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_null_handles_are_argument_errors():
    """Calls on null handles fail with HM_ERR_ARG before touching a device."""
    from paper_1709_04419_amd import hmlik
    lib = hmlik._lib
    z = (ctypes.c_double * 4)()
    assert lib.hm_dataset_set_z(None, z, 1, 0) == hmlik.HM_ERR_ARG
    assert lib.hm_factor(None) == hmlik.HM_ERR_ARG
    out = ctypes.c_void_p()
    opts = hmlik.hm_tree_opts(64, 2.0)
    assert lib.hm_dataset_create(None, z, 2, 2, ctypes.byref(opts), 0, ctypes.byref(out)) == hmlik.HM_ERR_ARG
    assert lib.hm_exact_block(None, 0, 1, 0, 1, z, 1, 0) == hmlik.HM_ERR_ARG


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_rejects_wrong_device_tensors():
    """A torch tensor given as a device pointer must be float64 on the context's
    GPU: a float32 tensor would make the library read 8 bytes per 4-byte entry,
    a CPU tensor is not device memory at all."""
    import torch

    from paper_1709_04419_amd import hmlik

    class FakeCtx:
        device = 0

    with pytest.raises(TypeError):
        hmlik._device_f64(torch.zeros(8, dtype=torch.float32), FakeCtx(), "Z")
    with pytest.raises(ValueError):
        hmlik._device_f64(torch.zeros(8, dtype=torch.float64), FakeCtx(), "Z")
    with pytest.raises(TypeError):
        hmlik._device_f64([1.0, 2.0], FakeCtx(), "Z")
