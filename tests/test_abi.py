"""The C-ABI library loads and exports every symbol include/lps.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lps.h")
LIB = os.path.join(ROOT, "paper_2507_06300_amd", "liblps.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lps_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["lps_create", "lps_destroy", "lps_psd_build", "lps_loglike_batch",
                     "lps_loglike_grad_batch", "lps_loglike_plain_fp64"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    lib.lps_strerror.restype = ctypes.c_char_p
    assert lib.lps_strerror(0) == b"ok"
    assert lib.lps_chunk_bins(0) > 0 and lib.lps_chunk_bins(1) > 0


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_structural_errors_before_any_launch():
    """NULL arguments are rejected on the host without touching a device."""
    import paper_2507_06300_amd as m
    L = m.lib()
    assert L.lps_create(None, 0, None) == 1
    out = ctypes.c_void_p()
    assert L.lps_create(None, 0, ctypes.byref(out)) == 1
    assert L.lps_loglike_batch(None, None, 0, None, None, None) == 1
    assert L.lps_destroy(None) == 0


def test_python_binding_symbol_list_matches_header():
    import paper_2507_06300_amd as m
    assert sorted(m.SYMBOLS) == declared_functions()
