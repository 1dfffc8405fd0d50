"""The C-ABI library loads and exports every entry point the header declares
(no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rpid.h")
LIB = os.path.join(ROOT, "paper_2104_05877_amd", "librpid.so")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rpid_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_path():
    names = declared_symbols()
    for n in ("rpid_sketch", "rpid_select_columns", "rpid_id_coeffs", "rpid_cur", "rpid_residual"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="librpid.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="librpid.so not built")
def test_binding_matches_header():
    from paper_2104_05877_amd import rpid

    assert sorted(rpid.symbols()) == declared_symbols()
    assert rpid.lib().rpid_version() == 1
    assert rpid.lib().rpid_status_string(-103) == b"dtype combination or size not supported"
