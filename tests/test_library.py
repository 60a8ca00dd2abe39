"""Host-side checks of the C-ABI library (no GPU calls)."""

import ctypes
import os
import re

import pytest

from paper_1011_5964_amd import lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    with open(os.path.join(ROOT, "include", "tvdeblur.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(tvdeblur_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert header_symbols() == sorted(L.EXPORTED_SYMBOLS)


@pytest.mark.skipif(not os.path.exists(L.LIB_PATH), reason="library not built")
def test_library_loads_and_exports_every_declared_symbol():
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in header_symbols():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(L.LIB_PATH), reason="library not built")
def test_struct_layouts_match_header():
    """Binding structs have the sizes implied by the header's field list."""
    assert ctypes.sizeof(L.Params) == 8 * 2 + 8 + 8 * 2 + 8 + 8 * 3
    assert ctypes.sizeof(L.Stats) == 4 + 4 * 256 + 4 + 8 * 256 * 2 + 4 + 4 + 8 + 8 * 3


@pytest.mark.skipif(not os.path.exists(L.LIB_PATH), reason="library not built")
def test_null_handle_errors_without_gpu():
    lib = L.load()
    assert lib.tvdeblur_set_bc(None, 2) == -1
    assert lib.tvdeblur_destroy(None) == 0
    assert lib.tvdeblur_last_error(None) is not None
