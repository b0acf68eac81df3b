"""CPU-side checks of the boundary: the HIP library loads without a GPU and
exports every function declared in include/cp_arls_lev.h; the binding's
structures match the header's layout."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cp_arls_lev.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cp_arls_lev_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2006_16438_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libcpal.so is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), f"{n} declared in the header but not exported"
    assert sorted(_lib.SYMBOLS) == names


def test_struct_layouts():
    from paper_2006_16438_amd import _lib
    assert ctypes.sizeof(_lib.cpal_mode_stats) == 56
    assert _lib.cpal_mode_stats.flags.offset == 48
    assert ctypes.sizeof(_lib.cpal_tensor) == 48
    assert ctypes.sizeof(_lib.cpal_options) == 72


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2006_16438_amd import _lib
    with pytest.raises(RuntimeError):
        _lib._lib = None
        _lib.load(str(tmp_path / "missing.so"))
    _lib._lib = None
