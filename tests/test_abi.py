"""CPU-side checks of the boundary: the HIP library loads without a GPU and
exports every function declared in include/cp_arls_lev.h; the binding's
structures match the header's layout."""
import ctypes
import os
import re
import subprocess

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


def _header_layout(tmp_path):
    """sizeof / offsetof of every ABI structure, printed by a C program
    compiled against the header with the host compiler."""
    from paper_2006_16438_amd import _lib
    structs = {"cpal_mode_stats": _lib.cpal_mode_stats, "cpal_tensor": _lib.cpal_tensor,
               "cpal_options": _lib.cpal_options, "cpal_allocator": _lib.cpal_allocator}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for name, st in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for f in st._fields_:
            lines.append(f'  printf("{name}.{f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True)
    return structs, dict(line.rsplit(" ", 1) for line in out.strip().splitlines())


def test_struct_layouts(tmp_path):
    structs, ref = _header_layout(tmp_path)
    for name, st in structs.items():
        assert ctypes.sizeof(st) == int(ref[name]), name
        for f in st._fields_:
            assert getattr(st, f[0]).offset == int(ref[f"{name}.{f[0]}"]), f"{name}.{f[0]}"


def _header_param_counts():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for m in re.finditer(r"\b(cp_arls_lev_\w+)\s*\(([^;]*?)\)\s*;", text, flags=re.S):
        args = m.group(2).strip()
        out[m.group(1)] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def test_binding_signatures_match_header():
    """Every declared call is bound with as many arguments as the header
    gives it (e.g. the allocator argument of the two init calls)."""
    from paper_2006_16438_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libcpal.so is not built; run __graft_entry__.build()")
    L = _lib.load()
    counts = _header_param_counts()
    assert set(counts) == set(_lib.SYMBOLS)
    for name, n in counts.items():
        assert len(getattr(L, name).argtypes) == n, name


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2006_16438_amd import _lib
    with pytest.raises(RuntimeError):
        _lib._lib = None
        _lib.load(str(tmp_path / "missing.so"))
    _lib._lib = None
