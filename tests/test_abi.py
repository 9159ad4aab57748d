"""The C-ABI library loads and exports every symbol include/dsw.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dsw.h")
LIB = os.path.join(ROOT, "paper_2004_13887_amd", "libdsw.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dsw_[A-Za-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("dsw_init_grid", "dsw_layout", "dsw_split_step", "dsw_residual", "dsw_line_solve_r",
              "dsw_line_solve_theta", "dsw_line_solve_phi", "dsw_get_status", "dsw_last_error",
              "dsw_free_grid"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdsw.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n


def test_binding_lists_every_symbol():
    from paper_2004_13887_amd import dsw
    assert sorted(dsw.SYMBOLS) == declared()
