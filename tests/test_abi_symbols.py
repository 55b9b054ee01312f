"""CPU-side checks of the C ABI boundary: the shared library loads without a GPU
and exports every function include/rp4d.h declares; the binding declares no
function the header lacks.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rp4d.h")
LIB = os.path.join(ROOT, "paper_2401_15758_amd", "librp4d.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rp4d_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_core_calls():
    names = declared()
    for core in ("rp4d_fwd", "rp4d_tlm", "rp4d_adj", "rp4d_hessian_block", "rp4d_build_precond",
                 "rp4d_pcg_solve", "rp4d_gn_step"):
        assert core in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_matches_header():
    from paper_2401_15758_amd import rp4d
    assert set(rp4d.EXPORTED) == set(declared())
    assert rp4d.version().startswith("rp4d")
