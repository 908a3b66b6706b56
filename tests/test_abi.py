"""The C-ABI library loads on the host and exports every function include/ahoc.h declares (CPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ahoc.h")
LIB = os.path.join(ROOT, "paper_2609_16478_amd", "libahoc.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ahoc_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ahoc_setup", "ahoc_schur_apply", "ahoc_solve", "ahoc_solve_batched",
                     "ahoc_destroy", "ahoc_nq"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libahoc.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libahoc.so not built")
def test_host_only_entry_points():
    import paper_2609_16478_amd as ah
    assert ah._lib.ahoc_status_string(ah.E_NOCONV) == b"not converged"
    o = ah.default_options()
    assert o.restart == 30 and o.tol == 1e-12 and o.precision == ah.FP64
    # argument validation happens before any device work
    h = ctypes.c_void_p()
    p = ah._Problem()
    p.dim = 4
    assert ah._lib.ahoc_setup(ctypes.byref(p), None, None, ctypes.byref(h)) == ah.E_INVALID
    p.dim = 2
    assert ah._lib.ahoc_setup(ctypes.byref(p), None, None, ctypes.byref(h)) == ah.E_INVALID  # NULL alpha
