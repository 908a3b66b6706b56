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
    assert ah._lib.ahoc_setup(ctypes.byref(p), None, None, None, ctypes.byref(h)) == ah.E_INVALID
    p.dim = 2
    assert ah._lib.ahoc_setup(ctypes.byref(p), None, None, None, ctypes.byref(h)) == ah.E_INVALID  # NULL alpha
    # Navier flags per face (x-, x+, y-, y+[, z-, z+]) -> bit 2 axis + side
    assert ah._navier_mask((False, True, True, True)) == 0b1110
    assert ah._navier_mask((True, False, False, False, False, True)) == 0b100001
    assert ah._navier_mask(()) == 0 and ah._navier_mask(5) == 5


@pytest.mark.skipif(not os.path.exists(LIB), reason="libahoc.so not built")
def test_argument_errors_before_device_work():
    """Every rejected argument is caught on the host (the pointers below are never read)."""
    import paper_2609_16478_amd as ah
    fake = ctypes.c_void_p(64)

    def problem(n, lo=(0.0, 0.0), hi=(1.0, 1.0)):
        p = ah._Problem()
        p.dim = 2
        for a in range(2):
            p.n[a], p.lo[a], p.hi[a] = n[a], lo[a], hi[a]
        p.alpha = fake
        p.f = fake
        return p

    h = ctypes.c_void_p()
    for p, code in ((problem((3, 16)), ah.E_INVALID),                         # n < 4
                    (problem((16, 8193)), ah.E_INVALID),                      # n > 8192
                    (problem((16, 16), hi=(1.0, 0.0)), ah.E_INVALID)):        # hi <= lo
        assert ah._lib.ahoc_setup(ctypes.byref(p), None, None, None, ctypes.byref(h)) == code
    # an allocator needs both callbacks
    al = ah._Allocator()
    al.alloc = ah._TORCH_ALLOC
    assert ah._lib.ahoc_setup(ctypes.byref(problem((16, 16))), None, ctypes.byref(al), None,
                              ctypes.byref(h)) == ah.E_INVALID
    p = problem((16, 16))
    p.navier = 1 << 4  # a z face of a 2-D problem
    assert ah._lib.ahoc_setup(ctypes.byref(p), None, None, None, ctypes.byref(h)) == ah.E_INVALID
    o = ah.default_options()
    o.precision = 7
    p = problem((16, 16))
    assert ah._lib.ahoc_setup(ctypes.byref(p), ctypes.byref(o), None, None, ctypes.byref(h)) == ah.E_INVALID
    # batches: a negative count is rejected, an empty batch is a no-op
    assert ah._lib.ahoc_solve_batched(-1, None, None, None, None, None, None) == ah.E_INVALID
    assert ah._lib.ahoc_solve_batched(0, None, None, None, None, None, None) == ah.OK
    # calibration copies: unknown pattern, rows not a multiple of 32 columns
    assert ah._lib.ahoc_copy_bandwidth(3, fake, fake, 64, 4, 4, None) == ah.E_INVALID
    assert ah._lib.ahoc_copy_bandwidth(1, fake, fake, 48, 4, 4, None) == ah.E_INVALID
    # kernel-choice query without a handle
    m = ctypes.c_int()
    assert ah._lib.ahoc_dst_choice(None, ah.FP64, 0, 0, ctypes.byref(m), None, None, None, None) == ah.E_INVALID
