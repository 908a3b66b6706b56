"""ahoc_poisson_noalloc (the allocation-free variant of ahoc_poisson, for callers that cannot
allocate device memory) against ahoc_poisson through a handle, and against the oracle's
sine-transform Poisson solve: FP64 to 1e-12 relative, FP32 transforms to 1e-5 (the bars of the
Poisson parity tests).  Two calls in a row share the fixed scratch array, the second on a
smaller grid; grids too large for the array are refused before any device work."""
import numpy as np
import pytest

import workloads as W
from oracle import fast

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ah():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_16478_amd as mod
    return mod


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _problem(n, hi):
    shape = tuple(m + 1 for m in reversed(n))
    return W.Problem(n, (0.0,) * len(n), hi, np.ones(shape), np.zeros(shape))


# (larger grid, then smaller grid) pairs; 20 and 7, 9 have no radix-2/3 FFT plan (direct pass)
PAIRS = {
    "3d": (((48, 40, 64), (1.0, 1.3, 0.8)), ((12, 10, 16), (0.7, 1.0, 1.1))),
    "2d": (((256, 96), (1.0, 0.6)), ((20, 9), (1.0, 1.0))),
    "3d_direct": (((20, 7, 9), (1.0, 0.5, 0.6)), ((4, 5, 4), (1.0, 1.0, 1.0))),
}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("pair", list(PAIRS))
def test_noalloc_poisson_matches_handle(ah, pair, prec):
    p = ah.FP64 if prec == "fp64" else ah.MIXED
    tol = 1e-12 if prec == "fp64" else 1e-5
    rng = np.random.default_rng(7)
    for n, hi in PAIRS[pair]:
        pb = _problem(n, hi)
        ft = fast.FastTier(pb)
        g = rng.standard_normal(ft.g.interior_shape)
        gt = torch.from_numpy(g).cuda()
        w = ah.poisson_noalloc(n, (0.0,) * len(n), hi, gt, precision=p)
        with ah.Solver(pb, precision=p) as s:
            ref = s.poisson(g).cpu().numpy()
        wn = w.cpu().numpy()
        assert _rel(wn, ref) < tol, (pair, n, prec, _rel(wn, ref))
        assert _rel(wn, ft.poisson(g)) < tol, (pair, n, prec)


def test_noalloc_poisson_in_place_and_refusals(ah):
    n, hi = (32, 24, 16), (1.0, 1.0, 1.0)
    g = torch.randn(15, 23, 31, dtype=torch.float64, device="cuda")
    ref = ah.poisson_noalloc(n, (0, 0, 0), hi, g)
    g2 = g.clone()
    ah.poisson_noalloc(n, (0, 0, 0), hi, g2, out=g2)  # w == g
    assert torch.equal(ref, g2)
    # padded interior above 63 MiB (FP64: 256^3 -> 255 * 255 * 256 * 8 B = 133 MB)
    big = torch.empty(1, dtype=torch.float64, device="cuda")
    na = (ah.c_int * 3)(256, 256, 256)
    lo = (ah.c_double * 3)(0, 0, 0)
    hi3 = (ah.c_double * 3)(1, 1, 1)
    rc = ah._lib.ahoc_poisson_noalloc(ah.FP64, 3, na, lo, hi3, ah._ptr(big), ah._ptr(big), ah._stream())
    assert rc == ah.E_INVALID
    na = (ah.c_int * 3)(3, 8, 8)
    rc = ah._lib.ahoc_poisson_noalloc(ah.FP64, 3, na, lo, hi3, ah._ptr(big), ah._ptr(big), ah._stream())
    assert rc == ah.E_INVALID
