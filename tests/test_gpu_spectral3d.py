"""GPU parity of the 3-D spectral path against the oracle (through the C ABI).

When every axis length has a length-specialised transform (32, 64, 96, ..., 4096) the GPU
takes the spectral form of the Schur matvec (Lemma 1 / Algorithm 1): the face-layer lift
and its 2-D spectra, the generated-spectrum inverse pass along z, the U-solve that stops at
the scaled spectrum and contracts it into face sums, and the boundary gather from those sums.
This is the path the 1024^3 benchmark times.  Here it is compared with the oracle's fast
tier (itself pinned to the direct solve of the coupled system), on unequal axes and a
non-unit box so that a mix-up of the per-face tables would show:

* ahoc_schur_apply against R(q) of the fast tier with zero data (= S_h q exactly);
* ahoc_schur_rhs against the fast tier's b = -R(0);
* ahoc_solve (FP64 and MIXED) against fast-tier solutions -- in the test at 32^3, from
  tests/golden/spectral3d_oracle.json (written by make_spectral3d_oracle.py, oracle only)
  at 64^3, 32 x 64 x 96 and 128^3;
* polynomial exactness (Sec. 2.2 stencils exact on quintics, one-sided formula on quartics)
  at 256^3, 512^3 and 1024^3 with one Navier face, where no CPU solve fits.

Tolerances: FP64 operator 1e-12 relative to the largest output, FP32 operator 2e-5 (unit
roundoff 6e-8 times the O(sqrt(N) log N) growth of the transforms); FP64 solves 1e-12
relative on U, MIXED solves 1e-10 (the benchmark spec's bound); the polynomial-exactness bounds
are stated at the test.
"""
import dataclasses
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import fast

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "spectral3d_oracle.json")))


@pytest.fixture(scope="module")
def ah():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_16478_amd as mod
    mod.set_dst_variant(0)
    return mod


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _box(n, hi):
    return W.manufactured(W.C3_ALPHA, W.C3_U, n, (0.0, 0.0, 0.0), hi)


SPEC = {
    "c3_32": lambda: W.config3(32),
    "c3_32x64x96": lambda: _box((32, 64, 96), (1.0, 1.3, 0.8)),
    "c3_96x32x64": lambda: _box((96, 32, 64), (0.8, 1.0, 1.3)),
}


def _homogeneous(p):
    """The same grid and alpha with zero data: its R(q) is S_h q exactly (R(0) = 0)."""
    z = np.zeros(tuple(m + 1 for m in reversed(p.n)))
    return dataclasses.replace(p, f=z, gD=None, gN=None, lapgD=None)


def _assert_spectral(s):
    """The handle's matvec ran the spectral form (generated-spectrum pass and face sums)."""
    kt = s.kernel_times()
    assert kt["dst_gen"][1] > 0 and kt["face_reduce"][1] > 0, kt


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", list(SPEC))
def test_schur_apply_spectral_matches_fast_tier(ah, case, prec):
    p = SPEC[case]()
    ft = fast.FastTier(_homogeneous(p))
    rng = np.random.default_rng(23)
    tol = 1e-12 if prec == "fp64" else 2e-5
    with ah.Solver(p, precision=ah.FP64 if prec == "fp64" else ah.MIXED) as s:
        assert s.nq == ft.g.n_q
        s.profile(True)
        for _ in range(2):
            q = rng.standard_normal(s.nq)
            y = s.schur_apply(q).cpu().numpy()
            ref = ft.R_of(q)
            assert _rel(y, ref) < tol, (case, prec, _rel(y, ref))
        _assert_spectral(s)


@pytest.mark.parametrize("case", list(SPEC))
def test_schur_rhs_spectral_matches_fast_tier(ah, case):
    """b = -R(0) with the data (inhomogeneous on the far faces of the boxes); the MIXED
    handle (Schur refinement) forms the same FP64 b."""
    p = SPEC[case]()
    ref = fast.FastTier(p).schur_rhs()
    for prec in (ah.FP64, ah.MIXED):
        with ah.Solver(p, precision=prec) as s:
            b = s.schur_rhs().cpu().numpy()
        assert _rel(b, ref) < 1e-11, (case, prec, _rel(b, ref))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_spectral_32_matches_fast_tier(ah, prec):
    p = W.config3(32)
    U, V, Q, info = fast.FastTier(p).solve(tol=1e-15, max_iters=300)
    assert info["converged"]
    with ah.Solver(p, precision=ah.FP64 if prec == "fp64" else ah.MIXED,
                   tol=1e-14 if prec == "fp64" else 1e-12) as s:
        s.profile(True)
        u, _, q, st = s.solve(want_q=True)
        _assert_spectral(s)
    assert st.converged, st
    assert _rel(u.cpu().numpy(), U) < (1e-12 if prec == "fp64" else 1e-10), (prec, st)
    if prec == "fp64":
        assert _rel(q.cpu().numpy(), Q) < 1e-10


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["c3_64", "c3_32x64x96", "c3_128"])
def test_solve_spectral_matches_fast_tier_golden(ah, case, prec):
    o = GOLD["cases"][case]
    p = W.manufactured(W.C3_ALPHA, W.C3_U, tuple(o["n"]), (0.0, 0.0, 0.0), tuple(o["hi"]),
                       xp="torch", device=torch.device("cuda:0"))
    with ah.Solver(p, precision=ah.FP64 if prec == "fp64" else ah.MIXED,
                   tol=1e-14 if prec == "fp64" else 1e-12) as s:
        s.profile(True)
        u, _, _, st = s.solve()
        _assert_spectral(s)
    assert st.converged, st
    nodes = np.asarray(o["nodes"])
    got = u[nodes[:, 0], nodes[:, 1], nodes[:, 2]].cpu().numpy()
    bound = (1e-12 if prec == "fp64" else 1e-10) * o["u_max"]
    dev = np.abs(got - np.asarray(o["u"])).max()
    print(f"{case} {prec}: max deviation at {len(nodes)} nodes {dev / o['u_max']:.2e} (relative), "
          f"{st.gmres_iters} its", flush=True)
    assert dev <= bound, (case, prec, dev / o["u_max"])
    err = (u - p.u_exact).abs().max().item()
    assert abs(err - o["err_u_inf"]) <= 1e-6 * o["err_u_inf"] + 1e-12 * o["u_max"], (err, o["err_u_inf"])


# Polynomial exactness at the benchmark's sizes: u of total degree 4 with alpha of degree 3
# (so v = alpha Delta u has degree 5), inhomogeneous data, the x+ face Navier.  The compact
# operators are exact for such data, so the discrete solution is the polynomial itself and
# the remaining difference is the Schur tolerance and rounding.  Bounds: FP64 (tol 1e-13):
# 2e-11 relative (rounding of the transforms, ~eps log2(N) per pass over O(10) passes, times
# the O(1/h) = O(N) conditioning of S_h at N = 1024: ~1e-16 * 10 * 10 * 1e3 = 1e-11);
# MIXED (tol 1e-11, FP64 residuals): 1e-10, the benchmark spec's bound.
@pytest.mark.parametrize("n", [256, 512, 1024])
def test_polynomial_exactness_spectral_large(ah, n):
    p = W.poly_exact(n, 3, xp="torch", device=torch.device("cuda:0"), chunk=32,
                     navier=(False, True, False, False, False, False))
    ue = p.u_exact
    scale = ue.abs().max().item()
    p.v_exact = None
    for prec, tol, bound in ((ah.FP64, 1e-13, 2e-11), (ah.MIXED, 1e-11, 1e-10)):
        with ah.Solver(p, precision=prec, tol=tol) as s:
            s.profile(True)
            u, _, _, st = s.solve()
            _assert_spectral(s)
        err = (u - ue).abs().max().item() / scale
        print(f"poly exactness n={n} prec={prec}: rel err {err:.2e}, {st.gmres_iters} its, "
              f"{st.sweeps} sweeps, {st.t_solve_ms:.0f} ms", flush=True)
        assert st.converged, st
        assert err < bound, (n, prec, err)
        del u
        torch.cuda.empty_cache()
