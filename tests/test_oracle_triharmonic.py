"""Pins of the triharmonic oracle (Sec. 4.2, "Triharmonic equation"; Table 5), CPU only.

* the one-sided fourth-normal-derivative weights solve the Taylor moment system (exact for
  normal polynomials of degree <= 6, first failure at degree 7 with moment 5/21);
* the whole discrete system is exact for u of total degree 5 (L_h u = M Delta u holds for
  degree <= 5, and v, w have lower degree), in 2-D and 3-D, clamped and Navier faces mixed,
  on non-unit boxes; planted errors (a dropped u_nn datum, a dropped tangential part, a
  three-point formula) break it;
* fourth-order convergence on a smooth solution;
* the matrix-free Schur tier equals the direct tier;
* Table 5 at 32^3 for both parameter settings, to half a unit of the printed digits.
"""
import json
import os
from fractions import Fraction
from math import factorial

import numpy as np
import pytest

import workloads as W
from oracle import triharmonic as T

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))

U2 = "1 + x - 2*y + x*y + 0.5*x**2*y**2 - 0.3*x**3*y + 0.2*x**4*y - 0.1*y**5 + 0.7*x**5 + 0.4*x**2*y**3"
U3 = "1 + x - 2*y + 0.5*z + x*y*z + 0.5*x**2*y**2*z - 0.3*x**3*z + 0.2*x**5 + 0.1*y**4*z - 0.7*z**2*x**3 + 0.25*z**5"


def _moments():
    a = T.ONE_SIDED4
    out = []
    for j in range(8):
        m = sum(a[k] * Fraction(k ** j, factorial(j)) for k in range(5))
        if j == 1:
            m += T.ONE_SIDED4_D1
        if j == 2:
            m += T.ONE_SIDED4_D2
        out.append(m)
    return out


def test_weights_solve_the_moment_system():
    mom = _moments()
    assert mom[:7] == [0, 0, 0, 0, 1, 0, 0]
    assert mom[7] == Fraction(5, 21)


def test_weights_are_the_unique_moment_solution():
    """Solve the 7 x 7 moment system (unknowns a_0..a_4, c_1, c_2) by exact elimination."""
    n = 7
    A = []
    for j in range(n):
        row = [Fraction(k ** j, factorial(j)) for k in range(5)]
        row += [Fraction(int(j == 1)), Fraction(int(j == 2))]
        row.append(Fraction(int(j == 4)))
        A.append(row)
    for c in range(n):
        piv = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c] / A[c][c]
                A[r] = [x - f * y for x, y in zip(A[r], A[c])]
    sol = [A[i][n] / A[i][i] for i in range(n)]
    assert tuple(sol[:5]) == T.ONE_SIDED4
    assert sol[5] == T.ONE_SIDED4_D1 and sol[6] == T.ONE_SIDED4_D2


@pytest.mark.parametrize("navier", [(False,) * 4, (False, True, True, False), (True, False, False, True)])
def test_polynomial_exactness_2d(navier):
    p = W.triharmonic(U2, (9, 7), (-0.3, 0.1), (0.9, 1.4), navier=navier)
    U, Q, asm = T.solve(p)
    assert np.abs(U - p.u_exact).max() < 1e-12 * np.abs(p.u_exact).max()


@pytest.mark.parametrize("navier", [(False,) * 6, (False, True, False, False, True, False)])
def test_polynomial_exactness_3d(navier):
    p = W.triharmonic(U3, (6, 7, 5), (-0.3, 0.1, 0.2), (0.9, 1.4, 1.1), navier=navier)
    U, Q, asm = T.solve(p)
    assert np.abs(U - p.u_exact).max() < 1e-11 * np.abs(p.u_exact).max()


@pytest.mark.parametrize("plant", ["no_unn", "no_tangential", "three_point"])
def test_planted_errors_break_exactness(plant, monkeypatch):
    p = W.triharmonic(U2, (9, 7), (-0.3, 0.1), (0.9, 1.4))
    if plant == "no_unn":
        monkeypatch.setattr(T, "ONE_SIDED4_D2", Fraction(0))
    elif plant == "no_tangential":
        p.tang4 = None
    else:  # the degree-5 formula from U_1..U_3 (h^2 error): exact only to degree 5 along the normal
        monkeypatch.setattr(T, "ONE_SIDED4", (Fraction(148, 3), Fraction(-60), Fraction(12), Fraction(-4, 3), Fraction(0)))
        monkeypatch.setattr(T, "ONE_SIDED4_D1", Fraction(40))
        monkeypatch.setattr(T, "ONE_SIDED4_D2", Fraction(12))
        p = W.triharmonic("x**6 + y**2*x", (9, 7), (-0.3, 0.1), (0.9, 1.4))
    U, Q, asm = T.solve(p)
    assert np.abs(U - p.u_exact).max() > 1e-8 * np.abs(p.u_exact).max(), plant


def test_fourth_order_2d():
    errs = []
    for n in (16, 32, 64):
        p = W.triharmonic("sin(5*x)*cos(y)*exp(0.5*y)", (n, n), navier=(False, True, True, True))
        U, Q, asm = T.solve(p)
        errs.append(np.abs(U - p.u_exact).max())
    assert all(14.0 < errs[i] / errs[i + 1] < 19.0 for i in range(2)), errs


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_fast_tier_equals_direct(case):
    if case == "2d":
        p = W.triharmonic("sin(3*x)*cos(2*y)*exp(x*y)", (24, 16), (0, 0), (1.0, 0.8), navier=(False, True, False, True))
    else:
        p = W.example3_tri(8)
    U, Q, asm = T.solve(p)
    Uf, Qf, info = T.TriFast(p).solve(tol=1e-14)
    assert info["converged"]
    assert np.abs(Uf - U).max() < 1e-11 * np.abs(U).max()
    # Q is h^-4 times a combination of U near the face: U's rounding (~1e-15 relative) grows
    # by h^-4 ~ 3e5 at n = 24, so Q agrees to ~1e-9 relative
    assert np.abs(Qf - Q).max() < 1e-7 * np.abs(Q).max()


def test_schur_objects_match_fast_tier():
    p = W.triharmonic("sin(3*x)*cos(2*y)", (12, 10), (0, 0), (1.0, 0.8), navier=(False, True, False, False))
    S, b, asm = T.schur(p)
    ft = T.TriFast(p)
    q = np.random.default_rng(3).standard_normal(S.shape[0])
    assert np.abs(ft.schur_matvec(q) - S @ q).max() < 1e-9 * np.abs(S @ q).max()
    assert np.abs(ft.schur_rhs() - b).max() < 1e-9 * np.abs(b).max()


def _half_unit(x):
    return 0.5 * 10.0 ** (np.floor(np.log10(x)) - 2)


@pytest.mark.parametrize("k", ["5,1,5", "25,5,25"])
def test_table5_at_32(k):
    ref = GOLD["triharmonic_table5"]["err_u_inf"][k]["32"]
    p = W.example3_tri(32, tuple(float(v) for v in k.split(",")))
    U, Q, info = T.TriFast(p).solve(tol=1e-12)
    assert info["converged"]
    err = np.abs(U - p.u_exact).max()
    assert abs(err - ref) <= _half_unit(ref), (err, ref)
