"""Pins for the oracle's beta term and Navier faces (CPU): -Delta(alpha Delta u) + beta Delta u = f
with beta constant; on a Navier face Delta u = g_L is given instead of u_n, so V = alpha g_L.

With v = alpha Delta u the v-equation becomes -Delta v + beta v / alpha = f, discretised
(Sec. 2.2) as -L_h V + M(beta V / alpha) = M f.  Pins, none of which restates that line:

* polynomial exactness of the whole coupled system with beta (the compact operators are
  exact for the degree-5 V of a degree-4 u and degree-3 alpha, so f = -Delta V + beta V/alpha
  is reproduced exactly), variable and constant alpha, positive and negative beta; and a
  planted omission (the beta term dropped while f keeps it) that breaks it;
* fourth-order convergence of a singularly perturbed case in the spirit of Example 1
  (alpha = eps constant, beta = 1);
* the fast tier (sine transforms with the shifted eigenvalue lambda_L - (beta/alpha) mu_M)
  against the direct tier;
* the weighting operator's symbol against its stencil applied to sine modes;
* Navier faces: Table 1 of the paper (Example 1, clamped at x = 0 and Navier elsewhere,
  alpha = eps, beta = 1) reproduced at 256 x 256 to its three printed digits for both eps;
  polynomial exactness with Navier faces in 2-D and 3-D; a planted loss of the Navier
  flags that breaks the solution; the fast tier against the direct tier;
* the high-wavenumber problem (beta = -k^2, indefinite v-equation): fourth order against a
  finer grid.
"""
import numpy as np
import pytest

import workloads as W
from oracle import direct, fast
from oracle.grid import Grid
from oracle.stencils import weighting, apply


@pytest.mark.parametrize("n,beta", [(8, 3.0), ((13, 9), -2.0), (16, 40.0)])
def test_polynomial_exactness_with_beta_2d(n, beta):
    p = W.poly_exact(n, 2, beta=beta)
    U, V, Q, asm = direct.solve(p)
    assert np.abs(U - p.u_exact).max() < 1e-12
    assert np.abs(V - p.v_exact).max() < 1e-9


@pytest.mark.parametrize("n,beta", [(5, 1.5), ((6, 4, 5), -0.7)])
def test_polynomial_exactness_with_beta_3d(n, beta):
    p = W.poly_exact(n, 3, beta=beta)
    U, V, Q, asm = direct.solve(p)
    assert np.abs(U - p.u_exact).max() < 1e-12
    assert np.abs(V - p.v_exact).max() < 1e-9


def test_dropped_beta_term_breaks_exactness():
    p = W.poly_exact(8, 2, beta=3.0)
    p.beta = 0.0  # f still carries beta Delta u
    U, *_ = direct.solve(p)
    assert np.abs(U - p.u_exact).max() > 1e-6


def test_fourth_order_singularly_perturbed():
    # alpha = eps, beta = 1: -eps Delta^2 u + Delta u = f (the operator of Example 1)
    errs = []
    for n in (16, 32, 64, 128):
        p = W.manufactured("0.01", "sin(pi*x)**2*sin(pi*y)**2*exp(x + y)", (n, n), beta=1.0)
        U, *_ = direct.solve(p)
        errs.append(np.abs(U - p.u_exact).max())
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(14.0 < r < 19.0 for r in ratios), (errs, ratios)


@pytest.mark.parametrize("maker", [
    lambda: W.manufactured("0.5", "sin(pi*x)**2*sin(pi*y)**2*exp(x + y)", (16, 12), (0.0, 0.0), (1.0, 0.75),
                           beta=2.0),
    lambda: W.manufactured("2", "sin(pi*x)**2*sin(pi*y)**2", (16, 16), beta=-5.0),
    lambda: W.manufactured("1", "sin(pi*x)**2*sin(pi*y)**2*sin(pi*z)**2", (8, 6, 10), beta=3.0),
], ids=["2d_aniso", "2d_negative", "3d"])
def test_fast_tier_with_beta_equals_direct(maker):
    p = maker()
    U, V, Q, _ = direct.solve(p)
    U2, V2, Q2, info = fast.FastTier(p).solve(tol=1e-14, restart=60)
    assert np.abs(U2 - U).max() <= 1e-12 * np.abs(U).max()
    assert np.abs(Q2 - Q).max() <= 1e-11 * np.abs(Q).max()


def test_fast_tier_rejects_variable_alpha_with_beta():
    with pytest.raises(ValueError):
        fast.FastTier(W.poly_exact(8, 2, beta=1.0))


@pytest.mark.parametrize("dim", [2, 3])
def test_weighting_symbol_matches_stencil_on_sine_modes(dim):
    n = (6, 5, 7)[:dim]
    g = Grid(n, (0.0,) * dim, (1.0, 0.7, 1.3)[:dim])
    M = weighting(dim)
    for k in ((1, 1, 1), (2, 4, 3), (5, 2, 6)):
        k = k[:dim]
        mode = np.ones(g.nodal_shape)
        for a in range(dim):
            shape = [1] * dim
            shape[dim - 1 - a] = n[a] + 1
            mode = mode * np.sin(np.pi * k[a] * np.arange(n[a] + 1) / n[a]).reshape(shape)
        mu = fast.weighting_symbol(n, k)
        inner = tuple(slice(1, m) for m in reversed(n))
        assert np.abs(apply(M, mode, g) - mu * mode[inner]).max() < 1e-14


# ------------------------------------------------------------------------------------------
# Navier faces (Delta u = g_L, so V = alpha g_L there) and the paper's Example 1
# ------------------------------------------------------------------------------------------

import json
import os

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.mark.parametrize("eps", ["1e-4", "1e-5"])
def test_example1_table1_at_256(eps):
    """The direct solve of Example 1 at 256 x 256 reproduces Table 1's max-norm error to the
    three printed digits (clamped x = 0, Navier elsewhere, alpha = eps, beta = 1)."""
    ref = GOLD["example1_table1"]["err_u_inf"][eps]["256"]
    p = W.example1(256, float(eps))
    U, *_ = direct.solve(p)
    err = np.abs(U - p.u_exact).max()
    assert abs(err - ref) <= 0.5e-2 * ref, (err, ref)  # within the printed rounding


@pytest.mark.parametrize("navier", [(False, True, True, True), (True, False, False, True), (True, True, True, True)])
def test_polynomial_exactness_with_navier_faces(navier):
    p = W.manufactured("2 + 0.3*x + 0.2*y + 0.1*x*y + 0.05*x**3",
                       "1 + x - 2*y + x*y + 0.5*x**2*y**2 - 0.3*x**3*y + 0.2*x**4 + 0.1*y**4",
                       (12, 9), (-0.3, 0.1), (0.9, 1.4), beta=1.5, navier=navier)
    U, V, Q, asm = direct.solve(p)
    assert np.abs(U - p.u_exact).max() < 1e-12
    assert np.abs(V - p.v_exact).max() < 1e-9


def test_polynomial_exactness_with_navier_faces_3d():
    p = W.manufactured("1.5", "1 + x - 2*y + 0.5*z + x*y*z + 0.5*x**2*y**2 - 0.3*x**3*z + 0.25*z**4",
                       (6, 5, 7), beta=-0.5, navier=(True, False, False, True, True, False))
    U, V, Q, asm = direct.solve(p)
    assert np.abs(U - p.u_exact).max() < 1e-12


def test_navier_data_matters():
    # planted: the Navier flags dropped (those faces treated as clamped with g_N = 0)
    p = W.example1(32, 1e-4)
    p.navier = ()
    U, *_ = direct.solve(p)
    assert np.abs(U - p.u_exact).max() > 1e-3 * np.abs(p.u_exact).max()


@pytest.mark.parametrize("maker", [
    lambda: W.example1(32, 1e-3),
    lambda: W.manufactured("1", "sin(pi*x)**2*sin(pi*y)**2*sin(pi*z)", (8, 6, 10), beta=2.0,
                           navier=(False, False, True, True, False, True)),
], ids=["ex1_2d", "3d"])
def test_fast_tier_with_navier_equals_direct(maker):
    p = maker()
    U, V, Q, _ = direct.solve(p)
    U2, V2, Q2, info = fast.FastTier(p).solve(tol=1e-14, restart=60)
    assert np.abs(U2 - U).max() <= 1e-11 * np.abs(U).max()


def test_high_wavenumber_fourth_order():
    """The high-wavenumber problem of Sec. 4.2 (alpha = 1, beta = -k^2: an indefinite
    v-equation) with a resolved source (k = 10, sigma = 0.1): the max-norm error against a
    256 x 256 solution falls at fourth order (ratio 15.2 between 64 and 128)."""
    ref = direct.solve(W.high_wavenumber(256, 2, k=10.0, sigma=0.1))[0]
    errs = []
    for n in (64, 128):
        U = direct.solve(W.high_wavenumber(n, 2, k=10.0, sigma=0.1))[0]
        errs.append(np.abs(U - ref[::256 // n, ::256 // n]).max())
    assert 13.0 < errs[0] / errs[1] < 19.0, errs


# ------------------------------------------------------------------------------------------
# variable beta (Remark 2: the v-equation is then iterated) and the paper's Example 2
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("dim,n,beta", [(2, (12, 9), "x + 2*y + 10"), (2, 10, "3 + x*y - y**2"),
                                        (3, (6, 5, 7), "x + y + z + 10")])
def test_polynomial_exactness_with_variable_beta(dim, n, beta):
    """With beta varying, M(beta V / alpha) must take beta at each neighbour of the stencil;
    the scheme then stays exact for u of degree 4 (the beta term of f is sampled, not
    discretised, and cancels only if the rows use the same nodal values)."""
    p = W.poly_exact(n, dim, beta=beta)
    assert not np.isscalar(p.beta)
    U, V, Q, asm = direct.solve(p)
    assert np.abs(U - p.u_exact).max() < 1e-11
    assert np.abs(V - p.v_exact).max() < 1e-8


def test_variable_beta_replaced_by_its_mean_breaks_exactness():
    # planted: the nodal beta replaced by its mean while f keeps the variable beta
    p = W.poly_exact((12, 9), 2, beta="x + 2*y + 10")
    p.beta = float(np.mean(p.beta))
    U, *_ = direct.solve(p)
    assert np.abs(U - p.u_exact).max() > 1e-6


def test_example2_fourth_order_small():
    """Example 2 (Sec. 4.1; variable alpha and beta, clamped at x = 0, Navier elsewhere) with
    (q, p) = (5, 1): the error falls by 14-17 from 8^3 to 16^3 (Table 2 starts at 32^3 with
    6.86e-4; the oracle's 32^3 solve, 6.848e-4, is stored by tests/golden/make_example2_oracle.py)."""
    errs = []
    for n in (8, 16):
        p = W.example2(n, 5.0, 1.0)
        U, *_ = direct.solve(p)
        errs.append(np.abs(U - p.u_exact).max())
    assert 12.0 < errs[0] / errs[1] < 17.0, errs


def test_fast_tier_rejects_variable_beta():
    with pytest.raises(ValueError):
        fast.FastTier(W.manufactured("1", "sin(pi*x)**2*sin(pi*y)**2", (8, 8), beta="1 + x"))


def test_stored_oracle_solutions_against_the_paper():
    """The oracle's stored large-size solutions (written by the committed scripts in
    tests/golden/) against what the paper prints: Tables 2 and 3 at 32^3 within 0.5 % (the
    paper's own GMRES tolerance, proportional to h^3.5, is loosest there), and the 4096^2
    solutions of Example 1 falling from Table 1's 2048^2 values at fourth order (ratios
    13-17; the printed 4096 entries are not used, see the design notes)."""
    g = os.path.join(os.path.dirname(__file__), "golden")
    ex1 = json.load(open(os.path.join(g, "example1_oracle.json")))
    ex2 = json.load(open(os.path.join(g, "example2_oracle.json")))
    ex3 = json.load(open(os.path.join(g, "example3_oracle.json")))
    t2 = GOLD["example2_table2"]["err_u_inf"]
    for key, case in ex2["cases"].items():
        assert abs(case["err_u_inf"] - t2[key]["32"]) <= 5e-3 * t2[key]["32"], key
    t3 = GOLD["example3_table3"]["err_u_inf"]
    for key, case in ex3["cases"].items():
        assert abs(case["err_u_inf"] - t3[key]["32"]) <= 5e-3 * t3[key]["32"], key
    t1 = GOLD["example1_table1"]["err_u_inf"]
    for eps, case in ex1["eps"].items():
        assert 13.0 < t1[eps]["2048"] / case["err_u_inf"] < 17.0, eps
