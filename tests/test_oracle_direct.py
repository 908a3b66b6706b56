"""Pins for the oracle's direct tier (CPU).

* polynomial exactness of the whole coupled system (degree-4 u, degree-3 alpha,
  inhomogeneous g_D, g_N, Delta u data): U = u at every node to rounding;
* fourth-order convergence on a manufactured variable-coefficient solution
  (the paper's claim, Sec. 3 Theorem 1 and Sec. 4.1);
* the lid-driven cavity of Table 6 and the clamped plate of Sec. 4.2.4;
* the explicit Schur complement: Lemma 1 (S_h Q = R(Q) - R(0), b = -R(0)),
  its conditioning growth O(1/h) (Sec. 4.1, Fig. 1 discussion), and for
  constant alpha the single-face representation of Lemma 4.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import direct, fast, dst
from oracle.grid import Grid

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.mark.parametrize("n", [8, 16, (13, 9)])
def test_polynomial_exactness_2d(n):
    p = W.poly_exact(n, 2)
    U, V, Q, asm = direct.solve(p)
    assert np.abs(U - p.u_exact).max() < 1e-13
    assert np.abs(V - p.v_exact).max() < 1e-10


@pytest.mark.parametrize("n", [5, (6, 4, 5)])
def test_polynomial_exactness_3d(n):
    p = W.poly_exact(n, 3)
    U, V, Q, asm = direct.solve(p)
    assert np.abs(U - p.u_exact).max() < 1e-13
    assert np.abs(V - p.v_exact).max() < 1e-10


def test_polynomial_exactness_fails_for_degree6():
    # a planted degree-6 term breaks exactness: the pin has teeth
    p = W.manufactured("1 + 0.1*x", "x**3*y**3 + y**6", (10, 10))
    U, V, Q, asm = direct.solve(p)
    assert np.abs(U - p.u_exact).max() > 1e-8


def test_fourth_order_2d_variable_coefficient():
    errs = []
    for n in (8, 16, 32, 64):
        p = W.config2(n)
        U, *_ = direct.solve(p)
        errs.append(np.abs(U - p.u_exact).max())
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(14.0 < r < 19.0 for r in ratios), (errs, ratios)


def test_fourth_order_3d_variable_coefficient():
    errs = []
    for n in (4, 8, 16):
        p = W.config3(n)
        U, *_ = direct.solve(p)
        errs.append(np.abs(U - p.u_exact).max())
    order = np.log2(errs[1] / errs[2])   # still pre-asymptotic at N = 8 -> 16
    assert 3.6 < order < 4.6, errs


def test_constant_coefficient_config1_converges():
    errs = []
    for n in (16, 32):
        p = W.config1(n)
        U, *_ = direct.solve(p)
        errs.append(np.abs(U - p.u_exact).max())
    # alpha = 1, u = sin^2 sin^2: u^(5) vanishes on the faces, so the leading term of the
    # one-sided formula drops out and the coarse-grid ratio exceeds 16 (pre-asymptotic)
    assert errs[0] / errs[1] > 14.0, errs


def test_lid_driven_cavity_table6():
    gold = GOLD["cavity"]
    n = 64
    U, V, Q, asm = direct.solve(W.cavity(n))
    k = np.unravel_index(np.argmax(np.abs(U)), U.shape)
    mx = np.abs(U).max()
    ref = gold["max_abs_psi"]["4096"]
    assert abs(mx - ref) < 2e-6, mx
    loc = (k[1] / n, k[0] / n)
    assert abs(loc[0] - gold["location"]["4096"][0]) <= 1.0 / n
    assert abs(loc[1] - gold["location"]["4096"][1]) <= 1.0 / n


def test_clamped_plate_central_load():
    gold = GOLD["plate"]
    n = 128
    U, V, Q, asm = direct.solve(W.plate(n))
    c = n // 2
    u_c = U[c, c]
    m_edge = V[n, c]     # V = alpha Delta u at (0.5, 1)
    assert u_c == pytest.approx(gold["central_deflection"], rel=3e-3)
    assert -m_edge == pytest.approx(gold["minus_moment_at_edge_midpoint"], rel=1.5e-3)


def test_plate_load_is_unit():
    for n in (16, 17):
        assert (W.plate(n).f.sum() / n ** 2) == pytest.approx(-1.0)


def test_schur_lemma1_matches_explicit_elimination():
    p = W.config2(16)
    S, b, asm = direct.schur(p)
    ft = fast.FastTier(p)
    R0 = ft.R_of(np.zeros(asm.grid.n_q))
    assert np.abs(b + R0).max() < 1e-12 * np.abs(b).max()
    rng = np.random.default_rng(0)
    for _ in range(3):
        q = rng.standard_normal(asm.grid.n_q)
        y = ft.R_of(q) - R0
        assert np.abs(S @ q - y).max() < 1e-11 * np.abs(y).max()


def test_schur_3d_lemma1():
    p = W.config3(6)
    S, b, asm = direct.schur(p)
    ft = fast.FastTier(p)
    q = np.random.default_rng(1).standard_normal(asm.grid.n_q)
    y = ft.schur_matvec(q, ft.schur_rhs())
    assert np.abs(S @ q - y).max() < 1e-11 * np.abs(y).max()


def test_schur_solution_matches_direct():
    p = W.config2(12)
    S, b, asm = direct.schur(p)
    U, V, Q, _ = direct.solve(p)
    assert np.abs(np.linalg.solve(S, b) - Q).max() < 1e-10 * np.abs(Q).max()


def test_schur_conditioning_grows_like_inverse_h():
    conds = []
    for n in (16, 32):
        S, b, asm = direct.schur(W.config2(n))
        conds.append(np.linalg.cond(S))
    assert 1.6 < conds[1] / conds[0] < 2.4, conds


def test_constant_alpha_face_block_diagonal_in_sine_basis():
    # For alpha = 1 the x- face's diagonal Schur block commutes with the face's
    # sine transform (single-face representation of Lemma 4 is mode-by-mode).
    n = 16
    S, b, asm = direct.schur(W.config1(n))
    m = n - 1
    B = S[:m, :m]
    T = dst.sine_matrix(n) * np.sqrt(2.0 / n)   # orthonormal
    D = T @ B @ T
    off = D - np.diag(np.diag(D))
    assert np.abs(off).max() < 1e-11 * np.abs(np.diag(D)).max()


def test_lemma4_single_face_closed_form_2d():
    # L_h psi = 0 in the interior, psi = g on x = 0, 0 elsewhere (h_x = h_y):
    # psi_{i,j} = sum_k g_hat_k sinh((N-i) a_k)/sinh(N a_k) sin(k pi j / N),
    # cosh a_k = (5 - 2 cos theta_k)/(2 + cos theta_k)  (Lemma 4; Sec. 3.1)
    n = 24
    p = W.config1(n)
    ft = fast.FastTier(W.Problem(p.n, p.lo, p.hi, p.alpha, np.zeros_like(p.f)))
    g = np.random.default_rng(5).standard_normal(n - 1)
    Q = np.zeros(ft.g.n_q)
    Q[: n - 1] = g
    psi = ft.v_solve(Q)          # -L_h V = 0 with V = Q on the x- face
    k = np.arange(1, n)
    th = k * np.pi / n
    a = np.arccosh((5 - 2 * np.cos(th)) / (2 + np.cos(th)))
    ghat = (2.0 / n) * (dst.sine_matrix(n) @ g)
    j = np.arange(1, n)
    ref = np.zeros((n + 1, n + 1))
    for i in range(0, n + 1):
        r = np.sinh((n - i) * a) / np.sinh(n * a)
        ref[1:n, i] = (dst.sine_matrix(n) @ (ghat * r))
    assert np.abs(psi[1:n, 0:n] - ref[1:n, 0:n]).max() < 1e-12 * np.abs(g).max()
