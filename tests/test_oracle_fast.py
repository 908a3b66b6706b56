"""Pins for the oracle's fast tier (Algorithm 1 with library transforms), CPU.

The fast tier must reproduce the direct tier (the plain definition) to the
GMRES tolerance, and its GMRES must solve dense systems like a dense LU.
"""
import numpy as np
import pytest

import workloads as W
from oracle import direct, fast


@pytest.mark.parametrize("maker", [
    lambda: W.config1(16), lambda: W.config2(16), lambda: W.poly_exact((12, 9), 2),
    lambda: W.cavity(16), lambda: W.config3(8), lambda: W.poly_exact((6, 5, 7), 3),
], ids=["c1", "c2", "poly2d", "cavity", "c3", "poly3d"])
def test_fast_equals_direct(maker):
    p = maker()
    U, V, Q, _ = direct.solve(p)
    ft = fast.FastTier(p)
    U2, V2, Q2, info = ft.solve(tol=1e-14, restart=60)
    assert info["converged"] if "converged" in info else True
    assert np.abs(U2 - U).max() <= 1e-12 * np.abs(U).max()
    assert np.abs(Q2 - Q).max() <= 1e-11 * max(np.abs(Q).max(), 1e-300)


def test_eigenvalues_match_stencil_on_sine_modes():
    # L_h applied (by its stencil table) to a separable sine mode returns lambda * mode
    from oracle.stencils import laplacian, apply
    from oracle.grid import Grid
    p = W.config3(6)
    g = Grid((6, 5, 7), (0, 0, 0), (1.0, 0.7, 1.3))
    ft = fast.FastTier(W.Problem(g.n, g.lo, g.hi, np.ones(g.nodal_shape), np.zeros(g.nodal_shape)))
    L = laplacian(g.h)
    for kx, ky, kz in ((1, 1, 1), (2, 4, 3), (5, 2, 6)):
        x = np.arange(g.n[0] + 1)
        y = np.arange(g.n[1] + 1)
        z = np.arange(g.n[2] + 1)
        mode = (np.sin(np.pi * kz * z / g.n[2])[:, None, None]
                * np.sin(np.pi * ky * y / g.n[1])[None, :, None]
                * np.sin(np.pi * kx * x / g.n[0])[None, None, :])
        Lm = apply(L, mode, g)
        lam = ft.lam[kz - 1, ky - 1, kx - 1]
        assert np.abs(Lm - lam * mode[1:-1, 1:-1, 1:-1]).max() < 1e-12 * abs(lam)
    _ = p


def test_gmres_against_dense_solve():
    rng = np.random.default_rng(7)
    n = 80
    A = np.eye(n) * 3 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    x, info = fast.gmres(lambda v: A @ v, b, tol=1e-13, restart=20)
    assert info["converged"]
    assert np.abs(x - np.linalg.solve(A, b)).max() < 1e-11


def test_gmres_restart_needed_and_iteration_cap():
    rng = np.random.default_rng(8)
    n = 60
    A = np.diag(np.linspace(1, 50, n)) + 0.1 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    x, info = fast.gmres(lambda v: A @ v, b, tol=1e-12, restart=5, max_iters=3)
    assert not info["converged"] and info["iters"] == 3
    x, info = fast.gmres(lambda v: A @ v, b, tol=1e-12, restart=5, max_iters=5000)
    assert info["converged"] and info["iters"] > 5


def test_fast_tier_fourth_order_at_larger_n():
    errs = []
    for n in (64, 128):
        p = W.config2(n)
        U, V, Q, info = fast.FastTier(p).solve(tol=1e-12)
        errs.append(np.abs(U - p.u_exact).max())
    assert 14.0 < errs[0] / errs[1] < 19.0
