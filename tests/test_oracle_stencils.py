"""Pins for the oracle's compact operators (CPU).

Every check compares against mathematics the paper fixes, not against the
oracle's own formulas: exactness on polynomials (rational arithmetic),
truncation order, the sine-mode recurrence printed in Appendix A, and the
moments of the one-sided normal formula of Section 2.2.
"""
import itertools
import json
import math
import os
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import stencils
from oracle.grid import Grid

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _monomials(dim, deg):
    for e in itertools.product(range(deg + 1), repeat=dim):
        if sum(e) == deg:
            yield e


def _mono_val(e, pt):
    v = F(1)
    for ea, xa in zip(e, pt):
        v *= xa ** ea
    return v


def _mono_lap(e, pt):
    tot = F(0)
    for a in range(len(e)):
        if e[a] >= 2:
            e2 = list(e)
            e2[a] -= 2
            tot += e[a] * (e[a] - 1) * _mono_val(e2, pt)
    return tot


def _residual_exact(e, h, pt):
    """L_h p - M Delta p at pt, exactly, for the monomial with exponents e."""
    L = stencils.laplacian(h)
    M = stencils.weighting(len(h), exact=True)
    shift = lambda o: tuple(pt[a] + o[a] * h[a] for a in range(len(h)))
    lhs = sum(w * _mono_val(e, shift(o)) for o, w in L.items())
    rhs = sum(w * _mono_lap(e, shift(o)) for o, w in M.items())
    return lhs - rhs


@pytest.mark.parametrize("dim", [2, 3])
def test_compact_laplacian_exact_on_degree_le5(dim):
    # anisotropic spacings and an off-origin point, exact rational arithmetic
    h = (F(1, 7), F(1, 5), F(2, 9))[:dim]
    pt = (F(3, 11), F(-2, 13), F(5, 17))[:dim]
    for deg in range(6):
        for e in _monomials(dim, deg):
            assert _residual_exact(e, h, pt) == 0, (deg, e)


@pytest.mark.parametrize("dim", [2, 3])
def test_compact_laplacian_not_exact_at_degree6(dim):
    h = (F(1, 7), F(1, 5), F(2, 9))[:dim]
    pt = (F(3, 11), F(-2, 13), F(5, 17))[:dim]
    bad = [e for e in _monomials(dim, 6) if _residual_exact(e, h, pt) != 0]
    assert bad, "a fourth-order compact operator must fail at some degree-6 monomial"


@pytest.mark.parametrize("dim", [2, 3])
def test_truncation_error_fourth_order(dim):
    # L_h u - M Delta u for a smooth non-polynomial u: O(h^4) (ratio ~16 per halving)
    def u(*x):
        return math.sin(1.3 * x[0] + 0.4) * math.exp(0.7 * x[1]) * (math.cos(0.9 * x[2]) if dim == 3 else 1.0)

    def lap(*x):
        c = 1.3 ** 2 - 0.7 ** 2 + (0.9 ** 2 if dim == 3 else 0.0)
        return -c * u(*x)

    pt = (0.31, 0.27, 0.44)[:dim]
    errs = []
    for hh in (0.04, 0.02, 0.01):
        h = (hh, 1.5 * hh, 0.8 * hh)[:dim]
        L = stencils.laplacian(h)
        M = stencils.weighting(dim)
        sh = lambda o: tuple(pt[a] + o[a] * h[a] for a in range(dim))
        r = sum(w * u(*sh(o)) for o, w in L.items()) - sum(w * lap(*sh(o)) for o, w in M.items())
        errs.append(abs(r))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 13.0 < r1 < 20.0 and 13.0 < r2 < 20.0, errs


def test_printed_half_prefactor_is_inconsistent():
    # The 3-D planes printed with prefactor 1/2 do not approximate M Delta u:
    # the residual stays O(1) under refinement.  With 1/12 it vanishes (test above).
    dim = 3
    u = lambda x, y, z: math.sin(x + 2 * y) * math.cos(z)
    lap = lambda x, y, z: -6.0 * u(x, y, z)
    pt = (0.2, 0.3, 0.4)
    res = []
    for hh in (0.02, 0.01):
        h = (hh, hh, hh)
        L = {o: 6.0 * w for o, w in stencils.laplacian(h).items()}  # 1/2 = 6 * 1/12
        M = stencils.weighting(dim)
        sh = lambda o: tuple(pt[a] + o[a] * h[a] for a in range(dim))
        res.append(abs(sum(w * u(*sh(o)) for o, w in L.items())
                       - sum(w * lap(*sh(o)) for o, w in M.items())))
    assert min(res) > 1.0


@pytest.mark.parametrize("theta", [0.3, 1.1, 2.5])
def test_2d_sine_mode_recurrence_matches_appendix(theta):
    # L_h psi with psi_{i,j} = c_i sin(theta j), h_x = h_y = h: the coefficient of
    # c_{i-1}, c_i, c_{i+1} in units of 1/(6 h^2) is (4 + 2cos), (8cos - 20), (4 + 2cos).
    h = 0.1
    L = stencils.laplacian((h, h))
    coef = {-1: 0.0, 0: 0.0, 1: 0.0}
    for (ox, oy), w in L.items():
        coef[ox] += w * math.cos(theta * oy)   # sin(theta (j+oy)) pairs to cos(theta oy) sin(theta j)
    scale = 6 * h * h
    assert coef[-1] * scale == pytest.approx(4 + 2 * math.cos(theta), rel=1e-13)
    assert coef[1] * scale == pytest.approx(4 + 2 * math.cos(theta), rel=1e-13)
    assert coef[0] * scale == pytest.approx(8 * math.cos(theta) - 20, rel=1e-13)
    # and cosh(alpha) = (5 - 2cos)/(2 + cos) solves the recurrence
    ca = (5 - 2 * math.cos(theta)) / (2 + math.cos(theta))
    assert -coef[0] / (2 * coef[1]) == pytest.approx(ca, rel=1e-13)


def test_one_sided_normal_formula_moments():
    w = [F(s) for s in GOLD["one_sided_formula"]["weights"]]
    assert [float(x) for x in w] == list(stencils.ONE_SIDED)
    assert float(F(GOLD["one_sided_formula"]["neumann_weight"])) == stencils.ONE_SIDED_GN
    mom = [sum(w[k] * F(k) ** p for k in range(4)) / math.factorial(p) for p in range(6)]
    # sum a_k U_k / h^2 = (11/3) u_x / h + u_xx + 0 + 0 + (h^3/10) u^(5) + ...
    assert mom[:5] == [0, F(11, 3), 1, 0, 0]
    assert mom[5] == F(1, 10)


def test_one_sided_formula_exact_for_quartics_outward_normal():
    # On the low face the outward derivative is -u_x; on the high face +u_x.
    p = lambda x: 0.3 - 1.2 * x + 0.7 * x ** 2 - 0.4 * x ** 3 + 0.25 * x ** 4
    dp = lambda x: -1.2 + 1.4 * x - 1.2 * x ** 2 + 1.0 * x ** 3
    d2p = lambda x: 1.4 - 2.4 * x + 3.0 * x ** 2
    h, x0, x1 = 0.05, 0.1, 0.9
    a = stencils.ONE_SIDED
    lo = sum(a[k] * p(x0 + k * h) for k in range(4)) / h ** 2 + stencils.ONE_SIDED_GN * (-dp(x0)) / h
    hi = sum(a[k] * p(x1 - k * h) for k in range(4)) / h ** 2 + stencils.ONE_SIDED_GN * (dp(x1)) / h
    assert lo == pytest.approx(d2p(x0), rel=1e-10)
    assert hi == pytest.approx(d2p(x1), rel=1e-10)


def test_weighting_operator_matches_paper():
    M3 = stencils.weighting(3, exact=True)
    assert M3[(0, 0, 0)] == F(6, 12) and all(M3[o] == F(1, 12) for o in M3 if o != (0, 0, 0))
    assert len(M3) == 7
    M2 = stencils.weighting(2, exact=True)
    assert M2[(0, 0)] == F(8, 12) and len(M2) == 5


def test_grid_q_layout():
    g = Grid((5, 6, 7))
    # faces x-, x+, y-, y+, z-, z+ ; sizes (Ny-1)(Nz-1), (Nx-1)(Nz-1), (Nx-1)(Ny-1)
    assert g.n_q == 2 * (5 * 6) + 2 * (4 * 6) + 2 * (4 * 5)
    assert g.q_nodes[0] == (0, 1, 1) and g.q_nodes[1] == (0, 2, 1)   # y fastest on x faces
    off = 2 * 30
    assert g.q_nodes[off] == (1, 0, 1) and g.q_nodes[off + 1] == (2, 0, 1)
    off += 2 * 24
    assert g.q_nodes[off] == (1, 1, 0) and g.q_nodes[off + 1] == (2, 1, 0)
    assert len(set(g.q_nodes)) == g.n_q
    assert all(g.is_face_interior(b) for b in g.q_nodes)
