"""Compact operators of Section 2.2, as explicit offset -> weight tables.

Test infrastructure only (see the package docstring).

* ``laplacian(h)``: the fourth-order compact Laplacian L_h.
  3-D: the planes L_{k-1}, L_k, L_{k+1} of Section 2.2 with the prefactor 1/12
  (the printed 1/2 is inconsistent with the weighting operator M: with 1/2 the
  truncation error does not vanish as h -> 0; 1/12 is the consistent value and
  is the one pinned by the truncation and polynomial-exactness tests).
  2-D: the nine-point compact Laplacian.  The printed 2-D operator of
  Section 3.1 lacks the corner weights; the nine-point stencil is the one whose
  sine-mode recurrence matches the coefficients (4 + 2 cos theta) and
  (8 cos theta - 20) of the proof of Lemma 4 in Appendix A, and the value
  cosh(alpha_k) = (5 - 2 cos theta)/(2 + cos theta) of Section 3.1.
* ``weighting(dim)``: the operator M (Sec. 2.2 in 3-D; Sec. 3.1 in 2-D).
* ``ONE_SIDED``: weights of the one-sided second normal derivative with
  Neumann data, Sec. 2.2: (delta_xx U)_0 = h^-2 (-85/18 U0 + 6 U1 - 3/2 U2
  + 2/9 U3) + (11 / (3h)) g_N, with g_N the outward normal derivative.
* ``apply(table, nodal, grid)``: a table applied at every interior node of a
  nodal array (Frobenius-product action, eqs. (Lh-action), (M-action)).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

ONE_SIDED = (-85.0 / 18.0, 6.0, -1.5, 2.0 / 9.0)
ONE_SIDED_GN = 11.0 / 3.0


def laplacian(h):
    """Offset (axis order) -> weight of L_h for spacings h = (h_x, h_y[, h_z]).

    Works with floats or with fractions.Fraction spacings (exact weights)."""
    dim = len(h)
    if dim == 2:
        ix2, iy2 = 1 / h[0] ** 2, 1 / h[1] ** 2
        t = {}
        for sx in (-1, 1):
            for sy in (-1, 1):
                t[(sx, sy)] = (ix2 + iy2) / 12
            t[(sx, 0)] = (10 * ix2 - 2 * iy2) / 12
            t[(0, sx)] = (10 * iy2 - 2 * ix2) / 12
        t[(0, 0)] = -20 * (ix2 + iy2) / 12
        return t
    ix2, iy2, iz2 = (1 / v ** 2 for v in h)
    t = {}
    # planes k +- 1 (Sec. 2.2, L_{k+-1}), entries read row by row: j+1, j, j-1
    for r in (-1, 1):
        t[(0, 1, r)] = (iy2 + iz2) / 12
        t[(-1, 0, r)] = (ix2 + iz2) / 12
        t[(0, 0, r)] = (8 * iz2 - 2 * ix2 - 2 * iy2) / 12
        t[(1, 0, r)] = (ix2 + iz2) / 12
        t[(0, -1, r)] = (iy2 + iz2) / 12
    # plane k (Sec. 2.2, L_k)
    for sx in (-1, 1):
        for sy in (-1, 1):
            t[(sx, sy, 0)] = (ix2 + iy2) / 12
    for s in (-1, 1):
        t[(0, s, 0)] = (8 * iy2 - 2 * ix2 - 2 * iz2) / 12
        t[(s, 0, 0)] = (8 * ix2 - 2 * iy2 - 2 * iz2) / 12
    t[(0, 0, 0)] = -16 * (ix2 + iy2 + iz2) / 12
    return t


def weighting(dim, exact=False):
    """Offset -> weight of M: (1/12)(8 centre + 4 neighbours) in 2-D, (1/12)(6 + 6) in 3-D."""
    one = Fraction(1) if exact else 1.0
    t = {}
    zero = (0,) * dim
    t[zero] = one * (8 if dim == 2 else 6) / 12
    for a in range(dim):
        for s in (-1, 1):
            o = [0] * dim
            o[a] = s
            t[tuple(o)] = one / 12
    return t


def apply(table, nodal, grid):
    """sum_o w_o W(p + o) at every interior node p; returns the interior array."""
    d = grid.dim
    out = np.zeros(grid.interior_shape)
    for off, w in table.items():
        sl = []
        for a in reversed(range(d)):
            lo = 1 + off[a]
            sl.append(slice(lo, lo + grid.nint[a]))
        out += w * nodal[tuple(sl)]
    return out
