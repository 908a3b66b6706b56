"""Plain definition: the coupled HOC system, assembled entry by entry and solved directly.

Test infrastructure only (see the package docstring).

Unknowns (Section 2.2, block system eq-coupled): U at interior nodes, V at
interior nodes, Q at face-interior nodes (Remark 1).  Rows, for a box with
clamped or Navier faces and a constant or nodal beta:

* u-rows (Sec. 2.2, L_h U = M(V/alpha)): at every interior node,
  L_h U - M(V/alpha) = 0, with U = g_D on the boundary.  M reaches the
  face-interior boundary nodes, where V = Q, so the u-rows couple to Q.
* v-rows (Sec. 2.2, -L_h V + M(beta V/alpha) = M f): at every interior node,
  with V = Q on face-interior nodes and, on edges and corners, V = alpha * (Delta u
  from the Dirichlet data) (Remark 1).  M reaches face-interior nodes only, so
  the beta term couples to interior V and to Q.
* q-rows (Lemma 1, boundary residual R): at every face-interior node of a clamped
  face, alpha_b [ (delta_nn U)_b + (tangential part of Delta u)_b ] - Q_b = 0 with the
  one-sided formula of Sec. 2.2, written for the face's outward normal; on a Navier
  face (Delta u = g_L given, eq-bc) V = alpha g_L there, i.e. alpha_b g_L,b - Q_b = 0.

The sign of the Q block follows Lemma 1 (R = alpha[...] - Q, so A22 = -I);
eq-coupled draws that block as +I.  Either sign gives the same solution.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from .grid import Grid
from .stencils import laplacian, weighting, ONE_SIDED, ONE_SIDED_GN


def _field(arr, grid):
    if arr is None:
        return np.zeros(grid.nodal_shape)
    return np.asarray(arr, dtype=np.float64)


class Assembled:
    """The assembled system A x = F with x = [U_int, V_int, Q]."""

    def __init__(self, grid, A, F, alpha, gD, lapgD):
        self.grid, self.A, self.F = grid, A, F
        self.alpha, self.gD, self.lapgD = alpha, gD, lapgD
        n = grid.n_int
        self.su = slice(0, n)
        self.sv = slice(n, 2 * n)
        self.sq = slice(2 * n, 2 * n + grid.n_q)

    # -- nodal reconstruction ----------------------------------------------------------
    def nodal_u(self, x):
        g = self.grid
        U = self.gD.copy()
        inner = tuple(slice(1, m) for m in reversed(g.n))
        U[inner] = x[self.su].reshape(g.interior_shape)
        return U

    def nodal_v(self, x):
        """V on all nodes: interior, Q on faces, alpha*lapgD on edges/corners."""
        g = self.grid
        V = self.alpha * self.lapgD
        inner = tuple(slice(1, m) for m in reversed(g.n))
        V[inner] = x[self.sv].reshape(g.interior_shape)
        q = x[self.sq]
        for p, idx in enumerate(g.q_nodes):
            V[tuple(reversed(idx))] = q[p]
        return V


def assemble(problem) -> Assembled:
    g = Grid(problem.n, problem.lo, problem.hi)
    alpha = _field(problem.alpha, g)
    f = _field(problem.f, g)
    gD = _field(problem.gD, g)
    gN = _field(problem.gN, g)
    lapgD = _field(problem.lapgD, g)
    if alpha.min() <= 0:
        raise ValueError("alpha must be positive")
    beta_in = getattr(problem, "beta", 0.0)
    if beta_in is None or np.isscalar(beta_in):
        beta_const = float(beta_in or 0.0)
        beta = None if beta_const == 0.0 else np.full(g.nodal_shape, beta_const)
    else:  # a variable beta, nodal
        beta = _field(beta_in, g)
    L = laplacian(g.h)
    M = weighting(g.dim)
    n = g.n_int
    N = 2 * n + g.n_q
    rows, cols, vals = [], [], []
    F = np.zeros(N)

    def add(r, c, v):
        rows.append(r)
        cols.append(c)
        vals.append(v)

    def shift(p, o):
        return tuple(p[a] + o[a] for a in range(g.dim))

    for p in g.interior_nodes():
        ip = g.interior_index(p)
        ru, rv = ip, n + ip
        # u-row: L_h U - M(V/alpha) = 0
        for o, w in L.items():
            q = shift(p, o)
            if g.is_interior(q):
                add(ru, g.interior_index(q), w)
            else:
                F[ru] -= w * g.at(gD, q)
        for o, w in M.items():
            q = shift(p, o)
            inv_a = 1.0 / g.at(alpha, q)
            if g.is_interior(q):
                add(ru, n + g.interior_index(q), -w * inv_a)
            elif g.is_face_interior(q):
                add(ru, 2 * n + g.q_of[q], -w * inv_a)
            else:
                raise AssertionError("M never reaches an edge or corner node")
        # v-row: -L_h V + M(beta V / alpha) = M f
        for o, w in L.items():
            q = shift(p, o)
            if g.is_interior(q):
                add(rv, n + g.interior_index(q), -w)
            elif g.is_face_interior(q):
                add(rv, 2 * n + g.q_of[q], -w)
            else:
                F[rv] += w * g.at(alpha, q) * g.at(lapgD, q)
        for o, w in M.items():
            q = shift(p, o)
            F[rv] += w * g.at(f, q)
            if beta is not None:
                c = w * g.at(beta, q) / g.at(alpha, q)
                if g.is_interior(q):
                    add(rv, n + g.interior_index(q), c)
                elif g.is_face_interior(q):
                    add(rv, 2 * n + g.q_of[q], c)
                else:
                    raise AssertionError("M never reaches an edge or corner node")
    # q-rows: alpha_b [ delta_nn U + 11 g_N / (3h) + lapgD ] - Q = 0 (clamped face),
    # alpha_b g_L - Q = 0 (Navier face)
    navier = tuple(getattr(problem, "navier", ()) or ())
    gL = _field(getattr(problem, "gL", None), g)
    for pq, b in enumerate(g.q_nodes):
        r = 2 * n + pq
        a, s = g.face_of(b)
        if navier and navier[2 * a + s]:
            add(r, r, -1.0)
            F[r] = -g.at(alpha, b) * g.at(gL, b)
            continue
        step = 1 if s == 0 else -1
        ha = g.h[a]
        ab = g.at(alpha, b)
        for kk in (1, 2, 3):
            q = list(b)
            q[a] += step * kk
            add(r, g.interior_index(tuple(q)), ab * ONE_SIDED[kk] / ha ** 2)
        add(r, r, -1.0)
        F[r] = -ab * (ONE_SIDED[0] * g.at(gD, b) / ha ** 2
                      + ONE_SIDED_GN * g.at(gN, b) / ha + g.at(lapgD, b))
    A = sps.csr_matrix((vals, (rows, cols)), shape=(N, N))
    A.sum_duplicates()
    return Assembled(g, A, F, alpha, gD, lapgD)


def solve(problem):
    """Direct sparse-LU solve of the coupled system.  Returns (U, V, Q, assembled)."""
    asm = assemble(problem)
    x = spla.splu(asm.A.tocsc()).solve(asm.F)
    return asm.nodal_u(x), asm.nodal_v(x), x[asm.sq].copy(), asm


def schur(problem):
    """Explicit S_h = A22 - A21 A11^{-1} A12 and b = F2 - A21 A11^{-1} F1 (Sec. 2.3, eq-schur).

    Dense; one sparse solve per column of A12.  Small grids only."""
    asm = assemble(problem)
    A = asm.A.tocsr()
    n2 = 2 * asm.grid.n_int
    A11 = A[:n2, :n2].tocsc()
    A12 = A[:n2, n2:].toarray()
    A21 = A[n2:, :n2]
    A22 = A[n2:, n2:].toarray()
    lu = spla.splu(A11)
    X = lu.solve(A12)
    S = A22 - A21 @ X
    b = asm.F[n2:] - A21 @ lu.solve(asm.F[:n2])
    return S, b, asm
