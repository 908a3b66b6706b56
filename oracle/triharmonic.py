"""Triharmonic extension of the augmented scheme (Sec. 4.2, "Triharmonic equation"; Table 5).

Test infrastructure only (see the package docstring).

Delta^3 u = f is split as Delta u = v, Delta v = w, Delta w = f.  The data fix u and v on
every face (on a clamped face v = u_nn + Delta_tau u from u_nn and u; on a Navier face Delta u
is given) and w on the Navier faces, edges and corners (Delta^2 u given); on the face
interiors of clamped faces w is the augmented unknown q (Sec. 4.2: q = w, which also
satisfies the augmented equation q = Delta^2 u).  Each of the three Poisson equations is
discretised by the fourth-order compact scheme of Sec. 2.2 (L_h X = M rhs).

The paper gives no discrete form of the augmented equation.  Reading taken here, in the
way Lemma 1 closes the biharmonic scheme (a second-kind row, Q with coefficient -1): on a
clamped face-interior node b with inward normal coordinate xi and spacing h,

    R_b = h^-4 ( sum_{k=1..4} a_k U_k + a_0 g_D + c_1 h u_xi + c_2 h^2 u_xixi )
          + (Delta^2 u - u_xixixixi)_b - Q_b = 0,

the one-sided fourth normal derivative of U that uses all three clamped data (u, u_n = -u_xi
for the outward g_N, and u_nn) and the nearest four interior nodes, plus the tangential part
of Delta^2 u that the data fix.  Its weights are the unique ones that are exact for
polynomials of degree <= 6 along the normal (Taylor moment conditions):
a = (11669/144, -104, 57/2, -56/9, 11/16), c_1 = 755/12, c_2 = 35/2; the first neglected
moment is 5/21 (error 5/21 h^3 u^(7)).  On a Navier face the row is bilap_b - Q_b = 0.

Tiers: ``assemble``/``solve`` (the coupled system for U, V, W and Q, sparse LU) and
``TriFast`` (the Schur system S Q = b matrix-free: three sine-transform Poisson solves per
matvec, plain GMRES), pinned to each other, to polynomial exactness and to Table 5.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import scipy.fft as sfft
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from .fast import gmres, laplacian_symbol
from .grid import Grid
from .stencils import apply, laplacian, weighting

# h^4 u'''' = a_0 U_0 + sum_k a_k U_k + c_1 (h u_xi) + c_2 (h^2 u_xixi) + O(h^7)
ONE_SIDED4 = (Fraction(11669, 144), Fraction(-104), Fraction(57, 2), Fraction(-56, 9), Fraction(11, 16))
ONE_SIDED4_D1 = Fraction(755, 12)   # weight of h * u_xi (inward first derivative)
ONE_SIDED4_D2 = Fraction(35, 2)     # weight of h^2 * u_xixi


def _f(arr, shape):
    return np.zeros(shape) if arr is None else np.asarray(arr, dtype=np.float64)


class _Data:
    """Nodal data of a TriProblem on its grid, with the clamped/Navier face flags."""

    def __init__(self, problem):
        g = Grid(problem.n, problem.lo, problem.hi)
        self.g = g
        sh = g.nodal_shape
        self.f = _f(problem.f, sh)
        self.gD = _f(problem.gD, sh)
        self.gN = _f(problem.gN, sh)
        self.gNN = _f(problem.gNN, sh)
        self.lapu = _f(problem.lapu, sh)
        self.bilap = _f(problem.bilap, sh)
        self.tang4 = _f(problem.tang4, sh)
        nav = tuple(problem.navier) if problem.navier else (False,) * (2 * g.dim)
        self.navier = nav

    def is_navier(self, b):
        a, s = self.g.face_of(b)
        return bool(self.navier[2 * a + s])

    def inward(self, b, k):
        """The node k steps inward from face-interior node b."""
        a, s = self.g.face_of(b)
        idx = list(b)
        idx[a] += k if s == 0 else -k
        return tuple(idx)

    def q_data(self, b):
        """Known part of the q-row at a clamped face-interior node (everything but U_1..U_4
        and Q)."""
        g = self.g
        a, _ = g.face_of(b)
        h = g.h[a]
        u_xi = -g.at(self.gN, b)  # outward g_N = -du/dxi
        return (float(ONE_SIDED4[0]) * g.at(self.gD, b) + float(ONE_SIDED4_D1) * h * u_xi
                + float(ONE_SIDED4_D2) * h * h * g.at(self.gNN, b)) / h ** 4 + g.at(self.tang4, b)


class Assembled:
    def __init__(self, data, A, F):
        self.d, self.A, self.F = data, A, F
        g = data.g
        self.n = g.n_int

    def nodal_u(self, x):
        g = self.d.g
        U = self.d.gD.copy()
        inner = tuple(slice(1, m) for m in reversed(g.n))
        U[inner] = x[:self.n].reshape(g.interior_shape)
        return U


def assemble(problem) -> Assembled:
    """The coupled system for x = [U_int, V_int, W_int, Q] (Q on every face interior; a
    Navier face's rows fix Q to Delta^2 u there)."""
    d = _Data(problem)
    g = d.g
    L = laplacian(g.h)
    M = weighting(g.dim)
    n = g.n_int
    N = 3 * n + g.n_q
    rows, cols, vals = [], [], []
    F = np.zeros(N)

    def add(r, c, v):
        rows.append(r)
        cols.append(c)
        vals.append(v)

    def shift(p, o):
        return tuple(p[a] + o[a] for a in range(g.dim))

    def w_col(q):
        """Column of W at node q, or None with its known value (edges, corners)."""
        if g.is_interior(q):
            return 2 * n + g.interior_index(q), 0.0
        if g.is_face_interior(q):
            return 3 * n + g.q_of[q], 0.0
        return None, g.at(d.bilap, q)

    for p in g.interior_nodes():
        ip = g.interior_index(p)
        ru, rv, rw = ip, n + ip, 2 * n + ip
        for o, w in L.items():
            q = shift(p, o)
            if g.is_interior(q):
                iq = g.interior_index(q)
                add(ru, iq, w)
                add(rv, n + iq, w)
                add(rw, 2 * n + iq, w)
            else:
                F[ru] -= w * g.at(d.gD, q)
                F[rv] -= w * g.at(d.lapu, q)
                c, val = w_col(q)
                if c is None:
                    F[rw] -= w * val
                else:
                    add(rw, c, w)
        for o, w in M.items():
            q = shift(p, o)
            # u-row: L_h U - M V = 0;  v-row: L_h V - M W = 0;  w-row: L_h W = M f
            if g.is_interior(q):
                add(ru, n + g.interior_index(q), -w)
            else:
                F[ru] += w * g.at(d.lapu, q)
            c, val = w_col(q)
            if c is None:
                F[rv] += w * val
            else:
                add(rv, c, -w)
            F[rw] += w * g.at(d.f, q)
    for pq, b in enumerate(g.q_nodes):
        r = 3 * n + pq
        add(r, r, -1.0)
        if d.is_navier(b):
            F[r] = -g.at(d.bilap, b)
            continue
        a, _ = g.face_of(b)
        h = g.h[a]
        for k in (1, 2, 3, 4):
            add(r, g.interior_index(d.inward(b, k)), float(ONE_SIDED4[k]) / h ** 4)
        F[r] = -d.q_data(b)
    A = sps.csr_matrix((vals, (rows, cols)), shape=(N, N))
    A.sum_duplicates()
    return Assembled(d, A, F)


def solve(problem):
    """Direct sparse-LU solve.  Returns (U nodal, Q, assembled)."""
    asm = assemble(problem)
    x = spla.splu(asm.A.tocsc()).solve(asm.F)
    return asm.nodal_u(x), x[3 * asm.n:].copy(), asm


def schur(problem):
    """Explicit S = A22 - A21 A11^-1 A12 and b = F2 - A21 A11^-1 F1 (dense, small grids)."""
    asm = assemble(problem)
    A = asm.A.tocsr()
    n3 = 3 * asm.n
    A11 = A[:n3, :n3].tocsc()
    A12 = A[:n3, n3:].toarray()
    A21 = A[n3:, :n3]
    A22 = A[n3:, n3:].toarray()
    lu = spla.splu(A11)
    S = A22 - A21 @ lu.solve(A12)
    b = asm.F[n3:] - A21 @ lu.solve(asm.F[:n3])
    return S, b, asm


class TriFast:
    """The Schur system of the triharmonic scheme, matrix-free: R(Q) from three Dirichlet
    solves for the compact L_h by sine transforms (W from Q, V from W, U from V), then the
    q-rows; S Q = R(Q) - R(0), b = -R(0); plain restarted GMRES."""

    def __init__(self, problem, workers=None):
        self.d = d = _Data(problem)
        g = d.g
        self.g = g
        self.workers = workers
        self.L = laplacian(g.h)
        self.M = weighting(g.dim)
        grids = np.meshgrid(*[np.arange(1, g.n[a]) for a in reversed(range(g.dim))], indexing="ij")
        self.lam = laplacian_symbol(g.n, g.h, list(reversed(grids)))
        self.inner = tuple(slice(1, m) for m in reversed(g.n))
        self._qidx = tuple(np.array([tuple(reversed(b)) for b in g.q_nodes], dtype=np.int64).T)
        self.nav = np.array([d.is_navier(b) for b in g.q_nodes])
        # per q node: the four inward interior nodes (memory order) and h^-4 weights
        self._inw = [tuple(np.array([tuple(reversed(d.inward(b, k))) for b in g.q_nodes]).T)
                     for k in (1, 2, 3, 4)]
        hq = np.array([g.h[g.face_of(b)[0]] for b in g.q_nodes])
        self._w4 = [float(ONE_SIDED4[k]) / hq ** 4 for k in (1, 2, 3, 4)]
        self._known = np.array([d.bilap[tuple(reversed(b))] if d.is_navier(b) else d.q_data(b)
                                for b in g.q_nodes])

    def poisson(self, G):
        Gh = sfft.dstn(G, type=1, workers=self.workers)
        return sfft.idstn(Gh / self.lam, type=1, workers=self.workers)

    def _dirichlet(self, src_nodal, bnd):
        """X with L_h X = M src at interior nodes and X = bnd on the boundary."""
        B = bnd.copy()
        B[self.inner] = 0.0
        X = bnd.copy()
        X[self.inner] = self.poisson(apply(self.M, src_nodal, self.g) - apply(self.L, B, self.g))
        return X

    def fields(self, Q, homogeneous=False):
        d = self.d
        z = np.zeros(self.g.nodal_shape)
        Wb = z.copy() if homogeneous else d.bilap.copy()
        Wb[self._qidx] = Q
        W = self._dirichlet(z if homogeneous else d.f, Wb)
        V = self._dirichlet(W, z if homogeneous else d.lapu)
        U = self._dirichlet(V, z if homogeneous else d.gD)
        return U, V, W

    def R_of(self, Q, homogeneous=False):
        U, _, _ = self.fields(Q, homogeneous)
        R = sum(w * U[idx] for w, idx in zip(self._w4, self._inw))
        R = np.where(self.nav, 0.0, R)
        if not homogeneous:
            R = R + self._known
        return R - Q

    def schur_rhs(self):
        return -self.R_of(np.zeros(self.g.n_q))

    def schur_matvec(self, Q):
        return self.R_of(Q, homogeneous=True)

    def solve(self, tol=1e-12, restart=60, max_iters=4000):
        b = self.schur_rhs()
        Q, info = gmres(self.schur_matvec, b, tol=tol, restart=restart, max_iters=max_iters)
        U, _, _ = self.fields(Q)
        return U, Q, info
