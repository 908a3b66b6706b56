"""Algorithm 1 step by step, with library DST-I transforms as the fast Poisson solver.

Test infrastructure only (see the package docstring).

Follows Section 2.3 and Algorithm 1 in the paper's order:

* the v-equation and u-equation (Sec. 2.2) are solved as Dirichlet problems
  for L_h by discrete sine transforms (Remark 2; Section 4 solver settings);
  L_h is diagonal in the tensor sine basis with eigenvalue
  lambda = sum_a s_a + sum_{a<b} (h_a^2 + h_b^2)/12 s_a s_b,
  s_a(k) = -(4/h_a^2) sin^2(k pi / (2 N_a)), which is L_h = sum_a d_aa +
  sum_{a<b} (h_a^2 + h_b^2)/12 d_aa d_bb read off the stencil weights;
* R(Q) is the boundary residual of Lemma 1;
* ConstructSchurRHS: b = -R(0);  SchurMatVec: Y = R(Q) + b (Algorithm 1);
* matrix-free restarted GMRES on S_h Q = b (modified Gram-Schmidt Arnoldi,
  Givens rotations), then V from Q^m and U from V.

The transforms come from scipy.fft (library primitive); all the rest is
numpy array arithmetic in FP64.
"""
from __future__ import annotations

import time

import numpy as np
import scipy.fft as sfft

from .grid import Grid
from .stencils import laplacian, weighting, apply, ONE_SIDED, ONE_SIDED_GN


def _f(arr, shape):
    return np.zeros(shape) if arr is None else np.asarray(arr, dtype=np.float64)


def laplacian_symbol(n, h, k):
    """Eigenvalue of the compact L_h (homogeneous Dirichlet) on the sine mode with indices
    k = (k_x, k_y[, k_z]) (arrays broadcast together) of a grid with n intervals and spacings
    h: sum_a s_a + sum_{a<b} (h_a^2 + h_b^2)/12 s_a s_b with s_a = -(4/h_a^2) sin^2(k_a pi /
    (2 n_a)), the 1-D second-difference symbol (Sec. 2.2 stencils, App. A recurrence)."""
    dim = len(n)
    S = [-(4.0 / h[a] ** 2) * np.sin(np.asarray(k[a]) * np.pi / (2 * n[a])) ** 2 for a in range(dim)]
    lam = sum(S)
    for a in range(dim):
        for b in range(a + 1, dim):
            lam = lam + (h[a] ** 2 + h[b] ** 2) / 12.0 * S[a] * S[b]
    return lam


def weighting_symbol(n, k):
    """Eigenvalue of the weighting operator M (homogeneous Dirichlet) on the sine mode with
    indices k (arrays broadcast together) of a grid with n intervals: sum over M's offsets o
    of w_o prod_a cos(pi k_a o_a / n_a) (M is symmetric, so each pair of opposite offsets
    turns the mode's shift into a cosine)."""
    dim = len(n)
    out = 0.0
    for o, w in weighting(dim).items():
        term = w
        for a in range(dim):
            if o[a]:
                term = term * np.cos(np.pi * np.asarray(k[a]) * o[a] / n[a])
        out = out + term
    return out


class FastTier:
    """Algorithm 1 with library sine transforms.  A nonzero beta needs a constant alpha:
    the v-equation -L_h V + (beta/alpha) M V = M f is then diagonal in the sine basis with
    the eigenvalue lambda_L - (beta/alpha) mu_M."""

    def __init__(self, problem, workers=None):
        g = Grid(problem.n, problem.lo, problem.hi)
        self.g = g
        self.workers = workers
        self.alpha = _f(problem.alpha, g.nodal_shape)
        beta = getattr(problem, "beta", 0.0)
        if beta is not None and not np.isscalar(beta):
            beta = np.asarray(beta, dtype=np.float64)
            if np.ptp(beta) > 1e-14 * np.abs(beta).max():
                raise ValueError("a variable beta needs the direct tier")
            beta = float(beta.flat[0])
        self.beta = float(beta or 0.0)
        if self.beta != 0.0 and np.ptp(self.alpha) > 1e-14 * np.abs(self.alpha).max():
            raise ValueError("a nonzero beta needs a constant alpha in the fast tier")
        self.c = self.beta / float(self.alpha.flat[0])
        self.f = _f(problem.f, g.nodal_shape)
        self.gD = _f(problem.gD, g.nodal_shape)
        self.gN = _f(problem.gN, g.nodal_shape)
        self.lapgD = _f(problem.lapgD, g.nodal_shape)
        self.navier = tuple(getattr(problem, "navier", ()) or ())
        self.gL = _f(getattr(problem, "gL", None), g.nodal_shape)
        self.L = laplacian(g.h)
        self.M = weighting(g.dim)
        self.lam = self._eigen()
        self.lam_v = self.lam
        if self.c != 0.0:
            grids = np.meshgrid(*[np.arange(1, g.n[a]) for a in reversed(range(g.dim))], indexing="ij")
            self.lam_v = self.lam - self.c * weighting_symbol(g.n, list(reversed(grids)))
        self.inner = tuple(slice(1, m) for m in reversed(g.n))
        # face-interior node coordinates in Q order, per face, as index arrays
        self._qidx = np.array([tuple(reversed(idx)) for idx in g.q_nodes], dtype=np.int64)
        self.Mf = apply(self.M, self.f, g)
        self.matvecs = 0

    # -- fast Poisson solver --------------------------------------------------------------
    def _eigen(self):
        g = self.g
        grids = np.meshgrid(*[np.arange(1, g.n[a]) for a in reversed(range(g.dim))], indexing="ij")
        return laplacian_symbol(g.n, g.h, list(reversed(grids)))

    def poisson(self, G):
        """Interior W with L_int W = G (homogeneous Dirichlet), by DST-I in every axis."""
        Gh = sfft.dstn(G, type=1, workers=self.workers)
        return sfft.idstn(Gh / self.lam, type=1, workers=self.workers)

    # -- boundary values --------------------------------------------------------------------
    def _v_boundary(self, Q):
        """Nodal array: V = Q on face-interior nodes, alpha * lapgD on edges/corners, 0 inside."""
        Vb = self.alpha * self.lapgD
        Vb[self.inner] = 0.0
        Vb[tuple(self._qidx.T)] = Q
        return Vb

    # -- the two subproblems ----------------------------------------------------------------
    def v_solve(self, Q):
        """-L_h V + (beta/alpha) M V = M f at interior nodes with boundary V from Q
        (Algorithm 1, v-equation)."""
        Vb = self._v_boundary(Q)
        Lb = apply(self.L, Vb, self.g)       # boundary contributions of L_h
        rhs = -self.Mf - Lb
        if self.c != 0.0:
            rhs = rhs + self.c * apply(self.M, Vb, self.g)  # and of (beta/alpha) M
        V = Vb.copy()
        Gh = sfft.dstn(rhs, type=1, workers=self.workers)
        V[self.inner] = sfft.idstn(Gh / self.lam_v, type=1, workers=self.workers)
        return V

    def u_solve(self, V):
        """L_h U = M(V/alpha) at interior nodes with U = g_D (Algorithm 1, u-equation)."""
        rhs = apply(self.M, V / self.alpha, self.g)
        Ub = self.gD.copy()
        Ub[self.inner] = 0.0
        rhs -= apply(self.L, Ub, self.g)
        U = self.gD.copy()
        U[self.inner] = self.poisson(rhs)
        return U

    def residual(self, U, Q):
        """R(Q) of Lemma 1 on every face-interior node, in Q order (alpha g_L - Q on a Navier
        face, where V is given)."""
        g = self.g
        R = np.empty(g.n_q)
        for p, b in enumerate(g.q_nodes):
            a, s = g.face_of(b)
            if self.navier and self.navier[2 * a + s]:
                R[p] = g.at(self.alpha, b) * g.at(self.gL, b) - Q[p]
                continue
            step = 1 if s == 0 else -1
            vals = []
            for kk in range(4):
                idx = list(b)
                idx[a] += step * kk
                vals.append(g.at(U, tuple(idx)))
            ha = g.h[a]
            dnn = sum(ONE_SIDED[kk] * vals[kk] for kk in range(4)) / ha ** 2 \
                + ONE_SIDED_GN * g.at(self.gN, b) / ha
            R[p] = g.at(self.alpha, b) * (dnn + g.at(self.lapgD, b)) - Q[p]
        return R

    # -- Algorithm 1 ---------------------------------------------------------------------------
    def R_of(self, Q):
        V = self.v_solve(Q)
        U = self.u_solve(V)
        return self.residual(U, Q)

    def schur_rhs(self):
        """ConstructSchurRHS: b = -R(0)."""
        return -self.R_of(np.zeros(self.g.n_q))

    def schur_matvec(self, Q, b):
        """SchurMatVec: Y = R(Q) + b."""
        self.matvecs += 1
        return self.R_of(Q) + b

    def solve(self, tol=1e-12, restart=30, max_iters=2000, Q0=None):
        t0 = time.perf_counter()
        b = self.schur_rhs()
        Q, info = gmres(lambda q: self.schur_matvec(q, b), b, tol=tol, restart=restart,
                        max_iters=max_iters, x0=Q0)
        V = self.v_solve(Q)
        U = self.u_solve(V)
        info["time_s"] = time.perf_counter() - t0
        return U, V, Q, info


def gmres(matvec, b, tol=1e-12, restart=30, max_iters=2000, x0=None):
    """Restarted GMRES(m): MGS Arnoldi, Givens rotations, stop on ||b - A x|| <= tol ||b||."""
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, {"iters": 0, "relres": 0.0, "converged": True}
    iters = 0
    history = []
    while True:
        r = b - matvec(x) if np.any(x) else b.copy()
        beta = np.linalg.norm(r)
        history.append(beta / bnorm)
        if beta <= tol * bnorm or iters >= max_iters:
            return x, {"iters": iters, "relres": beta / bnorm,
                       "converged": beta <= tol * bnorm, "history": history}
        m = restart
        Vb = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        Vb[0] = r / beta
        j_used = 0
        for j in range(m):
            w = matvec(Vb[j])
            iters += 1
            for i in range(j + 1):
                H[i, j] = np.dot(Vb[i], w)
                w = w - H[i, j] * Vb[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                Vb[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rho = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / rho
            sn[j] = H[j + 1, j] / rho
            H[j, j] = rho
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            j_used = j + 1
            history.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= tol * bnorm or iters >= max_iters:
                break
        y = np.zeros(j_used)
        for i in reversed(range(j_used)):
            y[i] = (g[i] - H[i, i + 1:j_used] @ y[i + 1:]) / H[i, i]
        x = x + Vb[:j_used].T @ y
