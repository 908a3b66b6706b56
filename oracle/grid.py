"""Uniform box grid, interior numbering and the ordering of the augmented unknowns Q.

Test infrastructure only (see the package docstring).

Grid (Section 2): nodes x_i = x_L + i h_x, i = 0..N_x (likewise y, z), with
h_a = (b_a - a_a) / N_a.  Node indices are tuples in axis order (i, j[, k]);
nodal numpy arrays are stored in memory order (z, y, x), x fastest, so node
(i, j, k) is ``arr[k, j, i]``.

Augmented unknowns (Sec. 2.1 augmented variable; Remark 1): one per node in
the *relative interior* of each clamped face (fully clamped box: every face).
Faces are ordered x-, x+, y-, y+[, z-, z+]; inside a face the remaining axes
are traversed row-major with the lowest axis fastest.
"""
from __future__ import annotations

import numpy as np


class Grid:
    def __init__(self, n, lo=None, hi=None):
        self.n = tuple(int(v) for v in n)
        self.dim = len(self.n)
        if self.dim not in (2, 3):
            raise ValueError("dim must be 2 or 3")
        if min(self.n) < 4:
            raise ValueError("the one-sided normal formula needs N_a >= 4")
        self.lo = tuple(float(v) for v in (lo if lo is not None else (0.0,) * self.dim))
        self.hi = tuple(float(v) for v in (hi if hi is not None else (1.0,) * self.dim))
        self.h = tuple((self.hi[a] - self.lo[a]) / self.n[a] for a in range(self.dim))
        self.nint = tuple(m - 1 for m in self.n)          # interior count per axis
        self.n_int = int(np.prod(self.nint))
        self.faces = [(a, s) for a in range(self.dim) for s in (0, 1)]
        self._build_q()

    # -- shapes -------------------------------------------------------------------------
    @property
    def nodal_shape(self):
        return tuple(m + 1 for m in reversed(self.n))

    @property
    def interior_shape(self):
        return tuple(reversed(self.nint))

    def at(self, arr, idx):
        return arr[tuple(reversed(idx))]

    # -- node classes ---------------------------------------------------------------------
    def n_boundary_axes(self, idx):
        return sum(1 for a in range(self.dim) if idx[a] in (0, self.n[a]))

    def is_interior(self, idx):
        return all(0 < idx[a] < self.n[a] for a in range(self.dim))

    def is_face_interior(self, idx):
        return self.n_boundary_axes(idx) == 1

    def interior_index(self, idx):
        """Linear index of an interior node in memory order (x fastest)."""
        lin = 0
        for a in reversed(range(self.dim)):
            lin = lin * self.nint[a] + (idx[a] - 1)
        return lin

    def interior_nodes(self):
        """All interior nodes in memory order (x fastest)."""
        rng = [range(1, self.n[a]) for a in range(self.dim)]
        if self.dim == 2:
            return [(i, j) for j in rng[1] for i in rng[0]]
        return [(i, j, k) for k in rng[2] for j in rng[1] for i in rng[0]]

    # -- augmented unknowns ---------------------------------------------------------------
    def face_nodes(self, face):
        a, s = face
        other = [b for b in range(self.dim) if b != a]
        fixed = 0 if s == 0 else self.n[a]
        out = []
        if self.dim == 2:
            (b,) = other
            for t in range(1, self.n[b]):
                idx = [0, 0]
                idx[a], idx[b] = fixed, t
                out.append(tuple(idx))
        else:
            b1, b2 = other  # b1 < b2, b1 fastest
            for t2 in range(1, self.n[b2]):
                for t1 in range(1, self.n[b1]):
                    idx = [0, 0, 0]
                    idx[a], idx[b1], idx[b2] = fixed, t1, t2
                    out.append(tuple(idx))
        return out

    def _build_q(self):
        self.q_nodes = []
        self.q_face = []
        for fi, face in enumerate(self.faces):
            nodes = self.face_nodes(face)
            self.q_nodes += nodes
            self.q_face += [fi] * len(nodes)
        self.n_q = len(self.q_nodes)
        self.q_of = {idx: p for p, idx in enumerate(self.q_nodes)}

    def face_of(self, idx):
        """(axis, side) of a face-interior node."""
        for a in range(self.dim):
            if idx[a] == 0:
                return (a, 0)
            if idx[a] == self.n[a]:
                return (a, 1)
        raise ValueError("not a boundary node")

    def coords(self):
        return [self.lo[a] + self.h[a] * np.arange(self.n[a] + 1) for a in range(self.dim)]
