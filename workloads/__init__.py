"""Seeded, synthetic problem generators shared by the oracle and the GPU path.

This module holds the *inputs* only: analytic coefficient fields alpha, the
manufactured solutions u, and the data that the model problem of Section 2
(eq. (1) with the clamped conditions (eq-bc)) derives from them:

    f      = -Delta(alpha Delta u) + beta Delta u  (beta a constant, 0 unless given)
    g_D    = u on the boundary
    g_N    = outward normal derivative of u on the relative interior of each face
    lapgD  = on face-interior nodes, the tangential part of Delta u (what the
             Dirichlet data fixes, Sec. 2.2 boundary Laplacian decomposition);
             on edges and corners, the full Delta u (Remark 1)

Nothing here discretises anything: no stencil, transform or solver lives in
this module, so it carries none of the method's arithmetic.  Arrays are nodal,
in memory order (z, y, x) with x fastest, and can be produced either as numpy
arrays (host) or as torch tensors on a device (for the large grids), using the
same symbolic derivation.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass, field
from typing import Any, Optional, Sequence

import numpy as np

__all__ = [
    "Problem", "manufactured", "config1", "config2", "config3", "config4_specs",
    "config4_instance", "cavity", "plate", "poly_exact", "node_coords", "example1",
    "high_wavenumber", "example2", "example3", "TriProblem", "triharmonic", "example3_tri",
]


@dataclass
class Problem:
    """One clamped problem on a box: grid, coefficients and data (nodal arrays).

    The equation is -Delta(alpha Delta u) + beta Delta u = f with beta a constant or a nodal
    array.  Every face
    carries u = g_D; a clamped face also u_n = g_N, a Navier face (navier[f]) Delta u = g_L
    instead (the boundary conditions eq-bc, with the Navier part of the boundary).

    n: intervals per axis, axis order (x, y[, z]).  lo/hi: box corners.
    Arrays are numpy (host) or torch tensors; None means identically zero.
    u_exact / v_exact are the analytic solution and v = alpha*Delta u sampled
    at the nodes when known (None otherwise).
    """
    n: tuple
    lo: tuple
    hi: tuple
    alpha: Any
    f: Any
    gD: Any = None
    gN: Any = None
    lapgD: Any = None
    u_exact: Any = None
    v_exact: Any = None
    name: str = ""
    meta: dict = field(default_factory=dict)
    beta: Any = 0.0      # constant, or a nodal array (variable beta)
    navier: tuple = ()   # per face (x-, x+, y-, y+[, z-, z+]): True = Navier (Delta u = g_L), else clamped
    gL: Any = None       # nodal Delta u, read on the face-interior nodes of Navier faces

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def h(self) -> tuple:
        return tuple((b - a) / m for a, b, m in zip(self.lo, self.hi, self.n))


def node_coords(n: Sequence[int], lo: Sequence[float], hi: Sequence[float]):
    """1-D node coordinates x_i = x_L + i h_x, i = 0..N_x, per axis (Sec. 2, grid)."""
    return [lo[a] + (hi[a] - lo[a]) * np.arange(n[a] + 1) / n[a] for a in range(len(n))]


# --------------------------------------------------------------------------------------
# symbolic derivation (sympy), cached per expression
# --------------------------------------------------------------------------------------

def _symbols(dim):
    import sympy as sp
    return sp.symbols("x y z")[:dim]


@functools.lru_cache(maxsize=None)
def _derive(alpha_src: str, u_src: str, dim: int, params: tuple = ()):
    """Derive f = -Delta(alpha Delta u), Delta u, grad u for string expressions."""
    import sympy as sp
    X = _symbols(dim)
    ns = {s.name: s for s in X}
    ns.update({p: sp.Symbol(p) for p in params})
    ns.update({"pi": sp.pi, "sin": sp.sin, "cos": sp.cos, "exp": sp.exp, "sqrt": sp.sqrt})
    alpha = sp.sympify(alpha_src, locals=ns)
    u = sp.sympify(u_src, locals=ns)
    lap = lambda w: sum(sp.diff(w, s, 2) for s in X)
    lu = lap(u)
    v = alpha * lu
    f = -lap(v)
    exprs = {
        "alpha": alpha, "u": u, "lapu": lu, "v": v, "f": f,
        **{f"du{a}": sp.diff(u, X[a]) for a in range(dim)},
        **{f"d2u{a}": sp.diff(u, X[a], 2) for a in range(dim)},
    }
    return X, tuple(sp.Symbol(p) for p in params), exprs


def _lambdify(expr, X, P, xp_name):
    import sympy as sp
    if xp_name == "torch":
        import torch
        mod = {"sin": torch.sin, "cos": torch.cos, "exp": torch.exp, "pi": math.pi,
               "sqrt": torch.sqrt}
    else:
        mod = {"sin": np.sin, "cos": np.cos, "exp": np.exp, "pi": math.pi, "sqrt": np.sqrt}
    return sp.lambdify(list(X) + list(P), expr, modules=[mod, "math"], cse=True)


@functools.lru_cache(maxsize=None)
def _expr_fn(src, dim, xp_name):
    """A plain expression in x, y[, z] (no derivatives), e.g. a variable beta."""
    import sympy as sp
    X = _symbols(dim)
    ns = {s.name: s for s in X}
    ns.update({"pi": sp.pi, "sin": sp.sin, "cos": sp.cos, "exp": sp.exp, "sqrt": sp.sqrt})
    return _lambdify(sp.sympify(src, locals=ns), X, (), xp_name)


@functools.lru_cache(maxsize=None)
def _fn(alpha_src, u_src, dim, params, key, xp_name):
    X, P, exprs = _derive(alpha_src, u_src, dim, params)
    return _lambdify(exprs[key], X, P, xp_name)


class _Eval:
    """Evaluate derived expressions on (sub)grids with numpy or torch."""

    def __init__(self, alpha_src, u_src, dim, params=(), pvals=(), xp="numpy",
                 device=None, dtype=None):
        self.a, self.u, self.dim = alpha_src, u_src, dim
        self.params, self.pvals = tuple(params), tuple(pvals)
        self.xp, self.device = xp, device
        self.dtype = dtype

    def coords(self, c1d, axis):
        """Reshape a 1-D coordinate array to broadcast along `axis` (memory order z,y,x)."""
        shape = [1] * self.dim
        shape[self.dim - 1 - axis] = len(c1d)
        if self.xp == "torch":
            import torch
            return torch.as_tensor(np.asarray(c1d), dtype=torch.float64,
                                   device=self.device).reshape(shape)
        return np.asarray(c1d, dtype=np.float64).reshape(shape)

    def __call__(self, key, cs):
        fn = _fn(self.a, self.u, self.dim, self.params, key, self.xp)
        out = fn(*cs, *self.pvals)
        if self.xp == "torch":
            import torch
            shape = tuple(torch.broadcast_shapes(*[tuple(c.shape) for c in cs]))
        else:
            shape = np.broadcast_shapes(*[c.shape for c in cs])
        return self._full(out, shape)

    def expr(self, src, cs):
        """Sample a plain expression (e.g. a variable beta) on the coordinates cs."""
        out = _expr_fn(src, self.dim, self.xp)(*cs)
        if self.xp == "torch":
            import torch
            shape = tuple(torch.broadcast_shapes(*[tuple(c.shape) for c in cs]))
        else:
            shape = np.broadcast_shapes(*[c.shape for c in cs])
        return self._full(out, shape)

    def _full(self, val, shape):
        if self.xp == "torch":
            import torch
            if not torch.is_tensor(val):
                val = torch.tensor(float(val), dtype=torch.float64, device=self.device)
            return val.to(torch.float64).expand(shape).contiguous()
        val = np.asarray(val, dtype=np.float64)
        return np.ascontiguousarray(np.broadcast_to(val, shape))


def _zeros(ev, shape):
    if ev.xp == "torch":
        import torch
        return torch.zeros(shape, dtype=torch.float64, device=ev.device)
    return np.zeros(shape)


def _boundary_data(ev: _Eval, n, c1d, want_gl=False):
    """Nodal g_D, g_N, lapgD (and with want_gl the full Delta u on every boundary node, the
    Navier data g_L) built from boundary evaluations only (O(N^{d-1}) work).

    Returns None for fields that vanish identically on the boundary."""
    dim = len(n)
    shape = tuple(n[a] + 1 for a in reversed(range(dim)))
    gD = _zeros(ev, shape)
    gN = _zeros(ev, shape)
    lap = _zeros(ev, shape)
    gl = _zeros(ev, shape) if want_gl else None
    mod = ev.xp == "torch"

    def sl(axis, idx):
        s = [slice(None)] * dim
        s[dim - 1 - axis] = slice(idx, idx + 1)
        return tuple(s)

    for a in range(dim):
        for side, idx in ((0, 0), (1, n[a])):
            cs = [ev.coords(c1d[b], b) if b != a else ev.coords(c1d[a][idx:idx + 1], a)
                  for b in range(dim)]
            u_b = ev("u", cs)
            gD[sl(a, idx)] = u_b
            # outward normal derivative: -d/dx_a on the low side, +d/dx_a on the high side
            du = ev(f"du{a}", cs)
            gN_b = -du if side == 0 else du
            lapu = ev("lapu", cs)
            tang = lapu - ev(f"d2u{a}", cs)
            # face-interior nodes only for g_N / tangential Laplacian
            inner = [slice(None)] * dim
            for b in range(dim):
                if b != a:
                    inner[dim - 1 - b] = slice(1, n[b])
            inner = tuple(inner)
            tgt = sl(a, idx)
            gsub = gN[tgt]
            gsub[inner] = gN_b[inner]
            gN[tgt] = gsub
            lsub = lap[tgt]
            # edges/corners get full Delta u (Remark 1); face interior the tangential part
            lsub[...] = lapu
            lsub[inner] = tang[inner]
            lap[tgt] = lsub
            if want_gl:
                gl[tgt] = lapu
    # Fields whose boundary values are pure rounding noise (e.g. sin(pi*1.0) ~ 1e-16
    # instead of 0) are reported as identically zero.
    out = []
    for arr in (gD, gN, lap):
        mx = float(arr.abs().max()) if mod else float(np.abs(arr).max())
        out.append(None if mx < 1e-12 else arr)
    if want_gl:
        out.append(gl)
    return out


def manufactured(alpha_src: str, u_src: str, n: Sequence[int], lo=None, hi=None, *,
                 params=(), pvals=(), xp="numpy", device=None, with_exact=True,
                 chunk=None, name="", beta=0.0, navier=()):
    """Sample a manufactured clamped problem.

    alpha_src/u_src: expressions in x, y[, z] (and `params`).  f follows the
    paper's sign convention of eq. (1), f = -Delta(alpha Delta u) + beta Delta u; beta is a
    constant or an expression in x, y[, z] (then Problem.beta is its nodal sample).
    navier: per face, True for a Navier face (g_L = Delta u sampled).
    xp = "numpy" gives host
    arrays; xp = "torch" builds the nodal fields on `device` (in z-chunks of
    `chunk` planes for large 3-D grids).
    """
    dim = len(n)
    lo = tuple(lo) if lo is not None else (0.0,) * dim
    hi = tuple(hi) if hi is not None else (1.0,) * dim
    ev = _Eval(alpha_src, u_src, dim, params, pvals, xp, device)
    c1d = node_coords(n, lo, hi)
    shape = tuple(n[a] + 1 for a in reversed(range(dim)))
    var_beta = isinstance(beta, str)
    beta_src = beta
    keys = ["alpha", "f"] + (["u", "v"] if with_exact else []) + (["lapu"] if beta else [])
    out = {}

    def sample(cs, sl):
        for k in keys:
            out[k][sl] = ev(k, cs)
        if var_beta:
            out["beta"][sl] = ev.expr(beta, cs)

    for k in keys + (["beta"] if var_beta else []):
        out[k] = _zeros(ev, shape)
    if dim == 3 and chunk is not None:
        for z0 in range(0, n[2] + 1, chunk):
            z1 = min(n[2] + 1, z0 + chunk)
            sample([ev.coords(c1d[0], 0), ev.coords(c1d[1], 1), ev.coords(c1d[2][z0:z1], 2)], slice(z0, z1))
    else:
        sample([ev.coords(c1d[a], a) for a in range(dim)], slice(None))
    if beta:
        bval = out.pop("beta") if var_beta else float(beta)
        out["f"] = out["f"] + bval * out.pop("lapu")
        beta = bval
    nav = tuple(bool(v) for v in navier) if any(navier) else ()
    if nav and len(nav) != 2 * dim:
        raise ValueError("navier needs one flag per face")
    bd = _boundary_data(ev, n, c1d, want_gl=bool(nav))
    gD, gN, lap = bd[:3]
    gL = bd[3] if nav else None
    return Problem(tuple(n), lo, hi, out["alpha"], out["f"], gD, gN, lap,
                   out.get("u"), out.get("v"), name=name,
                   meta={"alpha": alpha_src, "u": u_src, "params": dict(zip(params, pvals)),
                         "beta": beta_src if var_beta else float(beta), "navier": nav},
                   beta=beta if var_beta else float(beta), navier=nav, gL=gL)


# --------------------------------------------------------------------------------------
# the benchmark configurations (all fully clamped, beta = 0)
# --------------------------------------------------------------------------------------

def config1(n=32, **kw):
    """2-D, alpha = 1, u = sin^2(pi x) sin^2(pi y) on the unit square (Delta^2 u = f form)."""
    return manufactured("1", "sin(pi*x)**2*sin(pi*y)**2", (n, n), name=f"c1_n{n}", **kw)


def config2(n=256, **kw):
    """2-D variable coefficient alpha = 1 + 0.5 sin(2 pi x) cos(2 pi y), u = sin^2 sin^2 e^{x+y}."""
    return manufactured("1 + 0.5*sin(2*pi*x)*cos(2*pi*y)",
                        "sin(pi*x)**2*sin(pi*y)**2*exp(x + y)", (n, n), name=f"c2_n{n}", **kw)


C3_ALPHA = "1 + 0.5*sin(2*pi*x)*sin(2*pi*y)*sin(2*pi*z)"
C3_U = "sin(pi*x)**2*sin(pi*y)**2*sin(pi*z)**2"


def config3(n=128, **kw):
    """3-D unit cube, alpha = 1 + 0.5 sin sin sin (2 pi), u = sin^2 sin^2 sin^2 (pi)."""
    return manufactured(C3_ALPHA, C3_U, (n, n, n), name=f"c3_n{n}", **kw)


C4_SIZES = (64, 96, 128, 192, 256, 384, 512)
C4_ALPHA = "1 + c*sin(2*pi*p*x)*cos(2*pi*q*y)"
C4_U = "sin(pi*x)**2*sin(pi*y)**2*cos(k*(x + y))"


def config4_specs(count=512, seed=0):
    """Seeded draws for the batched 2-D workload.

    Per instance, in this order: n uniform over C4_SIZES, c ~ U(0, 0.8),
    p, q integers in [1, 4], k ~ U(10, 80)."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        n = int(rng.choice(C4_SIZES))
        c = float(rng.uniform(0.0, 0.8))
        p = int(rng.integers(1, 5))
        q = int(rng.integers(1, 5))
        k = float(rng.uniform(10.0, 80.0))
        specs.append({"n": n, "c": c, "p": p, "q": q, "k": k})
    return specs


def config4_instance(spec, **kw):
    return manufactured(C4_ALPHA, C4_U, (spec["n"], spec["n"]), params=("c", "p", "q", "k"),
                        pvals=(spec["c"], spec["p"], spec["q"], spec["k"]),
                        name=f"c4_n{spec['n']}", **kw)


EX1_U = "256*(x**2 + eps*(1 - exp(-x/sqrt(eps)))**2)*(x - 1)**2*y**2*(y - 1)**2"


def example1(n=256, eps=1e-4, **kw):
    """The 2-D singularly perturbed test of the paper's first convergence experiment:
    -eps Delta^2 u + Delta u = f (alpha = eps, beta = 1) on the unit square, clamped at
    x = 0 and Navier on the other faces, with the manufactured boundary-layer solution EX1_U."""
    return manufactured(repr(float(eps)), EX1_U.replace("eps", repr(float(eps))), (n, n), beta=1.0,
                        navier=(False, True, True, True), name=f"ex1_n{n}_eps{eps:g}", **kw)


EX2_U = "(x**2 - x)*(y**2 - y)*(z**2 - z)*exp(q*((x - 0.5)**2 + (y - 0.5)**2 + (z - p)**2))"
EX2_ALPHA = "x**2 + y**2 + z**2 + 1"
EX2_BETA = "x + y + z + 10"


def example2(n=32, q=10.0, p=0.2, alpha=EX2_ALPHA, beta=EX2_BETA, **kw):
    """The 3-D peaked test of the paper's second convergence experiment: alpha = x^2 + y^2 +
    z^2 + 1, beta = x + y + z + 10 (variable), clamped at x = 0 and Navier on the other faces,
    with the manufactured solution EX2_U (peak sharpness q, peak height p along z).  The
    paper's timing table uses the same solution for the classical biharmonic equation
    (alpha = "1", beta = 0)."""
    nn = tuple(n) if isinstance(n, (tuple, list)) else (n, n, n)
    return manufactured(alpha, EX2_U, nn, params=("q", "p"), pvals=(float(q), float(p)), beta=beta,
                        navier=(False, True, True, True, True, True), name=f"ex2_n{nn[0]}_q{q:g}_p{p:g}", **kw)


EX3_U = "sin(k1*x)*cos(k2*y)*sin(k3*z)"


def example3(n=32, k=(5.0, 1.0, 5.0), alpha=EX2_ALPHA, beta=EX2_BETA, **kw):
    """The 3-D oscillatory test of the paper (Table 3): u = sin(k1 x) cos(k2 y) sin(k3 z) with
    the coefficients of Example 2 (alpha = x^2 + y^2 + z^2 + 1, beta = x + y + z + 10), clamped
    at x = 0 and Navier on the other faces; all boundary data inhomogeneous.  The timing
    table uses it for the classical biharmonic equation (alpha = "1", beta = 0)."""
    nn = tuple(n) if isinstance(n, (tuple, list)) else (n, n, n)
    k = tuple(float(v) for v in k)
    return manufactured(alpha, EX3_U, nn, params=("k1", "k2", "k3"), pvals=k, beta=beta,
                        navier=(False, True, True, True, True, True),
                        name=f"ex3_n{nn[0]}_k{k[0]:g}_{k[1]:g}_{k[2]:g}", **kw)


def cavity(n=64):
    """Lid-driven cavity stream function: Delta^2 psi = 0, psi = 0, psi_n = 1 on y = 1."""
    dim = 2
    shape = (n + 1, n + 1)
    gN = np.zeros(shape)
    gN[n, 1:n] = 1.0  # y = 1 face interior; outward normal is +y, [-u_y, u_x] = [-1, 0]
    return Problem((n, n), (0.0, 0.0), (1.0, 1.0), np.ones(shape), np.zeros(shape),
                   None, gN, None, name=f"cavity_n{n}")


def plate(n=64):
    """Clamped unit plate under a unit central load (load reading: trapezoid weights on even n).

    The paper's load 1/(4h^2) on |x-1/2| <= h, |y-1/2| <= h covers 9 nodes on an
    even grid; we weight them by the tensor trapezoid rule (1, 1/2, 1/4) so that
    the load integrates to one.  On odd n the literal 4-node reading is used.
    Sign: the paper's form -Delta(alpha Delta u) = f with Delta^2 u = load gives
    f = -load.
    """
    h = 1.0 / n
    x = np.arange(n + 1) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    load = np.zeros((n + 1, n + 1))
    mask = (np.abs(X - 0.5) <= h + 1e-12) & (np.abs(Y - 0.5) <= h + 1e-12)
    if n % 2 == 0:
        w1 = np.where(np.abs(x - 0.5) < 1e-12, 1.0, 0.5)
        W = np.outer(w1, w1)
        load[mask] = W[mask] / (4 * h * h)
    else:
        load[mask] = 1.0 / (4 * h * h)
    return Problem((n, n), (0.0, 0.0), (1.0, 1.0), np.ones((n + 1, n + 1)), -load,
                   name=f"plate_n{n}")


def high_wavenumber(n, dim=2, k=50.0, sigma=0.02, xp="numpy", device=None):
    """The high-wavenumber test of Sec. 4.2: -Delta^2 u - k^2 Delta u = (1e5 / (pi sigma^2))
    exp(-|x - 1/2|^2 / sigma^2) on the unit box with homogeneous clamped conditions, i.e.
    alpha = 1, beta = -k^2 in -Delta(alpha Delta u) + beta Delta u = f.  No closed-form
    solution: errors are measured against a finer grid."""
    n = tuple(n) if isinstance(n, (tuple, list)) else (int(n),) * dim
    dim = len(n)
    c1d = node_coords(n, (0.0,) * dim, (1.0,) * dim)
    shape = tuple(m + 1 for m in reversed(n))
    if xp == "torch":
        import torch
        r2 = torch.zeros(shape, dtype=torch.float64, device=device)
        for a in range(dim):
            ax = torch.as_tensor(c1d[a], dtype=torch.float64, device=device)
            sh = [1] * dim
            sh[dim - 1 - a] = n[a] + 1
            r2 = r2 + ((ax - 0.5) ** 2).reshape(sh)
        f = 1e5 / (np.pi * sigma ** 2) * torch.exp(-r2 / sigma ** 2)
        alpha = torch.ones(shape, dtype=torch.float64, device=device)
    else:
        r2 = np.zeros(shape)
        for a in range(dim):
            sh = [1] * dim
            sh[dim - 1 - a] = n[a] + 1
            r2 = r2 + ((c1d[a] - 0.5) ** 2).reshape(sh)
        f = 1e5 / (np.pi * sigma ** 2) * np.exp(-r2 / sigma ** 2)
        alpha = np.ones(shape)
    return Problem(n, (0.0,) * dim, (1.0,) * dim, alpha, f, beta=-float(k) ** 2,
                   name=f"hwp{dim}d_n{n[0]}_k{k:g}", meta={"k": float(k), "sigma": float(sigma)})


def poly_exact(n, dim=2, **kw):
    """Polynomial-exactness problem: u of total degree 4, alpha of degree 3, all data nonzero.

    For such data v = alpha Delta u has degree <= 5, so the compact scheme
    reproduces u at every node to rounding (the operators are exact for
    polynomials of degree <= 5 and the one-sided normal formula for degree <= 4).
    """
    if dim == 2:
        u = "1 + x - 2*y + x*y + 0.5*x**2*y**2 - 0.3*x**3*y + 0.2*x**4 + 0.1*y**4 - 0.7*x**2 + 0.4*y**3"
        a = "2 + 0.3*x + 0.2*y + 0.1*x*y + 0.05*x**3"
        lo, hi = (-0.3, 0.1), (0.9, 1.4)
    else:
        u = ("1 + x - 2*y + 0.5*z + x*y*z + 0.5*x**2*y**2 - 0.3*x**3*z + 0.2*x**4"
             " + 0.1*y**4 - 0.7*z**2*x + 0.4*y**3 + 0.25*z**4 - 0.2*y*z**3")
        a = "2 + 0.3*x + 0.2*y - 0.1*z + 0.1*x*y*z + 0.05*z**3"
        lo, hi = (-0.3, 0.1, 0.2), (0.9, 1.4, 1.1)
    return manufactured(a, u, n if isinstance(n, (tuple, list)) else (n,) * dim, lo, hi,
                        name=f"poly{dim}d", **kw)


# --------------------------------------------------------------------------------------
# the triharmonic extension (Sec. 4.2): Delta^3 u = f
# --------------------------------------------------------------------------------------

@dataclass
class TriProblem:
    """One triharmonic problem Delta^3 u = f on a box (Sec. 4.2, "Triharmonic equation").

    Clamped faces carry u = g_D, u_n = g_N, u_nn = g_NN; Navier faces (navier[f]) u = g_D,
    Delta u and Delta^2 u.  Nodal arrays (memory order z, y, x), None = identically zero:
      f      the right-hand side Delta^3 u
      gD     u on boundary nodes
      gN     outward normal derivative on face-interior nodes of clamped faces
      gNN    second normal derivative on face-interior nodes of clamped faces
      lapu   Delta u on every boundary node (the boundary values of v = Delta u, which the
             data fix on every face: u_nn plus the tangential Laplacian of g_D on a clamped
             face, given on a Navier face)
      bilap  Delta^2 u on boundary nodes (read on Navier faces, edges and corners, where w =
             Delta v is known)
      tang4  on face-interior nodes of clamped faces, Delta^2 u minus its pure normal part
             u_nnnn (what the Dirichlet data and g_NN fix: 2 Delta_tau u_nn + Delta_tau^2 u)
    """
    n: tuple
    lo: tuple
    hi: tuple
    f: Any
    gD: Any = None
    gN: Any = None
    gNN: Any = None
    lapu: Any = None
    bilap: Any = None
    tang4: Any = None
    u_exact: Any = None
    name: str = ""
    navier: tuple = ()
    meta: dict = field(default_factory=dict)

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def h(self) -> tuple:
        return tuple((b - a) / m for a, b, m in zip(self.lo, self.hi, self.n))


@functools.lru_cache(maxsize=None)
def _derive_tri(u_src: str, dim: int, params: tuple = ()):
    import sympy as sp
    X = _symbols(dim)
    ns = {s.name: s for s in X}
    ns.update({p: sp.Symbol(p) for p in params})
    ns.update({"pi": sp.pi, "sin": sp.sin, "cos": sp.cos, "exp": sp.exp, "sqrt": sp.sqrt})
    u = sp.sympify(u_src, locals=ns)
    lap = lambda w: sum(sp.diff(w, s, 2) for s in X)
    v = lap(u)
    w = lap(v)
    ex = {"u": u, "v": v, "w": w, "f": lap(w)}
    for a in range(dim):
        ex[f"d1u{a}"] = sp.diff(u, X[a])
        ex[f"d2u{a}"] = sp.diff(u, X[a], 2)
        ex[f"d4u{a}"] = sp.diff(u, X[a], 4)
    return X, tuple(sp.Symbol(p) for p in params), ex


def triharmonic(u_src: str, n: Sequence[int], lo=None, hi=None, *, params=(), pvals=(), navier=(),
                xp="numpy", device=None, chunk=None, name=""):
    """Sample a manufactured triharmonic problem: f = Delta^3 u and the boundary data of
    TriProblem from the expression u_src (in x, y[, z] and `params`)."""
    dim = len(n)
    lo = tuple(lo) if lo is not None else (0.0,) * dim
    hi = tuple(hi) if hi is not None else (1.0,) * dim
    X, P, ex = _derive_tri(u_src, dim, tuple(params))
    fns = {k: _lambdify(e, X, P, xp) for k, e in ex.items()}
    ev = _Eval("1", u_src, dim, params, pvals, xp, device)
    c1d = node_coords(n, lo, hi)
    shape = tuple(n[a] + 1 for a in reversed(range(dim)))

    def at(key, cs):
        out = fns[key](*cs, *pvals)
        if xp == "torch":
            import torch
            shp = tuple(torch.broadcast_shapes(*[tuple(c.shape) for c in cs]))
        else:
            shp = np.broadcast_shapes(*[c.shape for c in cs])
        return ev._full(out, shp)

    f = _zeros(ev, shape)
    ue = _zeros(ev, shape)
    if dim == 3 and chunk is not None:
        for z0 in range(0, n[2] + 1, chunk):
            z1 = min(n[2] + 1, z0 + chunk)
            cs = [ev.coords(c1d[0], 0), ev.coords(c1d[1], 1), ev.coords(c1d[2][z0:z1], 2)]
            f[z0:z1] = at("f", cs)
            ue[z0:z1] = at("u", cs)
    else:
        cs = [ev.coords(c1d[a], a) for a in range(dim)]
        f[...] = at("f", cs)
        ue[...] = at("u", cs)
    nav = tuple(bool(v) for v in navier) if any(navier) else (False,) * (2 * dim)
    if len(nav) != 2 * dim:
        raise ValueError("navier needs one flag per face")
    gD, gN, gNN, lapu, bilap, tang4 = (_zeros(ev, shape) for _ in range(6))

    def sl(axis, idx):
        s_ = [slice(None)] * dim
        s_[dim - 1 - axis] = slice(idx, idx + 1)
        return tuple(s_)

    for a in range(dim):
        for side, idx in ((0, 0), (1, n[a])):
            cs = [ev.coords(c1d[b], b) if b != a else ev.coords(c1d[a][idx:idx + 1], a) for b in range(dim)]
            tgt = sl(a, idx)
            gD[tgt] = at("u", cs)
            lapu[tgt] = at("v", cs)
            bilap[tgt] = at("w", cs)
            if nav[2 * a + side]:
                continue
            inner = [slice(None)] * dim
            for b in range(dim):
                if b != a:
                    inner[dim - 1 - b] = slice(1, n[b])
            inner = tuple(inner)
            du = at(f"d1u{a}", cs)
            vals = {"gN": -du if side == 0 else du, "gNN": at(f"d2u{a}", cs),
                    "tang4": at("w", cs) - at(f"d4u{a}", cs)}
            for key, arr in (("gN", gN), ("gNN", gNN), ("tang4", tang4)):
                sub = arr[tgt]
                sub[inner] = vals[key][inner]
                arr[tgt] = sub
    out = []
    for arr in (gD, gN, gNN, lapu, bilap, tang4):
        mx = float(arr.abs().max()) if xp == "torch" else float(np.abs(arr).max())
        out.append(None if mx < 1e-12 else arr)
    return TriProblem(tuple(n), lo, hi, f, *out, u_exact=ue, name=name or f"tri{dim}d",
                      navier=nav, meta={"u": u_src, "params": dict(zip(params, pvals))})


EX3_TRI_U = "sin(k1*x)*cos(k2*y)*sin(k3*z)"


def example3_tri(n=32, k=(5.0, 1.0, 5.0), **kw):
    """The triharmonic test of Sec. 4.2 (Table 5): the solution of the 3-D oscillatory example,
    u = sin(k1 x) cos(k2 y) sin(k3 z), on the unit cube, clamped at x = 0 and Navier on the
    other faces (the boundary setting of the paper's convergence tests)."""
    nn = tuple(n) if isinstance(n, (tuple, list)) else (n, n, n)
    k = tuple(float(v) for v in k)
    return triharmonic(EX3_TRI_U, nn, params=("k1", "k2", "k3"), pvals=k,
                       navier=(False, True, True, True, True, True),
                       name=f"tri_ex3_n{nn[0]}_k{k[0]:g}_{k[1]:g}_{k[2]:g}", **kw)
