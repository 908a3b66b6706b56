"""Python binding of libahoc (the MI355X augmented HOC biharmonic solver).

Argument marshalling only: every step of the solver runs in the HIP library
behind the C ABI declared in include/ahoc.h.  PyTorch provides device memory
and the current stream.  Importing this package on a machine without the
built library raises ImportError -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libahoc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "(hipcc --offload-arch=gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

OK, E_INVALID, E_NOMEM, E_NOCONV, E_HIP, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
FP64, MIXED = 0, 1
BIHARMONIC, TRIHARMONIC = 0, 1

c_int, c_double, c_void_p, c_size_t = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t


class _Problem(ctypes.Structure):
    _fields_ = [("dim", c_int), ("n", c_int * 3), ("lo", c_double * 3), ("hi", c_double * 3),
                ("alpha", c_void_p), ("f", c_void_p), ("gD", c_void_p), ("gN", c_void_p),
                ("lapgD", c_void_p), ("beta", c_double), ("navier", c_int), ("gL", c_void_p),
                ("beta_nodal", c_void_p), ("equation", c_int), ("gNN", c_void_p), ("lapu", c_void_p),
                ("bilap", c_void_p), ("tang4", c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("precision", c_int), ("restart", c_int), ("max_iters", c_int), ("tol", c_double),
                ("inner_tol", c_double), ("sweep_tol", c_double), ("max_sweeps", c_int),
                ("tile_fp64", c_int), ("tile_fp32", c_int), ("precond", c_int),
                ("refine", c_int), ("use_graph", c_int), ("warm_start", c_int), ("vsolve_max_iters", c_int)]


class _Stats(ctypes.Structure):
    _fields_ = [("converged", c_int), ("gmres_iters", c_int), ("sweeps", c_int), ("matvecs", c_int),
                ("schur_relres", c_double), ("last_update", c_double), ("t_solve_ms", c_double),
                ("graph_steps", c_int), ("dst_gemm", c_int), ("vsolve_iters", c_int),
                ("vsolve_relres", c_double)]


_ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, c_size_t, c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", c_void_p)]


def _torch_alloc(nbytes, ctx):
    """ahoc_allocator.alloc backed by PyTorch's caching allocator; ctx = device index + 1.
    Returns NULL (-> AHOC_E_NOMEM) instead of raising."""
    try:
        torch = _torch()
        dev = int(ctx or 1) - 1
        return torch.cuda.caching_allocator_alloc(int(nbytes), device=dev)
    except Exception:  # out of memory or no device: the library reports AHOC_E_NOMEM
        return None


def _torch_free(ptr, ctx):
    try:
        if ptr:
            _torch().cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


# the callbacks live as long as the module (handles keep the function pointers)
_TORCH_ALLOC = _ALLOC_FN(_torch_alloc)
_TORCH_FREE = _FREE_FN(_torch_free)


def torch_allocator(device=0):
    """An ahoc_allocator that takes device memory from PyTorch's caching allocator."""
    return _Allocator(_TORCH_ALLOC, _TORCH_FREE, c_void_p(int(device) + 1))


_H = c_void_p
_lib.ahoc_default_options.argtypes = [ctypes.POINTER(_Options)]
_lib.ahoc_setup.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(_Options), ctypes.POINTER(_Allocator), c_void_p,
                            ctypes.POINTER(_H)]
_lib.ahoc_setup.restype = c_int
_lib.ahoc_nq.argtypes = [_H]
_lib.ahoc_nq.restype = c_size_t
_lib.ahoc_schur_apply.argtypes = [_H, c_void_p, c_void_p, c_void_p]
_lib.ahoc_schur_apply.restype = c_int
_lib.ahoc_precond_apply.argtypes = [_H, c_void_p, c_void_p, c_void_p]
_lib.ahoc_precond_apply.restype = c_int
_lib.ahoc_schur_rhs.argtypes = [_H, c_void_p, c_void_p]
_lib.ahoc_schur_rhs.restype = c_int
_lib.ahoc_solve.argtypes = [_H, c_void_p, c_void_p, c_void_p, ctypes.POINTER(_Stats), c_void_p]
_lib.ahoc_solve.restype = c_int
_lib.ahoc_solve_batched.argtypes = [c_int, ctypes.POINTER(_Problem), ctypes.POINTER(_Options),
                                    ctypes.POINTER(_Allocator), ctypes.POINTER(c_void_p), ctypes.POINTER(_Stats),
                                    c_void_p]
_lib.ahoc_solve_batched.restype = c_int
_lib.ahoc_poisson.argtypes = [_H, c_void_p, c_void_p, c_void_p]
_lib.ahoc_poisson.restype = c_int
_lib.ahoc_poisson_noalloc.argtypes = [c_int, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_double),
                                      ctypes.POINTER(c_double), c_void_p, c_void_p, c_void_p]
_lib.ahoc_poisson_noalloc.restype = c_int
_lib.ahoc_dst1.argtypes = [c_int, c_int, ctypes.POINTER(c_int), c_int, c_void_p, c_void_p, c_void_p]
_lib.ahoc_dst1.restype = c_int
_lib.ahoc_profile.argtypes = [_H, c_int]
_lib.ahoc_profile.restype = c_int
_lib.ahoc_kernel_times.argtypes = [_H, c_int, ctypes.POINTER(c_double), ctypes.POINTER(ctypes.c_longlong),
                                   ctypes.POINTER(c_double)]
_lib.ahoc_kernel_times.restype = c_int
_lib.ahoc_set_dst_variant.argtypes = [c_int]
_lib.ahoc_set_dst_variant.restype = c_int
_lib.ahoc_set_dst_tile.argtypes = [c_int, c_int, c_int]
_lib.ahoc_set_dst_tile.restype = c_int
_lib.ahoc_dst_choice.argtypes = [_H, c_int, c_int, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                                 ctypes.POINTER(c_double), ctypes.POINTER(c_double), ctypes.POINTER(c_double)]
_lib.ahoc_dst_choice.restype = c_int
_lib.ahoc_copy_bandwidth.argtypes = [c_int, c_void_p, c_void_p, c_int, c_int, c_int, c_void_p]
_lib.ahoc_copy_bandwidth.restype = c_int
_lib.ahoc_destroy.argtypes = [_H]
_lib.ahoc_status_string.argtypes = [c_int]
_lib.ahoc_status_string.restype = ctypes.c_char_p
_lib.ahoc_last_error.restype = ctypes.c_char_p

KERNEL_KINDS = ["dst_rows", "dst_strided", "dst_fused", "lift", "rhs_u", "gather", "krylov", "resid",
                "matvec", "dst_gen", "face_reduce", "precond", "vsolve", "dst_xmul"]

EXPORTED = ["ahoc_set_dst_variant", "ahoc_set_dst_tile", "ahoc_dst_choice", "ahoc_copy_bandwidth", "ahoc_profile", "ahoc_kernel_times", "ahoc_default_options", "ahoc_setup", "ahoc_nq", "ahoc_schur_apply", "ahoc_precond_apply", "ahoc_schur_rhs",
            "ahoc_solve", "ahoc_solve_batched", "ahoc_poisson", "ahoc_poisson_noalloc", "ahoc_dst1", "ahoc_destroy",
            "ahoc_status_string", "ahoc_last_error"]


class AhocError(RuntimeError):
    def __init__(self, code, where=""):
        msg = _lib.ahoc_status_string(code).decode()
        last = (_lib.ahoc_last_error() or b"").decode()
        super().__init__(f"{where}: {msg} ({code}) {last}")
        self.code = code


def _check(code, where):
    if code != OK:
        raise AhocError(code, where)


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(x, device):
    """A contiguous float64 tensor on `device` (numpy or torch input); None stays None."""
    if x is None:
        return None
    torch = _torch()
    if isinstance(x, np.ndarray):
        return torch.from_numpy(np.array(x, dtype=np.float64, order="C", copy=True)).to(device)
    return x.to(device=device, dtype=torch.float64).contiguous()


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def default_options(precision=FP64, **kw) -> _Options:
    o = _Options()
    _lib.ahoc_default_options(ctypes.byref(o))
    o.precision = precision
    for k, v in kw.items():
        if v is not None:
            setattr(o, k, v)
    return o


@dataclass
class Stats:
    converged: bool
    gmres_iters: int
    sweeps: int
    matvecs: int
    schur_relres: float
    last_update: float
    t_solve_ms: float
    graph_steps: int = 0
    dst_gemm: int = 0
    vsolve_iters: int = 0
    vsolve_relres: float = 0.0


def _stats(s: _Stats) -> Stats:
    return Stats(bool(s.converged), s.gmres_iters, s.sweeps, s.matvecs, s.schur_relres,
                 s.last_update, s.t_solve_ms, s.graph_steps, s.dst_gemm, s.vsolve_iters,
                 s.vsolve_relres)


def _allocator_arg(allocator, device):
    """'torch' (default): PyTorch's caching allocator; None: the library's hipMalloc;
    or an _Allocator."""
    if allocator is None:
        return None
    if isinstance(allocator, str):
        if allocator != "torch":
            raise ValueError(f"unknown allocator {allocator!r}")
        idx = device.index if getattr(device, "index", None) is not None else 0
        return ctypes.byref(torch_allocator(idx))
    return ctypes.byref(allocator)


_FIELDS = ("alpha", "f", "gD", "gN", "lapgD", "gL")
_TRI_FIELDS = ("gNN", "lapu", "bilap", "tang4")


def _equation(problem) -> int:
    """TRIHARMONIC for a workloads.TriProblem-like object (it carries bilap), else BIHARMONIC."""
    return TRIHARMONIC if hasattr(problem, "bilap") else BIHARMONIC


def _navier_mask(navier) -> int:
    """Per-face flags (x-, x+, y-, y+[, z-, z+]) or an int bitmask -> bitmask."""
    if isinstance(navier, int):
        return navier
    return sum(1 << f for f, v in enumerate(navier or ()) if v)


def _problem_tensors(problem, device):
    """Device tensors of the nodal fields (_FIELDS, a variable beta or None, then _TRI_FIELDS)
    and the constant beta (0 when beta is nodal)."""
    beta = getattr(problem, "beta", 0.0)
    scalar = beta is None or np.isscalar(beta) or (hasattr(beta, "ndim") and beta.ndim == 0)
    tens = [_dev(getattr(problem, k, None), device) for k in _FIELDS]
    tens.append(None if scalar else _dev(beta, device))
    tens += [_dev(getattr(problem, k, None), device) for k in _TRI_FIELDS]
    return tens, (float(beta or 0.0) if scalar else 0.0)


def _problem_struct(n, lo, hi, tens, beta=0.0, navier=(), equation=BIHARMONIC):
    dim = len(n)
    p = _Problem()
    p.dim = dim
    p.beta = float(beta or 0.0)
    p.navier = _navier_mask(navier)
    p.equation = int(equation)
    for a in range(3):
        p.n[a] = int(n[a]) if a < dim else 0
        p.lo[a] = float(lo[a]) if a < dim else 0.0
        p.hi[a] = float(hi[a]) if a < dim else 0.0
    (p.alpha, p.f, p.gD, p.gN, p.lapgD, p.gL, p.beta_nodal,
     p.gNN, p.lapu, p.bilap, p.tang4) = [(t.data_ptr() if t is not None else None) for t in tens]
    return p


class Solver:
    """One problem set up on the GPU (wraps an ahoc_handle).

    `problem` carries n, lo, hi, nodal alpha, f, gD, gN, lapgD (numpy or torch, memory
    order z, y, x) and optionally beta (a constant, or a nodal array: FP64 only) and Navier
    faces (navier: per-face flags or a bitmask, gL: nodal Delta u read on them), e.g. a
    workloads.Problem; or, for the triharmonic equation Delta^3 u = f, f, gD, gN, gNN, lapu,
    bilap, tang4 and navier (a workloads.TriProblem).

    allocator: "torch" (default) takes the handle's device memory from PyTorch's caching
    allocator (ahoc_allocator callbacks); None lets the library call hipMalloc.
    """

    def __init__(self, problem, precision=FP64, device="cuda:0", allocator="torch", **opts):
        torch = _torch()
        self.device = torch.device(device)
        self.n = tuple(problem.n)
        self.dim = len(self.n)
        tens, beta = _problem_tensors(problem, self.device)
        self._p = _problem_struct(self.n, problem.lo, problem.hi, tens, beta, getattr(problem, "navier", ()),
                                  _equation(problem))
        self.options = default_options(precision, **opts)
        h = _H()
        with torch.cuda.device(self.device):
            _check(_lib.ahoc_setup(ctypes.byref(self._p), ctypes.byref(self.options),
                                   _allocator_arg(allocator, self.device), _stream(), ctypes.byref(h)),
                   "ahoc_setup")
        self._h = h
        self.nq = int(_lib.ahoc_nq(h))
        self.nodal_shape = tuple(m + 1 for m in reversed(self.n))
        self.interior_shape = tuple(m - 1 for m in reversed(self.n))

    def close(self):
        if getattr(self, "_h", None):
            _lib.ahoc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _vec(self, x, size):
        t = _dev(x, self.device)
        assert t.numel() == size
        return t

    def schur_apply(self, q):
        torch = _torch()
        q = self._vec(q, self.nq)
        y = torch.empty(self.nq, dtype=torch.float64, device=self.device)
        _check(_lib.ahoc_schur_apply(self._h, _ptr(q), _ptr(y), _stream()), "ahoc_schur_apply")
        return y

    def precond_apply(self, q):
        """y = P^-1 q with the handle's boundary-symbol preconditioner."""
        torch = _torch()
        q = self._vec(q, self.nq)
        y = torch.empty(self.nq, dtype=torch.float64, device=self.device)
        _check(_lib.ahoc_precond_apply(self._h, _ptr(q), _ptr(y), _stream()), "ahoc_precond_apply")
        return y

    def dst_choice(self, precision, axis, kind):
        """Setup-time kernel choice for the plain DST passes of one axis (kind 0 contiguous,
        1 strided): (method, tile, t_default_us, t_gemm_us, t_best_us); method 0 default FFT
        kernel, 1 matrix-core pass, 2 one-tile FFT kernel with `tile` pairs, -1 not timed."""
        m, t = c_int(0), c_int(0)
        td, tg, tb = c_double(0.0), c_double(0.0), c_double(0.0)
        _check(_lib.ahoc_dst_choice(self._h, int(precision), int(axis), int(kind), ctypes.byref(m), ctypes.byref(t),
                                    ctypes.byref(td), ctypes.byref(tg), ctypes.byref(tb)), "ahoc_dst_choice")
        return m.value, t.value, td.value, tg.value, tb.value

    def schur_rhs(self):
        torch = _torch()
        b = torch.empty(self.nq, dtype=torch.float64, device=self.device)
        _check(_lib.ahoc_schur_rhs(self._h, _ptr(b), _stream()), "ahoc_schur_rhs")
        return b

    def poisson(self, g):
        torch = _torch()
        g = _dev(g, self.device).reshape(-1)
        w = torch.empty_like(g)
        _check(_lib.ahoc_poisson(self._h, _ptr(g), _ptr(w), _stream()), "ahoc_poisson")
        return w.reshape(self.interior_shape)

    def profile(self, enable=True):
        """Per-kernel-class HIP-event timing of subsequent solves (resets the totals)."""
        _check(_lib.ahoc_profile(self._h, 1 if enable else 0), "ahoc_profile")

    def kernel_times(self):
        """{kind: (total_ms, launches, algorithmic bytes per launch)} since profile()."""
        out = {}
        for k, name in enumerate(KERNEL_KINDS):
            ms, cnt, by = c_double(), ctypes.c_longlong(), c_double()
            _check(_lib.ahoc_kernel_times(self._h, k, ctypes.byref(ms), ctypes.byref(cnt),
                                          ctypes.byref(by)), "ahoc_kernel_times")
            out[name] = (ms.value, cnt.value, by.value)
        return out

    def solve(self, want_v=False, want_q=False, out=None, q0=None):
        """Solve; q0 (length N_q) is the GMRES initial guess -- the handle must have been
        set up with warm_start=1.  Returns (u, v or None, q or None, Stats); q is returned
        when want_q or q0 is given."""
        torch = _torch()
        u = out if out is not None else torch.empty(self.nodal_shape, dtype=torch.float64,
                                                    device=self.device)
        v = torch.empty(self.nodal_shape, dtype=torch.float64, device=self.device) if want_v else None
        if q0 is not None:
            if not self.options.warm_start:
                raise ValueError("q0 needs a handle set up with warm_start=1")
            q = self._vec(q0, self.nq).clone()
        else:
            q = torch.empty(self.nq, dtype=torch.float64, device=self.device) if want_q else None
        s = _Stats()
        rc = _lib.ahoc_solve(self._h, _ptr(u), _ptr(v), _ptr(q), ctypes.byref(s), _stream())
        if rc not in (OK, E_NOCONV):
            _check(rc, "ahoc_solve")
        self.status = rc  # OK or E_NOCONV (outputs hold the last iterate)
        return u, v, q, _stats(s)


def solve_batched(problems: Sequence, precision=FP64, device="cuda:0", allocator="torch", **opts):
    """Solve independent problems with shared options; returns (list of u, list of Stats, status).

    An instance that is rejected (E_INVALID, E_UNSUPPORTED) or does not converge does not
    stop the others: the call returns the first such status and that instance's Stats say
    converged=False; device or memory failures raise AhocError."""
    torch = _torch()
    dev = torch.device(device)
    keep, structs, outs = [], [], []
    for pb in problems:
        tens, beta = _problem_tensors(pb, dev)
        keep.append(tens)
        structs.append(_problem_struct(pb.n, pb.lo, pb.hi, tens, beta, getattr(pb, "navier", ()), _equation(pb)))
        outs.append(torch.empty(tuple(m + 1 for m in reversed(pb.n)), dtype=torch.float64, device=dev))
    cnt = len(problems)
    parr = (_Problem * cnt)(*structs)
    uarr = (c_void_p * cnt)(*[o.data_ptr() for o in outs])
    sarr = (_Stats * cnt)()
    o = default_options(precision, **opts)
    rc = _lib.ahoc_solve_batched(cnt, parr, ctypes.byref(o), _allocator_arg(allocator, dev), uarr, sarr, _stream())
    if rc not in (OK, E_NOCONV, E_INVALID, E_UNSUPPORTED):
        _check(rc, "ahoc_solve_batched")
    return outs, [_stats(s) for s in sarr], rc


def set_dst_variant(variant: int):
    """0 = automatic (plain passes of an operator use the kernel its setup timed fastest), 1 = generic DST kernel
    everywhere, 2 = length-specialised kernels only, 3 = one-tile strided kernels, 4 = matrix-core
    products for every plain pass of even N <= 128, 5 = automatic without setup-time choices."""
    _check(_lib.ahoc_set_dst_variant(int(variant)), "ahoc_set_dst_variant")


def set_dst_tile(pass_kind: int, precision: int, pairs: int):
    """Default work-group tile (pencil pairs) of one DST pass kind: 0 rows, 1 strided, 2 fused;
    pairs = 0 restores the built-in choice."""
    _check(_lib.ahoc_set_dst_tile(int(pass_kind), int(precision), int(pairs)), "ahoc_set_dst_tile")


def copy_bandwidth(pattern, x, out):
    """Calibration copy out <- x of a float32 [nz][ny][nx] tensor (nx % 32 == 0): pattern 0
    linear, 1 the strided DST passes' tiles along y, 2 along z (asynchronous, current stream)."""
    assert x.dtype == out.dtype and x.dim() == 3 and x.is_contiguous() and out.is_contiguous()
    nz, ny, nx = x.shape
    _check(_lib.ahoc_copy_bandwidth(int(pattern), _ptr(x), _ptr(out), nx, ny, nz, _stream()), "ahoc_copy_bandwidth")


def poisson_noalloc(n, lo, hi, g, precision=FP64, out=None):
    """w = L_int^{-1} g on the interior of a box grid (homogeneous Dirichlet) through
    ahoc_poisson_noalloc: no handle, and the library allocates nothing (its work array and
    tables live in a fixed per-GPU device array).  g: interior-shaped float64 tensor on the
    device (memory order z, y, x); out: optional preallocated result of the same shape."""
    torch = _torch()
    dim = len(n)
    g = g.to(dtype=torch.float64).contiguous()
    w = out if out is not None else torch.empty_like(g)
    assert w.shape == g.shape and w.dtype == torch.float64 and w.is_contiguous()
    na = (c_int * 3)(*([int(v) for v in n] + [0] * (3 - dim)))
    lo_ = (c_double * 3)(*([float(v) for v in lo] + [0.0] * (3 - dim)))
    hi_ = (c_double * 3)(*([float(v) for v in hi] + [0.0] * (3 - dim)))
    _check(_lib.ahoc_poisson_noalloc(int(precision), dim, na, lo_, hi_, _ptr(g), _ptr(w), _stream()),
           "ahoc_poisson_noalloc")
    return w


def dst1(x, axis, precision=FP64):
    """Batched DST-I along `axis` (axis order x, y[, z]) of an interior-shaped tensor (memory order)."""
    torch = _torch()
    dim = x.dim()
    nint = (c_int * 3)(*([x.shape[dim - 1 - a] for a in range(dim)] + [1] * (3 - dim)))
    dt = torch.float64 if precision == FP64 else torch.float32
    xin = x.to(dtype=dt).contiguous()
    out = torch.empty_like(xin)
    _check(_lib.ahoc_dst1(precision, dim, nint, axis, _ptr(xin), _ptr(out), _stream()), "ahoc_dst1")
    return out
