"""MI355X geometric-multigrid solver for periodic Poisson and moving-mesh
(variable-coefficient) problems.

Thin PyTorch binding of the C ABI in ``include/mg.h``: torch supplies device
memory and the stream; every step of the solver runs in the HIP kernels of
``libmg.so``.  Nothing here falls back to a CPU implementation: if the library
is missing or no GPU is present, the calls raise.

Paper: "Fast(er)PM and Moving Mesh: JAX-native Geometric Multigrid Methods"
(Sec. 2.3 V-cycle, Sec. 3 warm-started defect correction, Sec. 4.3 curvilinear
operator, Sec. 4.8 implicit adjoint).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

from . import _lib
from ._lib import MGError

__all__ = ["Multigrid", "SolveInfo", "geometry", "geometry_bwd", "geometry_fn", "solve", "solve_fn",
           "predict", "accel", "MGError"]

_PRECISION = {"fp64": _lib.MG_FP64, "mixed": _lib.MG_MIXED, "fp32": _lib.MG_FP32}
_SMOOTHER = {"chebyshev": _lib.MG_CHEBYSHEV, "jacobi": _lib.MG_JACOBI}
_PREDICTOR = {"recycle": _lib.MG_PREDICT_RECYCLE, "growth": _lib.MG_PREDICT_GROWTH,
              "linear": _lib.MG_PREDICT_LINEAR, "quadratic": _lib.MG_PREDICT_QUADRATIC}


def _torch():
    import torch

    return torch


def _stream_ptr():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _check_field(t, n, dtype, name, comps=1):
    torch = _torch()
    shape = (n, n, n) if comps == 1 else (comps, n, n, n)
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if tuple(t.shape) != shape:
        raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


@dataclass
class SolveInfo:
    cycles: int
    rel_res0: float
    rel_res: float
    history: List[float] = field(default_factory=list)
    status: int = 0

    @property
    def converged(self) -> bool:
        return self.status == _lib.MG_OK


class Multigrid:
    """Solver context for an ``n^3`` periodic grid.

    ``coeff`` (optional) is a ``(6, n, n, n)`` float32/float64 GPU tensor of the
    symmetric coefficient ``C`` in order (xx, yy, zz, xy, xz, yz); it is copied.
    ``psi`` (optional, instead of ``coeff``) is an ``(n, n, n)`` float64 GPU
    deformation potential: every level is then rediscretised from the
    potential restricted to it (``mg_create_psi``).
    ``precision``: "fp64", "mixed" (float V-cycle, double residual/update/coarsest
    solve) or "fp32".  ``levels`` defaults to ``log2(n) - 1`` (coarsest 4^3).
    ``options`` is the ``mg_params.options`` mask of reference switches
    (``MG_OPT_*``; 0 runs every fused kernel).
    """

    def __init__(self, n: int, levels: Optional[int] = None, degree: int = 3, coeff=None,
                 precision: str = "mixed", h: Optional[float] = None, alpha: float = 8.0,
                 smoother: str = "chebyshev", omega: float = 2.0 / 3.0, sweeps: int = 2, psi=None,
                 options: int = 0):
        torch = _torch()
        lib = _lib.load()
        p = _lib.MgParams()
        lib.mg_params_default(ctypes.byref(p), int(n))
        if levels is not None:
            p.levels = int(levels)
        p.cheb_degree = int(degree)
        p.cheb_alpha = float(alpha)
        if h is not None:
            p.h = float(h)
        p.precision = _PRECISION[precision]
        p.smoother = _SMOOTHER[smoother]
        p.jacobi_omega = float(omega)
        p.jacobi_sweeps = int(sweeps)
        p.options = int(options)
        self.n = int(n)
        self.params = p
        self.precision = precision
        self.levels = p.levels
        self.h = p.h
        self.var = coeff is not None or psi is not None
        if coeff is not None and psi is not None:
            raise ValueError("give coeff or psi, not both")
        cptr, cdt = None, _lib.MG_DTYPE_F64
        if coeff is not None:
            if coeff.dtype not in (torch.float32, torch.float64):
                raise ValueError("coeff must be float32 or float64")
            _check_field(coeff, self.n, coeff.dtype, "coeff", comps=6)
            cptr = _ptr(coeff)
            cdt = _lib.MG_DTYPE_F64 if coeff.dtype == torch.float64 else _lib.MG_DTYPE_F32
        h_ctx = ctypes.c_void_p()
        if psi is not None:
            _check_field(psi, self.n, torch.float64, "psi")
            st = lib.mg_create_psi(ctypes.byref(p), _ptr(psi), _stream_ptr(), ctypes.byref(h_ctx))
            if st != _lib.MG_OK:
                raise MGError(st, "mg_create_psi")
        else:
            st = lib.mg_create(ctypes.byref(p), cptr, cdt, _stream_ptr(), ctypes.byref(h_ctx))
            if st != _lib.MG_OK:
                raise MGError(st, "mg_create")
        self._ctx = h_ctx

    # ---------------------------------------------------------------- lifecycle
    def close(self):
        if getattr(self, "_ctx", None):
            _lib.load().mg_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, st, where):
        detail = _lib.load().mg_last_error(self._ctx).decode()
        return MGError(st, where, detail)

    def _sync_stream(self):
        _lib.load().mg_set_stream(self._ctx, _stream_ptr())

    # ---------------------------------------------------------------- solves
    def solve(self, b, phi0=None, tol: float = 1e-10, max_cycles: int = 50, history: bool = True,
              raise_on_error: bool = True, out=None) -> Tuple[object, SolveInfo]:
        """Solve ``M phi = b - mean(b)`` from ``phi0`` (zero if None); returns
        ``(phi, info)`` with zero-mean ``phi``."""
        torch = _torch()
        _check_field(b, self.n, torch.float64, "b")
        if out is None:
            out = torch.zeros_like(b) if phi0 is None else phi0.clone()
        elif phi0 is not None and phi0.data_ptr() != out.data_ptr():
            out.copy_(phi0)
        _check_field(out, self.n, torch.float64, "phi")
        return out, self._run("mg_solve", out, b, tol, max_cycles, history, raise_on_error)

    def solve_pcg(self, b, phi0=None, tol: float = 1e-10, max_iter: int = 50, history: bool = True,
                  raise_on_error: bool = True, out=None) -> Tuple[object, SolveInfo]:
        """Multigrid-preconditioned CG from ``phi0`` (``mg_solve_pcg``);
        ``info.cycles`` counts CG iterations."""
        torch = _torch()
        _check_field(b, self.n, torch.float64, "b")
        if out is None:
            out = torch.zeros_like(b) if phi0 is None else phi0.clone()
        elif phi0 is not None and phi0.data_ptr() != out.data_ptr():
            out.copy_(phi0)
        _check_field(out, self.n, torch.float64, "phi")
        return out, self._run("mg_solve_pcg", out, b, tol, max_iter, history, raise_on_error)

    def solve_adjoint(self, phibar, lam0=None, tol: float = 1e-10, max_cycles: int = 50,
                      history: bool = True, raise_on_error: bool = True):
        torch = _torch()
        _check_field(phibar, self.n, torch.float64, "phibar")
        lam = torch.zeros_like(phibar) if lam0 is None else lam0.clone()
        return lam, self._run("mg_solve_adjoint", lam, phibar, tol, max_cycles, history, raise_on_error)

    def _run(self, fname, x, rhs, tol, max_cycles, history, raise_on_error):
        lib = _lib.load()
        self._sync_stream()
        cap = max_cycles + 1 if history else 0
        hist = (ctypes.c_double * max(cap, 1))()
        info = _lib.MgSolveInfo()
        info.history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double)) if history else None
        info.history_cap = cap
        st = getattr(lib, fname)(self._ctx, _ptr(x), _ptr(rhs), float(tol), int(max_cycles), ctypes.byref(info))
        res = SolveInfo(info.cycles, info.rel_res0, info.rel_res,
                        [hist[i] for i in range(min(info.cycles + 1, cap))] if history else [], st)
        if st not in (_lib.MG_OK, _lib.MG_ERR_NOT_CONVERGED) or (raise_on_error and st != _lib.MG_OK):
            raise self._err(st, fname)
        return res

    def cycles(self, phi, b, cycles: int) -> float:
        """Exactly ``cycles`` warm defect-correction cycles on ``phi`` in place
        (``mg_cycles``), then the gauge; returns the final relative residual."""
        torch = _torch()
        _check_field(phi, self.n, torch.float64, "phi")
        _check_field(b, self.n, torch.float64, "b")
        self._sync_stream()
        out = ctypes.c_double(0.0)
        st = _lib.load().mg_cycles(self._ctx, _ptr(phi), _ptr(b), int(cycles), ctypes.byref(out))
        if st != _lib.MG_OK:
            raise self._err(st, "mg_cycles")
        return out.value

    _STEPS = {"smooth": _lib.MG_STEP_SMOOTH, "smooth_zero": _lib.MG_STEP_SMOOTH_ZERO,
              "prolong_smooth": _lib.MG_STEP_PROLONG_SMOOTH, "residual_restrict": _lib.MG_STEP_RESIDUAL_RESTRICT,
              "prolong": _lib.MG_STEP_PROLONG, "vcycle": _lib.MG_STEP_VCYCLE}

    def inner_step(self, step: str, level: int = 0, x=None, e=None, b=None):
        """One V-cycle step in the context's inner precision through the
        kernels the solver itself launches (``mg_inner_step``); double in and
        out.  ``step``: smooth, smooth_zero, prolong_smooth, residual_restrict,
        prolong or vcycle."""
        torch = _torch()
        nl = self._level_n(level)
        for name, t, m in (("x", x, nl), ("b", b, nl), ("e", e, nl // 2)):
            if t is not None:
                _check_field(t, m, torch.float64, name)
        ref = b if b is not None else x
        shape = (nl // 2,) * 3 if step == "residual_restrict" else (nl,) * 3
        out = torch.empty(shape, dtype=torch.float64, device=ref.device)
        self._sync_stream()
        p = lambda t: _ptr(t) if t is not None else None  # noqa: E731
        st = _lib.load().mg_inner_step(self._ctx, self._STEPS[step], int(level), p(x), p(e), p(b), _ptr(out))
        if st != _lib.MG_OK:
            raise self._err(st, "mg_inner_step")
        return out

    def vcycle(self, phi, b, rel_res: bool = False):
        """One defect-correction cycle in place: ``phi <- phi + V(b - M phi)``."""
        torch = _torch()
        _check_field(phi, self.n, torch.float64, "phi")
        _check_field(b, self.n, torch.float64, "b")
        self._sync_stream()
        out = ctypes.c_double(0.0)
        st = _lib.load().mg_vcycle(self._ctx, _ptr(phi), _ptr(b), ctypes.byref(out) if rel_res else None)
        if st != _lib.MG_OK:
            raise self._err(st, "mg_vcycle")
        return out.value if rel_res else None

    def coeff_grad(self, lam, phi, dtype=None):
        """``dL/dC = -d(lam^T M(C) phi)/dC`` as a ``(6, n, n, n)`` tensor."""
        torch = _torch()
        dtype = torch.float64 if dtype is None else dtype
        _check_field(lam, self.n, torch.float64, "lam")
        _check_field(phi, self.n, torch.float64, "phi")
        cbar = torch.empty((6, self.n, self.n, self.n), dtype=dtype, device=phi.device)
        self._sync_stream()
        dt = _lib.MG_DTYPE_F64 if dtype == torch.float64 else _lib.MG_DTYPE_F32
        st = _lib.load().mg_coeff_grad(self._ctx, _ptr(lam), _ptr(phi), _ptr(cbar), dt)
        if st != _lib.MG_OK:
            raise self._err(st, "mg_coeff_grad")
        return cbar

    # ---------------------------------------------------------------- single steps
    def _level_n(self, level):
        return self.n >> level

    def apply(self, u, level: int = 0):
        torch = _torch()
        _check_field(u, self._level_n(level), torch.float64, "u")
        out = torch.empty_like(u)
        self._sync_stream()
        st = _lib.load().mg_apply(self._ctx, level, _ptr(u), _ptr(out))
        if st != _lib.MG_OK:
            raise self._err(st, "mg_apply")
        return out

    def smooth(self, x, b, level: int = 0):
        torch = _torch()
        _check_field(x, self._level_n(level), torch.float64, "x")
        _check_field(b, self._level_n(level), torch.float64, "b")
        x = x.clone()
        self._sync_stream()
        st = _lib.load().mg_smooth(self._ctx, level, _ptr(x), _ptr(b))
        if st != _lib.MG_OK:
            raise self._err(st, "mg_smooth")
        return x

    def residual_restrict(self, x, b, level: int = 0):
        torch = _torch()
        nl = self._level_n(level)
        _check_field(b, nl, torch.float64, "b")
        if x is not None:
            _check_field(x, nl, torch.float64, "x")
        out = torch.empty((nl // 2,) * 3, dtype=torch.float64, device=b.device)
        self._sync_stream()
        st = _lib.load().mg_residual_restrict(self._ctx, level, _ptr(x) if x is not None else None, _ptr(b), _ptr(out))
        if st != _lib.MG_OK:
            raise self._err(st, "mg_residual_restrict")
        return out

    def prolong_add(self, e, x, level: int = 0):
        torch = _torch()
        nl = self._level_n(level)
        _check_field(x, nl, torch.float64, "x")
        _check_field(e, nl // 2, torch.float64, "e")
        x = x.clone()
        self._sync_stream()
        st = _lib.load().mg_prolong_add(self._ctx, level, _ptr(e), _ptr(x))
        if st != _lib.MG_OK:
            raise self._err(st, "mg_prolong_add")
        return x

    def coarse_solve(self, r):
        torch = _torch()
        _check_field(r, self._level_n(self.levels - 1), torch.float64, "r")
        e = torch.empty_like(r)
        self._sync_stream()
        st = _lib.load().mg_coarse_solve(self._ctx, _ptr(r), _ptr(e))
        if st != _lib.MG_OK:
            raise self._err(st, "mg_coarse_solve")
        return e

    def level_lmax(self):
        arr = (ctypes.c_double * self.levels)()
        _lib.load().mg_level_lmax(self._ctx, arr)
        return list(arr)

    # ---------------------------------------------------------------- timing
    def enable_kernel_timing(self, mask: int = _lib.MG_TIME_STEP):
        """Time fine-level kernels of the kinds in ``mask`` (MG_TIME_STEP
        one-step smoothing, MG_TIME_PAIR two-step passes, MG_TIME_TRIPLE
        three-step passes, MG_TIME_OUTER the outer defect kernel,
        MG_TIME_TRANSFER residual + restriction and prolongation; 0 or False
        disables, True means MG_TIME_STEP)."""
        st = _lib.load().mg_enable_kernel_timing(self._ctx, int(mask))
        if st != _lib.MG_OK:
            raise self._err(st, "mg_enable_kernel_timing")

    def kernel_timing(self):
        """(launches, total_ms, algorithmic_bytes) of the timed fine-level
        kernels since the last call."""
        k = ctypes.c_int(0)
        ms = ctypes.c_double(0.0)
        by = ctypes.c_double(0.0)
        st = _lib.load().mg_kernel_timing(self._ctx, ctypes.byref(k), ctypes.byref(ms), ctypes.byref(by))
        if st != _lib.MG_OK:
            raise self._err(st, "mg_kernel_timing")
        return k.value, ms.value, by.value


# ---------------------------------------------------------------------- predictors, forces
def predict(kind: str, history, growth: float = 1.0, out=None):
    """Initial guess from earlier solutions, newest first (``mg_predict``):
    "recycle", "growth" (``growth * phi1``), "linear" or "quadratic"."""
    torch = _torch()
    need = {"recycle": 1, "growth": 1, "linear": 2, "quadratic": 3}[kind]
    if len(history) < need:
        raise ValueError(f"{kind} needs {need} earlier solutions")
    n = history[0].shape[0]
    for k, t in enumerate(history[:need]):
        _check_field(t, n, torch.float64, f"history[{k}]")
    out = torch.empty_like(history[0]) if out is None else out
    _check_field(out, n, torch.float64, "out")
    ptrs = [_ptr(history[k]) if k < need else None for k in range(3)]
    st = _lib.load().mg_predict(n, _PREDICTOR[kind], ptrs[0], ptrs[1], ptrs[2], float(growth), _ptr(out),
                                _stream_ptr())
    if st != _lib.MG_OK:
        raise MGError(st, "mg_predict")
    return out


def accel(phi, psi=None, scale: float = 1.0, h: Optional[float] = None, dtype=None):
    """``a = -scale J^-1 grad phi`` as a ``(3, n, n, n)`` tensor (``mg_accel``)."""
    torch = _torch()
    n = phi.shape[0]
    _check_field(phi, n, torch.float64, "phi")
    if psi is not None:
        _check_field(psi, n, torch.float64, "psi")
    dtype = torch.float64 if dtype is None else dtype
    h = 1.0 / n if h is None else h
    a = torch.empty((3, n, n, n), dtype=dtype, device=phi.device)
    dt = _lib.MG_DTYPE_F64 if dtype == torch.float64 else _lib.MG_DTYPE_F32
    st = _lib.load().mg_accel(n, float(h), _ptr(phi), _ptr(psi) if psi is not None else None, float(scale),
                              _ptr(a), dt, _stream_ptr())
    if st != _lib.MG_OK:
        raise MGError(st, "mg_accel")
    return a


# ---------------------------------------------------------------------- geometry
def geometry(psi, h: Optional[float] = None, dtype=None):
    """``(C, sqrt_g)`` of the deformation potential ``psi`` (Sec. 4.2)."""
    torch = _torch()
    n = psi.shape[0]
    _check_field(psi, n, torch.float64, "psi")
    dtype = torch.float64 if dtype is None else dtype
    h = 1.0 / n if h is None else h
    C = torch.empty((6, n, n, n), dtype=dtype, device=psi.device)
    sg = torch.empty_like(psi)
    dt = _lib.MG_DTYPE_F64 if dtype == torch.float64 else _lib.MG_DTYPE_F32
    st = _lib.load().mg_geometry(n, float(h), _ptr(psi), _ptr(C), dt, _ptr(sg), _stream_ptr())
    if st != _lib.MG_OK:
        raise MGError(st, "mg_geometry")
    return C, sg


def geometry_bwd(psi, Cbar, sqrtgbar=None, h: Optional[float] = None):
    torch = _torch()
    n = psi.shape[0]
    _check_field(psi, n, torch.float64, "psi")
    Cbar = Cbar.to(torch.float64).contiguous()
    _check_field(Cbar, n, torch.float64, "Cbar", comps=6)
    if sqrtgbar is not None:
        sqrtgbar = sqrtgbar.to(torch.float64).contiguous()
        _check_field(sqrtgbar, n, torch.float64, "sqrtgbar")
    h = 1.0 / n if h is None else h
    out = torch.empty_like(psi)
    st = _lib.load().mg_geometry_bwd(n, float(h), _ptr(psi), _ptr(Cbar),
                                     _ptr(sqrtgbar) if sqrtgbar is not None else None, _ptr(out), _stream_ptr())
    if st != _lib.MG_OK:
        raise MGError(st, "mg_geometry_bwd")
    return out


# ---------------------------------------------------------------------- autograd
def _autograd():
    torch = _torch()

    class GeometryFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, psi, h, dtype):
            C, sg = geometry(psi, h, dtype)
            ctx.save_for_backward(psi)
            ctx.h = h
            return C, sg

        @staticmethod
        def backward(ctx, Cbar, sgbar):
            (psi,) = ctx.saved_tensors
            if Cbar is None:
                Cbar = torch.zeros((6,) + tuple(psi.shape), dtype=torch.float64, device=psi.device)
            return geometry_bwd(psi, Cbar, sgbar, ctx.h), None, None

    class SolveFn(torch.autograd.Function):
        """phi = M(C)^+ (b - mean b): implicit adjoint, differentiated at the
        converged solution rather than through the cycles (Sec. 4.8).  The
        implicit gradient holds only at a converged solve, so a forward or
        adjoint solve that misses its tolerance raises MGError."""

        @staticmethod
        def forward(ctx, b, C, opts):
            mg = _solve_context(b.shape[0], C, opts["ctx"])
            phi, info = mg.solve(b.detach().contiguous(), tol=opts["tol"], max_cycles=opts["max_cycles"])
            ctx.mg = mg
            ctx.opts = opts
            ctx.c_dtype = None if C is None else C.dtype
            ctx.save_for_backward(phi)
            return phi

        @staticmethod
        def backward(ctx, phibar):
            (phi,) = ctx.saved_tensors
            mg = ctx.mg
            lam, _ = mg.solve_adjoint(phibar.contiguous().to(torch.float64), tol=ctx.opts["tol"],
                                      max_cycles=ctx.opts["max_cycles"])
            Cbar = None
            if ctx.c_dtype is not None and ctx.needs_input_grad[1]:
                Cbar = mg.coeff_grad(lam, phi, dtype=ctx.c_dtype)
            return lam, Cbar, None

    return GeometryFn, SolveFn


_FNS = None
# Contexts of the differentiable solve, reused while the coefficient tensor is
# the same object with an unchanged version counter (setup restricts C to
# every level, bounds the spectra and factors the coarsest operator).
_SOLVE_CTX = []
_SOLVE_CTX_MAX = 2


def _solve_context(n, C, ctx_opts):
    import weakref

    key = (int(n), tuple(sorted(ctx_opts.items())),
           None if C is None else (C.data_ptr(), C.dtype, tuple(C.shape), C._version))
    for i, (k, ref, mg) in enumerate(_SOLVE_CTX):
        if k == key and (C is None or ref() is C):
            _SOLVE_CTX.insert(0, _SOLVE_CTX.pop(i))
            return mg
    mg = Multigrid(n, coeff=None if C is None else C.detach(), **ctx_opts)
    _SOLVE_CTX.insert(0, (key, None if C is None else weakref.ref(C), mg))
    del _SOLVE_CTX[_SOLVE_CTX_MAX:]
    return mg


def _fns():
    global _FNS
    if _FNS is None:
        _FNS = _autograd()
    return _FNS


def geometry_fn(psi, h: Optional[float] = None, dtype=None):
    """Differentiable :func:`geometry` (backward through ``mg_geometry_bwd``)."""
    torch = _torch()
    h = 1.0 / psi.shape[0] if h is None else h
    return _fns()[0].apply(psi, h, torch.float64 if dtype is None else dtype)


def solve(b, C=None, tol: float = 1e-10, max_cycles: int = 100, **ctx_opts):
    """Differentiable solve ``phi = M(C)^+ (b - mean b)`` with respect to ``b`` and ``C``."""
    opts = {"ctx": ctx_opts, "tol": tol, "max_cycles": max_cycles}
    return _fns()[1].apply(b, C, opts)


solve_fn = solve
