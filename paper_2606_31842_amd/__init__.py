"""Python binding of libwaveholtz (the WaveHoltz filter and deflated Krylov solvers
on MI355X).  PyTorch supplies device memory and the stream; every computation
runs in the library's HIP kernels.  There is no CPU fallback: if the library is
missing or no GPU is present, calls raise.

Arrays are nodal torch float64 tensors of shape (n+1,)*dim on the GPU (last axis
x); boundary entries of inputs are ignored and of outputs are zero.
"""
from __future__ import annotations

import ctypes as C
import threading
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import _native as nat
from ._native import (WH_F64, WH_MIXED, WH_FPI, WH_CG, WH_DCG, WH_GMRES, WH_BICGSTAB, WH_DEFL_NONE,  # noqa: F401
                      WH_DEFL_SINE, WH_DEFL_DENSE_EXACT, WH_DEFL_DENSE, WH_DEFL_FACTORED, WH_OK,
                      WH_ENOCONV)

_SOLVERS = {"fpi": WH_FPI, "cg": WH_CG, "dcg": WH_DCG, "gmres": WH_GMRES, "bicgstab": WH_BICGSTAB}
_PRECISIONS = {"f64": WH_F64, "mixed": WH_MIXED}


class WaveHoltzError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"waveholtz status {status}: {msg}")
        self.status = status


def _torch():
    import torch
    return torch


_ctx_lock = threading.Lock()
_ctxs = {}


def context(device: Optional[int] = None):
    """A library context bound to the device and torch's current stream."""
    torch = _torch()
    if not torch.cuda.is_available():
        raise RuntimeError("libwaveholtz needs a ROCm GPU; none is visible")
    lib = nat.load()
    dev = torch.cuda.current_device() if device is None else device
    stream = torch.cuda.current_stream(dev).cuda_stream
    with _ctx_lock:
        ctx = _ctxs.get(dev)
        if ctx is None:
            h = C.c_void_p()
            st = lib.wh_create(C.byref(h), dev, C.c_void_p(stream))
            if st != 0:
                raise WaveHoltzError(st, "wh_create failed: " + lib.wh_last_error(None).decode())
            ctx = h
            _ctxs[dev] = ctx
        lib.wh_set_stream(ctx, C.c_void_p(stream))
    return ctx


def params(omega: float, **kw) -> nat.WhParams:
    p = nat.WhParams()
    nat.load().wh_params_default(C.byref(p))
    p.omega = float(omega)
    for k, v in kw.items():
        if k == "solver":
            v = _SOLVERS[v] if isinstance(v, str) else v
        if k == "precision":
            v = _PRECISIONS[v] if isinstance(v, str) else v
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def _grid(dim, n, order=2):
    return nat.WhGrid(dim, n, int(order))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check(lib, ctx, st, allow_noconv=True):
    if st < 0 or (st > 0 and not allow_noconv):
        raise WaveHoltzError(st, lib.wh_last_error(ctx).decode())


def _nodal(t, dim, n, name):
    torch = _torch()
    if t is None:
        return None
    if t.dtype != torch.float64 or not t.is_cuda or tuple(t.shape) != (n + 1,) * dim or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape {(n + 1,) * dim}")
    return t


def _workspace(bytes_):
    torch = _torch()
    return torch.empty(max(int(bytes_), 256), dtype=torch.uint8, device="cuda")


@dataclass
class Deflation:
    """A deflation set: analytic sine modes (``modes``: (n_d, dim) ints), dense
    eigenvector columns ``V`` ((n_d, (n+1)^dim) float64 CUDA tensor, row k = column k)
    with their ``lambda2``, or 2D eigenvectors as separable terms (``fx``, ``fy``:
    (T, n+1) float64 CUDA tensors, ``term_mode``: (T,) ints, mode k = sum over its
    terms of fy_t(y) fx_t(x)) with their ``lambda2``."""
    kind: int
    modes: Optional[np.ndarray] = None
    V: Optional[object] = None
    lambda2: Optional[np.ndarray] = None
    fx: Optional[object] = None
    fy: Optional[object] = None
    term_mode: Optional[np.ndarray] = None

    @property
    def n_d(self):
        if self.kind == WH_DEFL_SINE:
            return int(self.modes.shape[0])
        if self.kind == WH_DEFL_FACTORED:
            return int(len(self.lambda2))
        return int(self.V.shape[0])

    def to_c(self):
        d = nat.WhDeflation()
        d.kind = self.kind
        d.n_d = self.n_d
        self._keep = []
        if self.modes is not None:
            m = np.ascontiguousarray(self.modes, dtype=np.int32)
            self._keep.append(m)
            d.modes = m.ctypes.data_as(C.POINTER(C.c_int32))
        if self.V is not None:
            d.V = C.c_void_p(self.V.data_ptr())
            d.ldv = int(self.V.stride(0))
        if self.lambda2 is not None:
            l2 = np.ascontiguousarray(self.lambda2, dtype=np.float64)
            self._keep.append(l2)
            d.lambda2 = l2.ctypes.data_as(C.POINTER(C.c_double))
        if self.term_mode is not None:
            tm = np.ascontiguousarray(self.term_mode, dtype=np.int32)
            self._keep.append(tm)
            d.n_terms = int(tm.shape[0])
            d.term_mode = tm.ctypes.data_as(C.POINTER(C.c_int32))
            d.fx = C.c_void_p(self.fx.data_ptr())
            d.fy = C.c_void_p(self.fy.data_ptr())
        return d


def factored_deflation(fx, fy, term_mode, lambda2) -> Deflation:
    """Deflation set of 2D eigenvectors of L_h given as separable terms: term t is
    fy[t](y) fx[t](x) and belongs to eigenvector term_mode[t] (non-decreasing), the form the
    compress_modes.py preprocessing script writes (Section 4.3); fx, fy: (T, n+1) arrays
    (numpy or CUDA tensors)."""
    torch = _torch()

    def dev(a):
        t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
        return t.to(device="cuda", dtype=torch.float64).contiguous()
    return Deflation(WH_DEFL_FACTORED, lambda2=np.asarray(lambda2, dtype=np.float64), fx=dev(fx), fy=dev(fy),
                     term_mode=np.asarray(term_mode, dtype=np.int32))


def select_sine_modes(dim: int, n: int, omega: float, n_d: int, order: int = 2):
    """(modes (n_d, dim) int32, lambda2 (n_d,)) nearest to resonance for the operator of
    this order (2, or 4)."""
    lib = nat.load()
    modes = np.zeros((n_d, dim), dtype=np.int32)
    lam2 = np.zeros(n_d)
    st = lib.wh_select_sine_modes(dim, n, int(order), float(omega), n_d, modes.ctypes.data_as(C.POINTER(C.c_int32)),
                                  lam2.ctypes.data_as(C.POINTER(C.c_double)))
    if st != 0:
        raise WaveHoltzError(st, "wh_select_sine_modes")
    return modes, lam2


def sine_deflation(dim, n, omega, n_d, order: int = 2) -> Deflation:
    modes, lam2 = select_sine_modes(dim, n, omega, n_d, order)
    return Deflation(WH_DEFL_SINE, modes=modes, lambda2=None)


def time_params(dim, n, omega, c_max=1.0, **kw):
    lib = nat.load()
    order = kw.pop("order", 2)
    p = params(omega, **kw)
    g = _grid(dim, n, order)
    m, nt = C.c_int32(), C.c_int32()
    dt, om = C.c_double(), C.c_double()
    st = lib.wh_time_params(C.byref(g), C.byref(p), float(c_max), C.byref(m), C.byref(nt), C.byref(dt),
                            C.byref(om))
    if st != 0:
        raise WaveHoltzError(st, "wh_time_params")
    return {"m": m.value, "nt": nt.value, "dt": dt.value, "omega_tilde": om.value}


def transfer(dim, n, omega, lambda2, c_max=1.0, **kw):
    lib = nat.load()
    order = kw.pop("order", 2)
    p = params(omega, **kw)
    g = _grid(dim, n, order)
    lam = np.ascontiguousarray(lambda2, dtype=np.float64).ravel()
    out = np.zeros_like(lam)
    st = lib.wh_transfer(C.byref(g), C.byref(p), float(c_max), lam.size,
                         lam.ctypes.data_as(C.POINTER(C.c_double)), out.ctypes.data_as(C.POINTER(C.c_double)))
    if st != 0:
        raise WaveHoltzError(st, "wh_transfer")
    return out


def workspace_bytes(dim, n, p: nat.WhParams, defl: Optional[Deflation] = None, order: int = 2) -> int:
    lib = nat.load()
    g = _grid(dim, n, order)
    d = defl.to_c() if defl is not None else None
    return int(lib.wh_workspace_bytes(C.byref(g), C.byref(p), C.byref(d) if d is not None else None))


def apply_filter(v, omega, f=None, c2=None, out=None, **kw):
    """Pi_h(v; f) on the GPU.  Returns (out, info)."""
    torch = _torch()
    dim = v.dim()
    n = v.shape[0] - 1
    _nodal(v, dim, n, "v"); _nodal(f, dim, n, "f"); _nodal(c2, dim, n, "c2")
    lib = nat.load()
    ctx = context(v.device.index)
    order = kw.pop("order", 2)
    p = params(omega, **kw)
    g = _grid(dim, n, order)
    out = torch.empty_like(v) if out is None else _nodal(out, dim, n, "out")
    ws = _workspace(lib.wh_workspace_bytes(C.byref(g), C.byref(p), None))
    info = nat.WhInfo()
    st = lib.wh_apply_filter(ctx, C.byref(g), _ptr(c2), _ptr(f), _ptr(v), _ptr(out), C.byref(p), _ptr(ws),
                             ws.numel(), C.byref(info))
    _check(lib, ctx, st)
    return out, info.as_dict()


def apply_filter_noalloc(v, omega, f=None, c2=None, out=None, **kw):
    """Pi_h(v; f) through wh_apply_filter_noalloc (no workspace; the library's fixed device
    scratch).  Returns (out, info)."""
    torch = _torch()
    dim = v.dim()
    n = v.shape[0] - 1
    _nodal(v, dim, n, "v"); _nodal(f, dim, n, "f"); _nodal(c2, dim, n, "c2")
    lib = nat.load()
    ctx = context(v.device.index)
    order = kw.pop("order", 2)
    p = params(omega, **kw)
    g = _grid(dim, n, order)
    out = torch.empty_like(v) if out is None else _nodal(out, dim, n, "out")
    info = nat.WhInfo()
    st = lib.wh_apply_filter_noalloc(ctx, C.byref(g), _ptr(c2), _ptr(f), _ptr(v), _ptr(out), C.byref(p),
                                     C.byref(info))
    _check(lib, ctx, st)
    return out, info.as_dict()


def solve(f, omega, c2=None, u0=None, defl: Optional[Deflation] = None, workspace=None, **kw):
    """Solve the WaveHoltz system for L u + omega^2 u = f.  Returns (u, info)."""
    torch = _torch()
    dim = f.dim()
    n = f.shape[0] - 1
    _nodal(f, dim, n, "f"); _nodal(c2, dim, n, "c2")
    lib = nat.load()
    ctx = context(f.device.index)
    order = kw.pop("order", 2)
    p = params(omega, **kw)
    g = _grid(dim, n, order)
    d = defl.to_c() if defl is not None else None
    need = lib.wh_workspace_bytes(C.byref(g), C.byref(p), C.byref(d) if d is not None else None)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need)
    u = torch.zeros_like(f) if u0 is None else _nodal(u0, dim, n, "u0").clone()
    info = nat.WhInfo()
    st = lib.wh_solve(ctx, C.byref(g), _ptr(c2), _ptr(f), C.byref(d) if d is not None else None, C.byref(p),
                      _ptr(u), _ptr(ws), ws.numel(), C.byref(info))
    _check(lib, ctx, st)
    return u, info.as_dict()


def helmholtz_residual(u, f, omega, c2=None, order=2):
    torch = _torch()
    dim = u.dim()
    n = u.shape[0] - 1
    lib = nat.load()
    ctx = context(u.device.index)
    g = _grid(dim, n, order)
    ws = _workspace(16 * 1024 + 4096)
    rel = C.c_double()
    st = lib.wh_helmholtz_residual(ctx, C.byref(g), _ptr(c2), _ptr(f), float(omega), _ptr(u), _ptr(ws),
                                   ws.numel(), C.byref(rel))
    _check(lib, ctx, st)
    return rel.value


def time_step_kernel(v, omega, c2=None, reps=50, shape=False, **kw):
    """Average milliseconds per launch of the time-stepping kernel the library picks
    for this grid (see wh_time_step_kernel).  With shape=True returns
    (ms, {"k": K, "rows": R, "waves": NW})."""
    dim = v.dim()
    n = v.shape[0] - 1
    lib = nat.load()
    ctx = context(v.device.index)
    order = kw.pop("order", 2)
    p = params(omega, **kw)
    g = _grid(dim, n, order)
    ws = _workspace(lib.wh_workspace_bytes(C.byref(g), C.byref(p), None))
    us = C.c_double()
    k, rows, waves = C.c_int32(), C.c_int32(), C.c_int32()
    st = lib.wh_time_step_kernel(ctx, C.byref(g), _ptr(c2), C.byref(p), int(reps), _ptr(ws), ws.numel(),
                                 C.byref(us), C.byref(k), C.byref(rows), C.byref(waves))
    _check(lib, ctx, st)
    if shape:
        return us.value / 1e3, {"k": k.value, "rows": rows.value, "waves": waves.value}
    return us.value / 1e3


def _batch(problems, n_defl, order=2):
    """ctypes problem array (and the output tensors) for wh_solve_batched / wh_time_batch_kernel."""
    torch = _torch()
    nb = len(problems)
    nds = [int(n_defl)] * nb if np.isscalar(n_defl) else [int(v) for v in n_defl]
    if len(nds) != nb:
        raise ValueError("n_defl needs one entry per problem")
    arr = (nat.WhProblem * nb)()
    outs = []
    ctx = None
    for i, pr in enumerate(problems):
        f, om = pr[0], pr[1]
        c2 = pr[2] if len(pr) > 2 else None
        n = f.shape[0] - 1
        _nodal(f, 2, n, "f"); _nodal(c2, 2, n, "c2")
        u = torch.empty_like(f)
        outs.append(u)
        arr[i].grid = _grid(2, n, order)
        arr[i].c2 = None if c2 is None else c2.data_ptr()
        arr[i].f = f.data_ptr()
        arr[i].omega = float(om)
        arr[i].u = u.data_ptr()
        arr[i].n_defl = nds[i]
        if ctx is None:
            ctx = context(f.device.index)
    return arr, outs, ctx


def batch_workspace_bytes(problems, n_defl=0, **kw) -> int:
    """Workspace bytes wh_solve_batched needs for these problems and parameters."""
    lib = nat.load()
    arr, _, _ = _batch(problems, n_defl, kw.pop("order", 2))
    p = params(float(problems[0][1]), **kw)
    return int(lib.wh_workspace_bytes_batched(len(problems), arr, C.byref(p)))


def solve_batched(problems, workspace=None, n_defl=0, **kw):
    """Solve many 2D problems in one device-driven batch (wh_solve_batched).

    problems: sequence of (f, omega) or (f, omega, c2) with nodal float64 CUDA tensors.
    n_defl: sine modes deflated per problem (an int for all, or one per problem; needs
    solver="dcg" and c == 1).  order=4: fourth-order differences (c == 1) for every problem.
    Returns (list of solutions, list of info dicts)."""
    lib = nat.load()
    nb = len(problems)
    arr, outs, ctx = _batch(problems, n_defl, kw.pop("order", 2))
    p = params(float(problems[0][1]), **kw)
    need = lib.wh_workspace_bytes_batched(nb, arr, C.byref(p))
    if need == 0:
        raise WaveHoltzError(-1, "invalid batch (wh_workspace_bytes_batched returned 0)")
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need)
    infos = (nat.WhInfo * nb)()
    st = lib.wh_solve_batched(ctx, nb, arr, C.byref(p), _ptr(ws), ws.numel(), infos)
    _check(lib, ctx, st)
    return outs, [infos[i].as_dict() for i in range(nb)]


def time_batch_kernel(problems, reps=20, workspace=None, n_defl=0, **kw):
    """(microseconds per launch, interior points per launch) of the batched solver's FP32 work
    kernel with every problem in its time-stepping phase (wh_time_batch_kernel)."""
    lib = nat.load()
    nb = len(problems)
    arr, _, ctx = _batch(problems, n_defl, kw.pop("order", 2))
    kw = dict(kw, precision="mixed")
    p = params(float(problems[0][1]), **kw)
    need = lib.wh_workspace_bytes_batched(nb, arr, C.byref(p))
    if need == 0:
        raise WaveHoltzError(-1, "invalid batch (wh_workspace_bytes_batched returned 0)")
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need)
    us, pts = C.c_double(), C.c_int64()
    st = lib.wh_time_batch_kernel(ctx, nb, arr, C.byref(p), int(reps), _ptr(ws), ws.numel(), C.byref(us),
                                  C.byref(pts))
    _check(lib, ctx, st)
    return us.value, pts.value


def coeff_bound(c2) -> float:
    """c_max = sqrt(max c2) of a nodal float64 CUDA coefficient array (wh_coeff_bound)."""
    dim, n = c2.dim(), c2.shape[0] - 1
    _nodal(c2, dim, n, "c2")
    lib = nat.load()
    ctx = context(c2.device.index)
    g = _grid(dim, n)
    out = C.c_double()
    _check(lib, ctx, lib.wh_coeff_bound(ctx, C.byref(g), _ptr(c2), C.byref(out)))
    return out.value


def solve_vjp(u, grad_u, f, omega, c2, ckpt_every=16, grad_c2=None, **kw):
    """grad_c2 (+)= (dPi_h/dc2)^T A^{-1} grad_u at the fixed point u (wh_solve_vjp)."""
    torch = _torch()
    n = u.shape[0] - 1
    for t, nm in ((u, "u"), (grad_u, "grad_u"), (f, "f"), (c2, "c2")):
        _nodal(t, 2, n, nm)
    lib = nat.load()
    ctx = context(u.device.index)
    if "c_max" not in kw:
        kw["c_max"] = coeff_bound(c2)
    p = params(omega, **kw)
    g = _grid(2, n)
    need = lib.wh_workspace_bytes_adjoint(C.byref(g), C.byref(p), int(ckpt_every))
    if need == 0:
        raise WaveHoltzError(-1, "invalid arguments for the adjoint workspace")
    ws = _workspace(need)
    out = torch.zeros_like(u) if grad_c2 is None else _nodal(grad_c2, 2, n, "grad_c2")
    info = nat.WhInfo()
    st = lib.wh_solve_vjp(ctx, C.byref(g), _ptr(c2), _ptr(f), _ptr(u), _ptr(grad_u), C.byref(p),
                          int(ckpt_every), _ptr(out), _ptr(ws), ws.numel(), C.byref(info))
    _check(lib, ctx, st)
    return out, info.as_dict()


def adjoint_grad(c2, sources, rec_idx, data, omega, ckpt_every=16, need_grad=True, **kw):
    """(J, dJ/dc2, info) for J = 1/2 sum_s ||R u_s - d_s||^2 (wh_adjoint_grad); with
    need_grad=False the misfit alone, (J, None, info)."""
    torch = _torch()
    n = c2.shape[0] - 1
    _nodal(c2, 2, n, "c2")
    lib = nat.load()
    ctx = context(c2.device.index)
    if "c_max" not in kw:
        kw["c_max"] = coeff_bound(c2)
    p = params(omega, **kw)
    g = _grid(2, n)
    srcs = [_nodal(f, 2, n, "source") for f in sources]
    fptr = (C.c_void_p * len(srcs))(*[f.data_ptr() for f in srcs])
    idx = rec_idx.to(device=c2.device, dtype=torch.int64).contiguous()
    d = data.to(device=c2.device, dtype=torch.float64).contiguous()
    assert d.shape == (len(srcs), idx.numel())
    need = lib.wh_workspace_bytes_adjoint(C.byref(g), C.byref(p), int(ckpt_every))
    if need == 0:
        raise WaveHoltzError(-1, "invalid arguments for the adjoint workspace")
    ws = _workspace(need)
    grad = torch.empty_like(c2) if need_grad else None
    J = C.c_double()
    info = nat.WhInfo()
    st = lib.wh_adjoint_grad(ctx, C.byref(g), _ptr(c2), len(srcs), fptr, idx.numel(), _ptr(idx), _ptr(d),
                             C.byref(p), int(ckpt_every), _ptr(grad), C.byref(J), _ptr(ws), ws.numel(),
                             C.byref(info))
    _check(lib, ctx, st)
    return J.value, grad, info.as_dict()


class WaveHoltzSolve:
    """torch.autograd.Function wrapper: u = WaveHoltzSolve.apply(f, c2, omega, kwargs)
    solves the 2D Helmholtz problem with the library; backward gives
    dL/df = H^{-1} dL/du (one more solve, H = L_h + omega^2 is symmetric) and
    dL/dc2 = (dPi_h/dc2)^T A^{-1} dL/du (wh_solve_vjp)."""

    @staticmethod
    def _fn():
        import torch

        class _F(torch.autograd.Function):
            @staticmethod
            def forward(ctx_, f, c2, omega, opts):
                u, _ = solve(f, omega, c2=c2, **opts)
                ctx_.save_for_backward(f, c2, u)
                ctx_.omega = omega
                ctx_.opts = opts
                return u

            @staticmethod
            def backward(ctx_, gu):
                f, c2, u = ctx_.saved_tensors
                gu = gu.contiguous()
                opts = {k: v for k, v in ctx_.opts.items() if k != "defl"}
                gf = gc2 = None
                if ctx_.needs_input_grad[0]:
                    gf, _ = solve(gu, ctx_.omega, c2=c2, **ctx_.opts)
                if ctx_.needs_input_grad[1]:
                    gc2, _ = solve_vjp(u, gu, f, ctx_.omega, c2, **{k: v for k, v in opts.items()
                                                                   if k not in ("solver",)})
                return gf, gc2, None, None

        return _F

    @classmethod
    def apply(cls, f, c2, omega, opts=None):
        return cls._fn().apply(f, c2, omega, opts or {})
