"""Python binding of libshenhip: argument marshalling only.

Tensors are torch CUDA (HIP) tensors; every call enqueues on torch's current
stream.  Shapes: right-hand sides and solutions are complex128 [..., N]
(wall-normal index last, contiguous), coefficients float64 [...] with the
same leading shape.  Every step of the solve runs in the HIP library.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L

_PREC = {"fp64": L.SHEN_FP64, "fp32_refine": L.SHEN_FP32_REFINE}
_QUAD = {"gc": L.SHEN_QUAD_GC, "gl": L.SHEN_QUAD_GL}
_VARIANT = {"auto": 0, "chain": 1, "wave": 2}


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _work_tensor(work, device):
    """(pointer, bytes) of an in-place workspace: a contiguous device tensor, or None."""
    if work is None:
        return None, 0
    if not isinstance(work, torch.Tensor) or not work.is_contiguous() or work.device != device:
        raise ValueError(f"work must be a contiguous tensor on {device}")
    return work.data_ptr(), work.numel() * work.element_size()


def _opts(device, precision="fp64", quad="gc", transpose=False, info=None, refine_max=8, refine_tol=1e-14,
          variant="auto", chunk=0, iters=None, work=None) -> L.ShenOpts:
    o = L.default_opts()
    o.stream = _stream_handle(device)
    o.precision = _PREC[precision]
    o.quad = _QUAD[quad]
    o.transpose = int(bool(transpose))
    o.refine_max = int(refine_max)
    o.refine_tol = float(refine_tol)
    o.info = info.data_ptr() if info is not None else None
    o.variant = _VARIANT[variant] if isinstance(variant, str) else int(variant)
    o.chunk = int(chunk)
    o.iters = iters.data_ptr() if iters is not None else None
    o.work, o.work_bytes = _work_tensor(work, device)
    return o


def _rows(x: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(x, torch.Tensor) or x.dtype != torch.complex128:
        raise TypeError(f"{name} must be a complex128 tensor")
    if not x.is_cuda:
        raise ValueError(f"{name} must be on a HIP device (no CPU path)")
    if x.dim() < 1:
        raise ValueError(f"{name} must have the wall-normal axis last")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return x


def _out(out, like: torch.Tensor, name: str = "out") -> torch.Tensor:
    """A fresh result like `like`, or the caller's tensor after checking it matches."""
    if out is None:
        return torch.empty_like(like)
    if not isinstance(out, torch.Tensor) or out.dtype != torch.complex128:
        raise TypeError(f"{name} must be a complex128 tensor")
    if tuple(out.shape) != tuple(like.shape):
        raise ValueError(f"{name} has shape {tuple(out.shape)}, expected {tuple(like.shape)}")
    if out.device != like.device:
        raise ValueError(f"{name} must be on {like.device}")
    return _rows(out, name)


def _like(x, ref: torch.Tensor, name: str) -> torch.Tensor:
    """An input that must match ref's shape and device (complex128, contiguous)."""
    x = _rows(x, name)
    if x.device != ref.device:
        raise ValueError(f"{name} must be on {ref.device}")
    if tuple(x.shape) != tuple(ref.shape):
        raise ValueError(f"{name} has shape {tuple(x.shape)}, expected {tuple(ref.shape)}")
    return x


def _coef(c: torch.Tensor, lead, device, name: str) -> torch.Tensor:
    if not isinstance(c, torch.Tensor) or c.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 tensor")
    if c.device != device:
        raise ValueError(f"{name} must be on {device}")
    if tuple(c.shape) != tuple(lead):
        raise ValueError(f"{name} has shape {tuple(c.shape)}, expected {tuple(lead)}")
    if not c.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return c


def _info_tensor(want, lead, device, name="info"):
    if want is None or want is False:
        return None
    if isinstance(want, torch.Tensor):
        if want.dtype != torch.int32 or tuple(want.shape) != tuple(lead) or not want.is_contiguous() or want.device != device:
            raise ValueError(f"{name} must be a contiguous int32 tensor of the batch shape on the same device")
        return want
    return torch.zeros(lead, dtype=torch.int32, device=device)


def _nsys(lead) -> int:
    n = 1
    for s in lead:
        n *= int(s)
    return n


def _result(u, inf, its):
    out = (u,)
    if inf is not None:
        out += (inf,)
    if its is not None:
        out += (its,)
    return out if len(out) > 1 else u


def helmholtz_solve(f, alpha, *, out=None, precision="fp64", quad="gc", transpose=False, info=None, refine_max=8,
                    refine_tol=1e-14, variant="auto", chunk=0, iters=None, work=None):
    """u = (S + alpha B)^{-1} f per system (or the transposed system).

    Returns u, then info and iters when requested (True or an int32 tensor of the batch
    shape): info per system, and for precision="fp32_refine" the corrections applied.
    work: a device tensor of at least nsys * factor_bytes(family, N) bytes, for in-place
    solves (out=f) on the wave kernels."""
    f = _rows(f, "f")
    N = f.shape[-1]
    lead = f.shape[:-1]
    alpha = _coef(alpha, lead, f.device, "alpha")
    u = _out(out, f)
    inf = _info_tensor(info, lead, f.device)
    its = _info_tensor(iters, lead, f.device, "iters")
    o = _opts(f.device, precision, quad, transpose, inf, refine_max, refine_tol, variant, chunk, its, work)
    L.check(L.lib().helmholtz_solve(N, _nsys(lead), alpha.data_ptr(), f.data_ptr(), u.data_ptr(), C.byref(o)),
            "helmholtz_solve")
    return _result(u, inf, its)


def biharmonic_solve(f, a, b, *, out=None, precision="fp64", quad="gc", transpose=False, info=None, refine_max=8,
                     refine_tol=1e-14, variant="auto", chunk=0, iters=None, work=None):
    """u = (Q + a A + b B)^{-1} f per system (or the transposed system); returns as helmholtz_solve."""
    f = _rows(f, "f")
    N = f.shape[-1]
    lead = f.shape[:-1]
    a = _coef(a, lead, f.device, "a")
    b = _coef(b, lead, f.device, "b")
    u = _out(out, f)
    inf = _info_tensor(info, lead, f.device)
    its = _info_tensor(iters, lead, f.device, "iters")
    o = _opts(f.device, precision, quad, transpose, inf, refine_max, refine_tol, variant, chunk, its, work)
    L.check(L.lib().biharmonic_solve(N, _nsys(lead), a.data_ptr(), b.data_ptr(), f.data_ptr(), u.data_ptr(), C.byref(o)),
            "biharmonic_solve")
    return _result(u, inf, its)


def factor_bytes(family, N, *, chunk=0):
    """Bytes per system of the factor-once state (shen_factor_bytes)."""
    o = L.default_opts()
    o.chunk = int(chunk)
    fam = {"helmholtz": L.SHEN_HELMHOLTZ, "biharmonic": L.SHEN_BIHARMONIC}[family]
    nb = L.lib().shen_factor_bytes(fam, int(N), C.byref(o))
    if nb < 0:
        raise L.ShenError(int(nb), "shen_factor_bytes")
    return int(nb)


class ShenFactor:
    """The factor-once state of one batch (helmholtz_factor / biharmonic_factor) with the
    configuration it was made for: family, N, quadrature and chunk length.  The factored
    calls take these from it and refuse a factor of another configuration, whose restart
    states would sit at other chunk boundaries or belong to other matrices."""

    def __init__(self, data: torch.Tensor, family: str, N: int, quad: str, chunk: int):
        self.data = data
        self.family = family
        self.N = int(N)
        self.quad = quad
        self.chunk = int(chunk)

    @property
    def shape(self):
        return self.data.shape

    def data_ptr(self) -> int:
        return self.data.data_ptr()


def _fac_tensor(family, N, lead, device, chunk):
    nb = factor_bytes(family, N, chunk=chunk)
    return torch.empty(tuple(lead) + (nb // 8,), dtype=torch.float64, device=device)


def _check_fac(fac, family, N, lead, device, quad=None, chunk=None):
    """fac's state tensor after checking that it was made for this call; returns (data, quad, chunk)."""
    if not isinstance(fac, ShenFactor):
        raise ValueError("fac must be the ShenFactor returned by helmholtz_factor / biharmonic_factor")
    quad = fac.quad if quad is None else quad
    chunk = fac.chunk if chunk is None else int(chunk)
    want = (family, int(N), quad, chunk)
    have = (fac.family, fac.N, fac.quad, fac.chunk)
    if want != have:
        raise ValueError(f"fac was made for (family, N, quad, chunk) = {have}, this call is {want}")
    nb = factor_bytes(family, N, chunk=chunk)
    d = fac.data
    if (not isinstance(d, torch.Tensor) or d.dtype != torch.float64 or d.device != device
            or tuple(d.shape) != tuple(lead) + (nb // 8,) or not d.is_contiguous()):
        raise ValueError(f"fac must hold a contiguous float64 tensor of shape {tuple(lead) + (nb // 8,)} on {device}")
    return d, quad, chunk


def helmholtz_factor(alpha, N, *, quad="gc", chunk=0):
    """Factor-once: the LU restart states of (S + alpha B) for every system (a ShenFactor)."""
    if not isinstance(alpha, torch.Tensor) or not alpha.is_cuda:
        raise ValueError("alpha must be a float64 tensor on a HIP device (no CPU path)")
    lead = alpha.shape
    alpha = _coef(alpha, lead, alpha.device, "alpha")
    fac = _fac_tensor("helmholtz", N, lead, alpha.device, chunk)
    o = _opts(alpha.device, quad=quad, chunk=chunk)
    L.check(L.lib().helmholtz_factor(int(N), _nsys(lead), alpha.data_ptr(), fac.data_ptr(), C.byref(o)), "helmholtz_factor")
    return ShenFactor(fac, "helmholtz", N, quad, chunk)


def biharmonic_factor(a, b, N, *, quad="gc", chunk=0):
    """Factor-once: the LU restart states of (Q + a A + b B) for every system (a ShenFactor)."""
    if not isinstance(a, torch.Tensor) or not a.is_cuda:
        raise ValueError("a must be a float64 tensor on a HIP device (no CPU path)")
    lead = a.shape
    a = _coef(a, lead, a.device, "a")
    b = _coef(b, lead, a.device, "b")
    fac = _fac_tensor("biharmonic", N, lead, a.device, chunk)
    o = _opts(a.device, quad=quad, chunk=chunk)
    L.check(L.lib().biharmonic_factor(int(N), _nsys(lead), a.data_ptr(), b.data_ptr(), fac.data_ptr(), C.byref(o)),
            "biharmonic_factor")
    return ShenFactor(fac, "biharmonic", N, quad, chunk)


def helmholtz_solve_factored(f, alpha, fac, *, out=None, quad=None, info=None, chunk=None):
    """u = (S + alpha B)^{-1} f from the states of helmholtz_factor (same alpha; quad and chunk
    are the factor's, and must match it when given)."""
    f = _rows(f, "f")
    N = f.shape[-1]
    lead = f.shape[:-1]
    alpha = _coef(alpha, lead, f.device, "alpha")
    facd, quad, chunk = _check_fac(fac, "helmholtz", N, lead, f.device, quad, chunk)
    u = _out(out, f)
    inf = _info_tensor(info, lead, f.device)
    o = _opts(f.device, quad=quad, info=inf, chunk=chunk)
    L.check(L.lib().helmholtz_solve_factored(N, _nsys(lead), alpha.data_ptr(), facd.data_ptr(), f.data_ptr(), u.data_ptr(),
                                             C.byref(o)), "helmholtz_solve_factored")
    return (u, inf) if inf is not None else u


def biharmonic_solve_factored(f, a, b, fac, *, out=None, quad=None, info=None, chunk=None):
    """u = (Q + a A + b B)^{-1} f from the states of biharmonic_factor (same a, b; quad and
    chunk are the factor's)."""
    f = _rows(f, "f")
    N = f.shape[-1]
    lead = f.shape[:-1]
    a = _coef(a, lead, f.device, "a")
    b = _coef(b, lead, f.device, "b")
    facd, quad, chunk = _check_fac(fac, "biharmonic", N, lead, f.device, quad, chunk)
    u = _out(out, f)
    inf = _info_tensor(info, lead, f.device)
    o = _opts(f.device, quad=quad, info=inf, chunk=chunk)
    L.check(L.lib().biharmonic_solve_factored(N, _nsys(lead), a.data_ptr(), b.data_ptr(), facd.data_ptr(), f.data_ptr(),
                                              u.data_ptr(), C.byref(o)), "biharmonic_solve_factored")
    return (u, inf) if inf is not None else u


def helmholtz_matvec(u, alpha, *, out=None, quad="gc", transpose=False):
    u = _rows(u, "u")
    N = u.shape[-1]
    lead = u.shape[:-1]
    alpha = _coef(alpha, lead, u.device, "alpha")
    y = _out(out, u)
    o = _opts(u.device, quad=quad, transpose=transpose)
    L.check(L.lib().helmholtz_matvec(N, _nsys(lead), alpha.data_ptr(), u.data_ptr(), y.data_ptr(), C.byref(o)),
            "helmholtz_matvec")
    return y


def biharmonic_matvec(u, a, b, *, out=None, quad="gc", transpose=False):
    u = _rows(u, "u")
    N = u.shape[-1]
    lead = u.shape[:-1]
    a = _coef(a, lead, u.device, "a")
    b = _coef(b, lead, u.device, "b")
    y = _out(out, u)
    o = _opts(u.device, quad=quad, transpose=transpose)
    L.check(L.lib().biharmonic_matvec(N, _nsys(lead), a.data_ptr(), b.data_ptr(), u.data_ptr(), y.data_ptr(), C.byref(o)),
            "biharmonic_matvec")
    return y


def _rhs(fn, name, u, K2, nu, dt, sh, out, quad, variant):
    u = _rows(u, "uhat")
    N = u.shape[-1]
    lead = u.shape[:-1]
    K2 = _coef(K2, lead, u.device, "K2")
    if sh is not None:
        sh = _like(sh, u, "sh")
    y = _out(out, u)
    o = _opts(u.device, quad=quad, variant=variant)
    L.check(fn(N, _nsys(lead), K2.data_ptr(), float(nu), float(dt), u.data_ptr(),
               sh.data_ptr() if sh is not None else None, y.data_ptr(), C.byref(o)), name)
    return y


def helmholtz_rhs(ghat, K2, nu, dt, sh=None, *, out=None, quad="gc", variant="auto"):
    """Right-hand side of one Crank-Nicolson step of the g equation (Sec. 3, eq. gfin), scaled so
    that helmholtz_solve(rhs, K2 + 2/(nu dt)) advances the step: (2/nu) S(h) - (S + (K2 - 2/(nu dt)) B) ghat.
    sh = S(h_g) (None omits it); out may be sh."""
    return _rhs(L.lib().helmholtz_rhs, "helmholtz_rhs", ghat, K2, nu, dt, sh, out, quad, variant)


def biharmonic_rhs(uhat, K2, nu, dt, sh=None, *, out=None, quad="gc", variant="auto"):
    """Right-hand side of one Crank-Nicolson step of the u equation (Sec. 3, eq. ufin), scaled so
    that biharmonic_solve(rhs, -(2 K2 + 2/(nu dt)), K2 (K2 + 2/(nu dt))) advances the step:
    (-2/nu) S(h) - (Q + (2/(nu dt) - 2 K2) A + K2 (K2 - 2/(nu dt)) B) uhat.  sh = S(h_u) (None omits
    it); out may be sh."""
    return _rhs(L.lib().biharmonic_rhs, "biharmonic_rhs", uhat, K2, nu, dt, sh, out, quad, variant)


def _transform(fn, name, x, space, out, quad):
    x = _rows(x, "input")
    if space not in L.SHEN_SPACE:
        raise ValueError(f"space must be one of {sorted(L.SHEN_SPACE)}")
    N = x.shape[-1]
    y = _out(out, x)
    if y.data_ptr() == x.data_ptr():
        raise ValueError(f"{name}: output must not be the input")
    o = _opts(x.device, quad=quad)
    L.check(fn(N, _nsys(x.shape[:-1]), L.SHEN_SPACE[space], x.data_ptr(), y.data_ptr(), C.byref(o)), name)
    return y


def scalar_product(u, space, *, out=None, quad="gc"):
    """S(u)_k = sum_j u(x_j) phi_k(x_j) sigma_j for point values u [..., N] at the Gauss ("gc") or
    Gauss-Lobatto ("gl") points, phi the basis of space "chebyshev", "dirichlet" or "biharmonic"
    (Sec. 2); entries k >= n are 0."""
    return _transform(L.lib().shen_scalar_product, "shen_scalar_product", u, space, out, quad)


def forward_transform(u, space, *, out=None, quad="gc"):
    """uhat = B^{-1} S(u): the space's coefficients of the point values u (Sec. 2)."""
    return _transform(L.lib().shen_forward_transform, "shen_forward_transform", u, space, out, quad)


def backward_transform(uhat, space, *, out=None, quad="gc"):
    """u(x_j) = sum_k uhat_k phi_k(x_j): point values of the series with coefficients uhat (Sec. 2)."""
    return _transform(L.lib().shen_backward_transform, "shen_backward_transform", uhat, space, out, quad)


def dirichlet_mass_solve(f, *, out=None, quad="gc"):
    """u = Bbar^{-1} f per system, Bbar the Dirichlet-basis mass matrix (Sec. 2 transforms); out may be f."""
    f = _rows(f, "f")
    N = f.shape[-1]
    u = _out(out, f)
    o = _opts(f.device, quad=quad)
    L.check(L.lib().dirichlet_mass_solve(N, _nsys(f.shape[:-1]), f.data_ptr(), u.data_ptr(), C.byref(o)),
            "dirichlet_mass_solve")
    return u


def biharmonic_mass_solve(f, *, out=None, quad="gc"):
    """u = Bchk^{-1} f per system, Bchk the biharmonic-basis mass matrix (Sec. 2 transforms); out may be f."""
    f = _rows(f, "f")
    N = f.shape[-1]
    u = _out(out, f)
    o = _opts(f.device, quad=quad)
    L.check(L.lib().biharmonic_mass_solve(N, _nsys(f.shape[:-1]), f.data_ptr(), u.data_ptr(), C.byref(o)),
            "biharmonic_mass_solve")
    return u


def dirichlet_derivative_solve(uhat, *, out=None, quad="gc"):
    """fhat = Bbar^{-1} Cbar uhat per system: Dirichlet-basis coefficients of du/dx for u in the
    biharmonic basis (Sec. 3); out may be uhat."""
    uhat = _rows(uhat, "uhat")
    N = uhat.shape[-1]
    fhat = _out(out, uhat)
    o = _opts(uhat.device, quad=quad)
    L.check(L.lib().dirichlet_derivative_solve(N, _nsys(uhat.shape[:-1]), uhat.data_ptr(), fhat.data_ptr(), C.byref(o)),
            "dirichlet_derivative_solve")
    return fhat

def helmholtz_adjoint(u, gbar, alpha, *, quad="gc", coef_grad=True, info=None, variant="auto", fac=None, chunk=0):
    """lambda = H^{-T} gbar and grad_alpha = -Re(lambda^H B u); returns (lambda, grad_alpha or None).

    With fac (from helmholtz_factor, same alpha, quad, chunk) the restart states are taken from it."""
    gbar = _rows(gbar, "gbar")
    N = gbar.shape[-1]
    lead = gbar.shape[:-1]
    alpha = _coef(alpha, lead, gbar.device, "alpha")
    lam = torch.empty_like(gbar)
    ga = torch.empty(lead, dtype=torch.float64, device=gbar.device) if coef_grad else None
    if coef_grad:
        u = _like(u, gbar, "u")
    inf = _info_tensor(info, lead, gbar.device)
    o = _opts(gbar.device, quad=quad, info=inf, variant=variant, chunk=chunk)
    up = u.data_ptr() if coef_grad else None
    gp = ga.data_ptr() if ga is not None else None
    if fac is not None:
        facd, _, _ = _check_fac(fac, "helmholtz", N, lead, gbar.device, quad, chunk)
        L.check(L.lib().helmholtz_adjoint_factored(N, _nsys(lead), alpha.data_ptr(), facd.data_ptr(), up, gbar.data_ptr(),
                                                   lam.data_ptr(), gp, C.byref(o)), "helmholtz_adjoint_factored")
    else:
        L.check(L.lib().helmholtz_adjoint(N, _nsys(lead), alpha.data_ptr(), up, gbar.data_ptr(), lam.data_ptr(), gp,
                                          C.byref(o)), "helmholtz_adjoint")
    return (lam, ga, inf) if inf is not None else (lam, ga)


def biharmonic_adjoint(u, gbar, a, b, *, quad="gc", coef_grad=True, info=None, variant="auto", fac=None, chunk=0):
    """lambda = H^{-T} gbar, grad_a = -Re(lambda^H A u), grad_b = -Re(lambda^H B u).

    With fac (from biharmonic_factor, same a, b, quad, chunk) the restart states are taken from it."""
    gbar = _rows(gbar, "gbar")
    N = gbar.shape[-1]
    lead = gbar.shape[:-1]
    a = _coef(a, lead, gbar.device, "a")
    b = _coef(b, lead, gbar.device, "b")
    lam = torch.empty_like(gbar)
    ga = torch.empty(lead, dtype=torch.float64, device=gbar.device) if coef_grad else None
    gb = torch.empty(lead, dtype=torch.float64, device=gbar.device) if coef_grad else None
    if coef_grad:
        u = _like(u, gbar, "u")
    inf = _info_tensor(info, lead, gbar.device)
    o = _opts(gbar.device, quad=quad, info=inf, variant=variant, chunk=chunk)
    up = u.data_ptr() if coef_grad else None
    gap = ga.data_ptr() if ga is not None else None
    gbp = gb.data_ptr() if gb is not None else None
    if fac is not None:
        facd, _, _ = _check_fac(fac, "biharmonic", N, lead, gbar.device, quad, chunk)
        L.check(L.lib().biharmonic_adjoint_factored(N, _nsys(lead), a.data_ptr(), b.data_ptr(), facd.data_ptr(), up,
                                                    gbar.data_ptr(), lam.data_ptr(), gap, gbp, C.byref(o)),
                "biharmonic_adjoint_factored")
    else:
        L.check(L.lib().biharmonic_adjoint(N, _nsys(lead), a.data_ptr(), b.data_ptr(), up, gbar.data_ptr(), lam.data_ptr(),
                                           gap, gbp, C.byref(o)), "biharmonic_adjoint")
    return (lam, ga, gb, inf) if inf is not None else (lam, ga, gb)


# --------------------------------------------------------------------------
# autograd
# --------------------------------------------------------------------------

def _factor_if_wave(family, N, make):
    """The factor-once states when the one-wavefront kernels cover N (their adjoint reuses them),
    else None (the solves then walk themselves)."""
    fam = L.SHEN_HELMHOLTZ if family == "helmholtz" else L.SHEN_BIHARMONIC
    c, g = C.c_int32(0), C.c_int32(0)
    if L.lib().shen_wave_config(fam, int(N), 0, C.byref(c), C.byref(g)) != L.SHEN_OK:
        return None
    return make()


class HelmholtzSolve(torch.autograd.Function):
    """u = (S + alpha B)^{-1} f with a hand-written adjoint:
    grad_f = H^{-T} grad_u, grad_alpha = -Re(grad_f^H B u)."""

    @staticmethod
    def forward(ctx, f, alpha, quad="gc"):
        f, alpha = f.contiguous(), alpha.contiguous()
        fac = _factor_if_wave("helmholtz", f.shape[-1], lambda: helmholtz_factor(alpha, f.shape[-1], quad=quad))
        if fac is not None:  # factor once for the forward solve and the backward pass
            u = helmholtz_solve_factored(f, alpha, fac, quad=quad)
        else:
            u = helmholtz_solve(f, alpha, quad=quad)
        ctx.save_for_backward(u, alpha)
        ctx.fac = fac
        ctx.quad = quad
        return u

    @staticmethod
    def backward(ctx, gu):
        u, alpha = ctx.saved_tensors
        need_c = ctx.needs_input_grad[1]
        lam, ga = helmholtz_adjoint(u, gu.contiguous(), alpha, quad=ctx.quad, coef_grad=need_c, fac=ctx.fac)
        return (lam if ctx.needs_input_grad[0] else None), (ga if need_c else None), None


class BiharmonicSolve(torch.autograd.Function):
    """u = (Q + a A + b B)^{-1} f with a hand-written adjoint:
    grad_f = H^{-T} grad_u, grad_a = -Re(grad_f^H A u), grad_b = -Re(grad_f^H B u)."""

    @staticmethod
    def forward(ctx, f, a, b, quad="gc"):
        f, a, b = f.contiguous(), a.contiguous(), b.contiguous()
        fac = _factor_if_wave("biharmonic", f.shape[-1], lambda: biharmonic_factor(a, b, f.shape[-1], quad=quad))
        if fac is not None:  # factor once for the forward solve and the backward pass
            u = biharmonic_solve_factored(f, a, b, fac, quad=quad)
        else:
            u = biharmonic_solve(f, a, b, quad=quad)
        ctx.save_for_backward(u, a, b)
        ctx.fac = fac
        ctx.quad = quad
        return u

    @staticmethod
    def backward(ctx, gu):
        u, a, b = ctx.saved_tensors
        need_c = ctx.needs_input_grad[1] or ctx.needs_input_grad[2]
        lam, ga, gb = biharmonic_adjoint(u, gu.contiguous(), a, b, quad=ctx.quad, coef_grad=need_c, fac=ctx.fac)
        return ((lam if ctx.needs_input_grad[0] else None), (ga if ctx.needs_input_grad[1] else None),
                (gb if ctx.needs_input_grad[2] else None), None)


def helmholtz(f, alpha, quad="gc"):
    """Differentiable Helmholtz solve (torch.autograd)."""
    return HelmholtzSolve.apply(f, alpha, quad)


def biharmonic(f, a, b, quad="gc"):
    """Differentiable biharmonic solve (torch.autograd)."""
    return BiharmonicSolve.apply(f, a, b, quad)
