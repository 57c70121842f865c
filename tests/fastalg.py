"""NumPy prototype of the O(N) direct solvers (tests only; never imported by the library).

Vectorised over systems, sequential over the wall-normal index k, written
from Sec. 4: the Helmholtz LU per odd/even chain with a constant tail in U,
and the biharmonic LU (Alg. LUbiharmonic / ReduceAB / LUSolveBiharmonic) in
the compact form that keeps only the rows k-2 and k-4 of U, whose tail is
P_k q_j + R_k s_j.  Also the transposed solves, the O(N) matvec, and the
FP32-solve / FP64-residual refinement.  It is checked against the oracle and
documents, step by step, the recurrences the HIP kernels implement.
"""
import numpy as np

PI = np.pi


def _c(k, N, gl):
    c = np.where(k == 0, 2.0, 1.0)
    if gl:
        c = np.where(k == N - 1, 2.0, c)
    return c


# ------------------------------- Helmholtz ---------------------------------

def helm_entries(k, alpha, N, gl=False, dt=np.float64):
    """Row k of S + alpha B: (H_{k,k-2}, H_kk, H_{k,k+2}, H_{k,j>=k+4})."""
    alpha = alpha.astype(dt)
    pi = dt(PI)
    hm = -alpha * (pi / 2)
    h0 = dt(2) * pi * dt((k + 1) * (k + 2)) + alpha * (pi / 2) * dt(_c(k, N, gl) + _c(k + 2, N, gl))
    hpp = dt(4) * pi * dt(k + 1)
    hp = hpp - alpha * (pi / 2)
    return hm, h0, hp, hpp


def helm_factor_forward(alpha, f, N, gl=False, dt=np.float64):
    """LU factors (l, d, e, g) per row and y = L^{-1} f."""
    n = N - 2
    ns = alpha.shape[0]
    d = np.zeros((ns, n), dt); e = np.zeros((ns, n), dt); g = np.zeros((ns, n), dt); l = np.zeros((ns, n), dt)
    cdt = np.complex128 if dt == np.float64 else np.complex64
    y = np.zeros((ns, n), cdt)
    for k in range(n):
        hm, h0, hp, hpp = helm_entries(k, alpha, N, gl, dt)
        if k < 2:
            d[:, k], e[:, k], g[:, k] = h0, hp, hpp
            y[:, k] = f[:, k]
        else:
            lk = hm / d[:, k - 2]
            l[:, k] = lk
            d[:, k] = h0 - lk * e[:, k - 2]
            e[:, k] = hp - lk * g[:, k - 2]
            g[:, k] = hpp - lk * g[:, k - 2]
            y[:, k] = f[:, k] - lk * y[:, k - 2]
    return l, d, e, g, y


def helm_back(d, e, g, y):
    ns, n = y.shape
    u = np.zeros_like(y)
    S = np.zeros((ns, n + 4), y.dtype)  # S[k] = sum_{j>=k, same parity} u_j
    for k in range(n - 1, -1, -1):
        u2 = u[:, k + 2] if k + 2 < n else 0
        uk = (y[:, k] - e[:, k] * u2 - g[:, k] * S[:, k + 4]) / d[:, k]
        u[:, k] = uk
        S[:, k] = uk + S[:, k + 2]
    return u


def helmholtz_solve(alpha, f, N, gl=False, dt=np.float64):
    n = N - 2
    _, d, e, g, y = helm_factor_forward(alpha, f[:, :n], N, gl, dt)
    out = np.zeros(f.shape, y.dtype)
    out[:, :n] = helm_back(d, e, g, y)
    return out


def helmholtz_solve_T(alpha, gv, N, gl=False):
    """H^T lam = g: U^T z = g forward (prefix sums of g_j z_j), then L^T lam = z backward."""
    n = N - 2
    l, d, e, g, _ = helm_factor_forward(alpha, np.zeros((alpha.shape[0], n), complex), N, gl)
    z = np.zeros((alpha.shape[0], n), complex)
    Z = np.zeros((alpha.shape[0], n + 4), complex)  # Z[k+4] = sum_{j<=k} g_j z_j
    for k in range(n):
        r = gv[:, k].copy()
        if k >= 2:
            r -= e[:, k - 2] * z[:, k - 2]
        r -= Z[:, k]  # j <= k-4
        z[:, k] = r / d[:, k]
        Z[:, k + 4] = Z[:, k + 2] + g[:, k] * z[:, k]
    lam = np.zeros_like(z)
    for k in range(n - 1, -1, -1):
        lam[:, k] = z[:, k] - (l[:, k + 2] * lam[:, k + 2] if k + 2 < n else 0)
    out = np.zeros(gv.shape, complex)
    out[:, :n] = lam
    return out


def helm_matvec(alpha, u, N, gl=False):
    n = N - 2
    ns = alpha.shape[0]
    out = np.zeros(u.shape, complex)
    S = np.zeros((ns, n + 4), complex)
    for k in range(n - 1, -1, -1):
        S[:, k] = u[:, k] + S[:, k + 2]
    for k in range(n):
        hm, h0, hp, hpp = helm_entries(k, alpha, N, gl)
        v = h0 * u[:, k] + hpp * S[:, k + 4]
        if k >= 2:
            v += hm * u[:, k - 2]
        if k + 2 < n:
            v += hp * u[:, k + 2]
        out[:, k] = v
    return out


# ------------------------------- biharmonic --------------------------------

def bih_gen(j, dt=np.float64):
    j = np.asarray(j, dtype=np.float64)
    pi = PI
    p = 8 * pi * j * (j + 1) * (j + 2) * (j + 4)
    q = 1 / (j + 3)
    r = 24 * pi * (j + 1) * (j + 2)
    s = (j + 2) ** 2 / (j + 3)
    return dt(p), dt(q), dt(r), dt(s)


def bih_entries(k, a, b, N, gl=False, dt=np.float64):
    """Row k of Q + a A + b B: (H_{k,k-4}, H_{k,k-2}, H_kk, H_{k,k+2}, H_{k,k+4}) and p_k, r_k."""
    a = a.astype(dt); b = b.astype(dt)
    pi = PI
    kk = float(k)
    B0 = 0.5 * pi * (_c(k, N, gl) + 4 * ((kk + 2) / (kk + 3)) ** 2 + _c(k + 4, N, gl) * ((kk + 1) / (kk + 3)) ** 2)
    B2 = -pi * ((kk + 2) / (kk + 3) + (kk + 4) * (kk + 1) / ((kk + 5) * (kk + 3)))
    B4 = 0.5 * pi * (kk + 1) / (kk + 3)
    Bm2 = -pi * (kk / (kk + 1) + (kk + 2) * (kk - 1) / ((kk + 3) * (kk + 1))) if k >= 2 else 0.0
    Bm4 = 0.5 * pi * (kk - 3) / (kk - 1) if k >= 4 else 0.0
    A0 = -4 * pi * (kk + 1) * (kk + 2) ** 2 / (kk + 3)
    A2 = 2 * pi * (kk + 1) * (kk + 2)
    Am2 = 2 * pi * (kk - 1) * (kk + 2)
    p, _, r, _ = bih_gen(k)
    _, q2, _, s2 = bih_gen(k + 2)
    _, q4, _, s4 = bih_gen(k + 4)
    Q0 = 8 * pi * (kk + 1) ** 2 * (kk + 2) * (kk + 4)
    hm4 = b * dt(Bm4)
    hm2 = a * dt(Am2) + b * dt(Bm2)
    h0 = dt(Q0) + a * dt(A0) + b * dt(B0)
    hp2 = dt(p * q2 + r * s2) + a * dt(A2) + b * dt(B2)
    hp4 = dt(p * q4 + r * s4) + b * dt(B4)
    return hm4, hm2, h0, hp2, hp4, dt(p), dt(r)


def bih_factor_forward(a, b, f, N, gl=False, dt=np.float64):
    """Compact LU rows (U0, U2, U4, P, R), multipliers (L1 = L_{k,k-2}, L2 = L_{k,k-4}), y."""
    n = N - 4
    ns = a.shape[0]
    Z = lambda: np.zeros((ns, n), dt)
    U0, U2, U4, P, R, L1, L2 = Z(), Z(), Z(), Z(), Z(), Z(), Z()
    cdt = np.complex128 if dt == np.float64 else np.complex64
    y = np.zeros((ns, n), cdt)
    for k in range(n):
        hm4, hm2, h0, hp2, hp4, pk, rk = bih_entries(k, a, b, N, gl, dt)
        _, q2, _, s2 = bih_gen(k + 2, dt)
        _, q4, _, s4 = bih_gen(k + 4, dt)
        tm2, t0, t2, t4, Pk, Rk = hm2, h0, hp2, hp4, np.full(ns, pk), np.full(ns, rk)
        yk = f[:, k].astype(cdt)
        if k >= 4:
            l2 = hm4 / U0[:, k - 4]
            L2[:, k] = l2
            tm2 = tm2 - l2 * U2[:, k - 4]
            t0 = t0 - l2 * U4[:, k - 4]
            t2 = t2 - l2 * (P[:, k - 4] * q2 + R[:, k - 4] * s2)
            t4 = t4 - l2 * (P[:, k - 4] * q4 + R[:, k - 4] * s4)
            Pk = Pk - l2 * P[:, k - 4]
            Rk = Rk - l2 * R[:, k - 4]
            yk = yk - l2 * y[:, k - 4]
        if k >= 2:
            l1 = tm2 / U0[:, k - 2]
            L1[:, k] = l1
            t0 = t0 - l1 * U2[:, k - 2]
            t2 = t2 - l1 * U4[:, k - 2]
            t4 = t4 - l1 * (P[:, k - 2] * q4 + R[:, k - 2] * s4)
            Pk = Pk - l1 * P[:, k - 2]
            Rk = Rk - l1 * R[:, k - 2]
            yk = yk - l1 * y[:, k - 2]
        U0[:, k], U2[:, k], U4[:, k], P[:, k], R[:, k] = t0, t2, t4, Pk, Rk
        y[:, k] = yk
    return U0, U2, U4, P, R, L1, L2, y


def bih_back(U0, U2, U4, P, R, y, dt=np.float64):
    ns, n = y.shape
    u = np.zeros_like(y)
    sq = np.zeros((ns, n + 8), y.dtype)  # sq[k] = sum_{j>=k, same parity} q_j u_j
    ss = np.zeros((ns, n + 8), y.dtype)
    for k in range(n - 1, -1, -1):
        v = y[:, k].copy()
        if k + 2 < n:
            v -= U2[:, k] * u[:, k + 2]
        if k + 4 < n:
            v -= U4[:, k] * u[:, k + 4]
        v -= P[:, k] * sq[:, k + 6] + R[:, k] * ss[:, k + 6]
        u[:, k] = v / U0[:, k]
        _, qk, _, sk = bih_gen(k, dt)
        sq[:, k] = qk * u[:, k] + sq[:, k + 2]
        ss[:, k] = sk * u[:, k] + ss[:, k + 2]
    return u


def biharmonic_solve(a, b, f, N, gl=False, dt=np.float64):
    n = N - 4
    U0, U2, U4, P, R, _, _, y = bih_factor_forward(a, b, f[:, :n], N, gl, dt)
    out = np.zeros(f.shape, y.dtype)
    out[:, :n] = bih_back(U0, U2, U4, P, R, y, dt)
    return out


def biharmonic_solve_T(a, b, gv, N, gl=False):
    """U^T z = g forward (prefix sums of P_j z_j and R_j z_j), then L^T lam = z backward."""
    n = N - 4
    ns = a.shape[0]
    U0, U2, U4, P, R, L1, L2, _ = bih_factor_forward(a, b, np.zeros((ns, n), complex), N, gl)
    z = np.zeros((ns, n), complex)
    SP = np.zeros((ns, n + 8), complex)  # SP[k+6] = sum_{j<=k} P_j z_j
    SR = np.zeros((ns, n + 8), complex)
    for k in range(n):
        r = gv[:, k].copy()
        if k >= 2:
            r -= U2[:, k - 2] * z[:, k - 2]
        if k >= 4:
            r -= U4[:, k - 4] * z[:, k - 4]
        _, qk, _, sk = bih_gen(k)
        r -= qk * SP[:, k] + sk * SR[:, k]
        z[:, k] = r / U0[:, k]
        SP[:, k + 6] = SP[:, k + 4] + P[:, k] * z[:, k]
        SR[:, k + 6] = SR[:, k + 4] + R[:, k] * z[:, k]
    lam = np.zeros_like(z)
    for k in range(n - 1, -1, -1):
        v = z[:, k].copy()
        if k + 2 < n:
            v -= L1[:, k + 2] * lam[:, k + 2]
        if k + 4 < n:
            v -= L2[:, k + 4] * lam[:, k + 4]
        lam[:, k] = v
    out = np.zeros(gv.shape, complex)
    out[:, :n] = lam
    return out


def bih_matvec(a, b, u, N, gl=False):
    n = N - 4
    ns = a.shape[0]
    out = np.zeros(u.shape, complex)
    sq = np.zeros((ns, n + 8), complex)
    ss = np.zeros((ns, n + 8), complex)
    for k in range(n - 1, -1, -1):
        _, qk, _, sk = bih_gen(k)
        sq[:, k] = qk * u[:, k] + sq[:, k + 2]
        ss[:, k] = sk * u[:, k] + ss[:, k + 2]
    for k in range(n):
        hm4, hm2, h0, hp2, hp4, pk, rk = bih_entries(k, a, b, N, gl)
        v = h0 * u[:, k] + pk * sq[:, k + 6] + rk * ss[:, k + 6]
        if k >= 2:
            v += hm2 * u[:, k - 2]
        if k >= 4:
            v += hm4 * u[:, k - 4]
        if k + 2 < n:
            v += hp2 * u[:, k + 2]
        if k + 4 < n:
            v += hp4 * u[:, k + 4]
        out[:, k] = v
    return out


# --------------------------- mixed precision --------------------------------

STAG_TOL = 5e-13  # rounding-floor acceptance bound of the kernels' refinement


def refine_solve(family, coeffs, f, N, gl=False, tol=1e-14, it_max=8):
    """u = solve32(f); repeat r = f - H u (FP64), u += solve32(r), with the kernels' stopping
    rule: converged at |du| <= tol |u|; a correction that fails to halve ends the iteration
    (the rounding floor, where the corrections are noise of about the size of the error left)
    and is accepted only when |du| <= max(tol, STAG_TOL) |u|; it_max corrections at most.
    Returns (u, u0 = the uncorrected FP32 solution, corrections applied, converged)."""
    if family == "helmholtz":
        s32 = lambda rhs: helmholtz_solve(coeffs[0], rhs.astype(np.complex64), N, gl, np.float32).astype(np.complex128)
        mv = lambda uu: helm_matvec(coeffs[0], uu, N, gl)
    else:
        s32 = lambda rhs: biharmonic_solve(coeffs[0], coeffs[1], rhs.astype(np.complex64), N, gl, np.float32).astype(np.complex128)
        mv = lambda uu: bih_matvec(coeffs[0], coeffs[1], uu, N, gl)
    u0 = s32(f)
    u = u0.copy()
    ns = f.shape[0]
    iters = np.zeros(ns, int)
    conv = np.zeros(ns, bool)
    active = np.ones(ns, bool)
    prev = np.full(ns, 1e300)
    if it_max == 0:
        return u, u0, iters, np.all(np.isfinite(u0), axis=1)
    for it in range(1, it_max + 1):
        if not active.any():
            break
        r = f - mv(u)
        du = s32(r)
        du[~active] = 0
        u = u + du
        iters += active
        dn = np.max(np.abs(du), axis=1)
        un = np.max(np.abs(u), axis=1)
        bad = ~(dn <= 1e300)
        ok = dn <= tol * un
        stag = ~bad & ~ok & (dn > 0.5 * prev)
        floor = stag & (dn <= max(tol, STAG_TOL) * un)
        conv |= active & (ok | floor)
        act_before = active.copy()
        active &= ~(bad | ok | stag)
        prev = np.where(act_before, dn, prev)
    return u, u0, iters, conv
