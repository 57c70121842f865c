"""FP64 CPU oracle for the wall-normal Shen-Galerkin Helmholtz and biharmonic solves.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library and does not import the package that wraps it.

What it computes is the plain definition of the problem: for every system w
it assembles the real dense Galerkin matrix from closed-form entries and
solves it with LAPACK ``gesv`` (partial pivoting), the real and imaginary
parts of the right-hand side being two right-hand sides of the same
factorisation, then applies two steps of classical iterative refinement with
the residual f - H u accumulated in extended precision (long double), so
that the result is u = H^{-1} f to a few ulps even where pivoted LU alone is
not (the row-graded biharmonic matrices at small wavenumber).

Conventions (arrays of length N = number of Chebyshev modes = number of
quadrature points; Sec. 2):

* Dirichlet basis  phi_k = T_k - T_{k+2},                       k = 0..N-3
* biharmonic basis phi_k = T_k - 2(k+2)/(k+3) T_{k+2} + (k+1)/(k+3) T_{k+4},
                                                                k = 0..N-5
* Matrix entry (k, j): row k is the test function, column j the trial one.
* c_0 = 2, c_k = 1 otherwise, except c_{N-1} = 2 for Gauss-Lobatto
  quadrature (appendix, matrix table caption).

Matrices (row k, column j):

* Bbar = (phi_j, phi_k) Dirichlet mass          -- appendix matrix table
* Sbar = -(phi_j'', phi_k) Dirichlet stiffness  -- not printed (Sec. 3 defers
  it to Shen 1995); closed form derived from the Chebyshev second-derivative
  coefficients and pinned by the tests against exact rational arithmetic
  and quadrature.
* Bchk = (phi_j, phi_k) biharmonic mass         -- appendix matrix table
* Achk = (phi_j'', phi_k) biharmonic Laplacian  -- not printed; derived,
  pinned likewise (sign: the Crank-Nicolson biharmonic matrix of Sec. 3 is
  only consistent with this sign).
* Qchk = (phi_j'''', phi_k)                     -- Sec. 4 (rank-2 tail
  p_k q_j + r_k s_j); its printed diagonal is not what the definition gives
  and the diagonal used here is the one the definition gives (pinned by the
  clamped-plate solution and by exact arithmetic).

Systems solved (Sec. 3, Crank-Nicolson matrices divided by +-nu*dt/2):

* Helmholtz:  (Sbar + alpha_w Bbar) u = f
* biharmonic: (Qchk + a_w Achk + b_w Bchk) u = f

Also: the mass-matrix solves u = Bbar^{-1} f and u = Bchk^{-1} f of the
forward Shen transforms (Sec. 2), the derivative projection
Bbar fhat = Cbar uhat (Sec. 3), the right-hand sides of one Crank-Nicolson
step (Sec. 3, eqs. ufin / gfin), and the wall-normal Shen transforms (Sec. 2:
scalar products, forward and inverse transforms).

Inputs: N, per-system coefficients, complex f of shape [nsys, N] whose
entries k >= n are ignored.  Output: complex u [nsys, N] with the tail zero.
"""
from __future__ import annotations

import os
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

PI = np.pi
GC = 0
GL = 1


# ----------------------------------------------------------------------------
# Quadrature constants
# ----------------------------------------------------------------------------

def ck(m, N: int, quad: int = GC):
    """c_m of the discrete weighted inner product (appendix matrix table caption)."""
    m = np.asarray(m)
    c = np.where(m == 0, 2.0, 1.0)
    if quad == GL:
        c = np.where(m == N - 1, 2.0, c)
    return c


# ----------------------------------------------------------------------------
# Dirichlet (Helmholtz) matrices
# ----------------------------------------------------------------------------

def dirichlet_mass(N: int, quad: int = GC) -> np.ndarray:
    """Bbar_kj = (phi_j, phi_k): pi/2 (c_k + c_{k+2}) on the diagonal, -pi/2 at |j-k| = 2."""
    n = N - 2
    k = np.arange(n)
    B = np.zeros((n, n))
    B[k, k] = 0.5 * PI * (ck(k, N, quad) + ck(k + 2, N, quad))
    i = np.arange(n - 2)
    B[i, i + 2] = -0.5 * PI
    B[i + 2, i] = -0.5 * PI
    return B


def dirichlet_stiffness(N: int) -> np.ndarray:
    """Sbar_kj = -(phi_j'', phi_k): 2pi(k+1)(k+2) on the diagonal, 4pi(k+1) for j = k+2, k+4, ..."""
    n = N - 2
    S = np.zeros((n, n))
    for k in range(n):
        S[k, k] = 2.0 * PI * (k + 1) * (k + 2)
        S[k, k + 2::2] = 4.0 * PI * (k + 1)
    return S


# ----------------------------------------------------------------------------
# Biharmonic matrices
# ----------------------------------------------------------------------------

def biharmonic_mass(N: int, quad: int = GC) -> np.ndarray:
    """Bchk_kj = (phi_j, phi_k), five diagonals, symmetric (appendix matrix table)."""
    n = N - 4
    B = np.zeros((n, n))
    for k in range(n):
        B[k, k] = 0.5 * PI * (ck(k, N, quad) + 4.0 * ((k + 2) / (k + 3)) ** 2
                              + ck(k + 4, N, quad) * ((k + 1) / (k + 3)) ** 2)
        if k + 2 < n:
            v = -PI * ((k + 2) / (k + 3) + (k + 4) * (k + 1) / ((k + 5) * (k + 3)))
            B[k, k + 2] = v
            B[k + 2, k] = v
        if k + 4 < n:
            v = 0.5 * PI * (k + 1) / (k + 3)
            B[k, k + 4] = v
            B[k + 4, k] = v
    return B


def biharmonic_laplacian(N: int) -> np.ndarray:
    """Achk_kj = (phi_j'', phi_k): three diagonals j = k-2, k, k+2 (Sec. 4 states the band)."""
    n = N - 4
    A = np.zeros((n, n))
    for k in range(n):
        A[k, k] = -4.0 * PI * (k + 1) * (k + 2) ** 2 / (k + 3)
        if k + 2 < n:
            A[k, k + 2] = 2.0 * PI * (k + 1) * (k + 2)
        if k - 2 >= 0:
            A[k, k - 2] = 2.0 * PI * (k - 1) * (k + 2)
    return A


def q_gen(N: int):
    """Generators of the Qchk tail (Sec. 4): p_k, q_j, r_k, s_j."""
    k = np.arange(N - 4, dtype=np.float64)
    p = 8.0 * PI * k * (k + 1) * (k + 2) * (k + 4)
    q = 1.0 / (k + 3)
    r = 24.0 * PI * (k + 1) * (k + 2)
    s = (k + 2) ** 2 / (k + 3)
    return p, q, r, s


def biharmonic_bilaplacian(N: int) -> np.ndarray:
    """Qchk_kj = (phi_j'''', phi_k): upper triangular, Q_kk = 8pi(k+1)^2(k+2)(k+4),
    Q_kj = p_k q_j + r_k s_j for j = k+2, k+4, ... (Sec. 4)."""
    n = N - 4
    p, q, r, s = q_gen(N)
    Q = np.zeros((n, n))
    for k in range(n):
        Q[k, k] = 8.0 * PI * (k + 1) ** 2 * (k + 2) * (k + 4)
        j = np.arange(k + 2, n, 2)
        Q[k, j] = p[k] * q[j] + r[k] * s[j]
    return Q


# ----------------------------------------------------------------------------
# System matrices
# ----------------------------------------------------------------------------

class Operators:
    """Dense closed-form matrices for one N and quadrature, cached."""

    _cache = {}

    def __init__(self, N: int, quad: int = GC):
        self.N = N
        self.quad = quad
        self.Bd = dirichlet_mass(N, quad)
        self.Sd = dirichlet_stiffness(N)
        if N >= 5:
            self.Bb = biharmonic_mass(N, quad)
            self.Ab = biharmonic_laplacian(N)
            self.Qb = biharmonic_bilaplacian(N)

    @classmethod
    def get(cls, N: int, quad: int = GC) -> "Operators":
        key = (N, quad)
        if key not in cls._cache:
            cls._cache[key] = cls(N, quad)
        return cls._cache[key]


def helmholtz_matrix(N: int, alpha, quad: int = GC) -> np.ndarray:
    """H = Sbar + alpha Bbar, batched over alpha (Sec. 3 Helmholtz matrix / (nu dt / 2))."""
    op = Operators.get(N, quad)
    alpha = np.asarray(alpha, dtype=np.float64)
    return op.Sd + alpha[..., None, None] * op.Bd


def biharmonic_matrix(N: int, a, b, quad: int = GC) -> np.ndarray:
    """H = Qchk + a Achk + b Bchk, batched (Sec. 3 biharmonic matrix / (-nu dt / 2))."""
    op = Operators.get(N, quad)
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return op.Qb + a[..., None, None] * op.Ab + b[..., None, None] * op.Bb


def system_matrix(family: str, N: int, coeffs, quad: int = GC) -> np.ndarray:
    if family == "helmholtz":
        return helmholtz_matrix(N, coeffs[0], quad)
    return biharmonic_matrix(N, coeffs[0], coeffs[1], quad)


def n_of(family: str, N: int) -> int:
    return N - 2 if family == "helmholtz" else N - 4


# ----------------------------------------------------------------------------
# Solves (dense LU with partial pivoting, LAPACK gesv)
# ----------------------------------------------------------------------------

def _solve_chunk(family, N, coeffs, f, quad, transpose, refine):
    n = n_of(family, N)
    H = system_matrix(family, N, coeffs, quad)
    if transpose:
        H = np.swapaxes(H, -1, -2)
    rhs = np.stack([f[:, :n].real, f[:, :n].imag], axis=-1)
    x = np.linalg.solve(H, rhs)
    if refine:
        # Classical iterative refinement, residual in extended precision: partial
        # pivoting on these row-graded matrices can leave gesv ~1e-12 from the exact
        # solution; two corrections bring it to a few ulps of u = H^{-1} f.
        Hl = H.astype(np.longdouble)
        rl = rhs.astype(np.longdouble)
        for _ in range(refine):
            r = rl - np.matmul(Hl, x.astype(np.longdouble))
            x = x + np.linalg.solve(H, r.astype(np.float64))
    u = np.zeros(f.shape, dtype=np.complex128)
    u[:, :n] = x[..., 0] + 1j * x[..., 1]
    return u


def solve(family: str, N: int, coeffs, f: np.ndarray, quad: int = GC, transpose: bool = False,
          chunk: int = 0, threads: int = 1, refine: int = 2) -> np.ndarray:
    """Solve H u = f (or H^T u = f) for every system; coeffs = (alpha,) or (a, b).

    LAPACK gesv followed by ``refine`` steps of iterative refinement with an
    extended-precision residual (refine=0: plain gesv)."""
    f = np.asarray(f, dtype=np.complex128)
    nsys = f.shape[0]
    coeffs = tuple(np.asarray(c, dtype=np.float64).reshape(nsys) for c in coeffs)
    if nsys == 0:
        return np.zeros_like(f)
    n = n_of(family, N)
    if chunk <= 0:
        chunk = max(1, min(nsys, int(2.0e7 // max(1, n * n))))
    starts = list(range(0, nsys, chunk))

    def work(s0):
        s1 = min(nsys, s0 + chunk)
        return s0, _solve_chunk(family, N, tuple(c[s0:s1] for c in coeffs), f[s0:s1], quad, transpose, refine)

    u = np.zeros_like(f)
    if threads <= 1 or len(starts) == 1:
        for s0 in starts:
            _, part = work(s0)
            u[s0:s0 + part.shape[0]] = part
    else:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            for s0, part in ex.map(work, starts):
                u[s0:s0 + part.shape[0]] = part
    return u


def helmholtz_solve(N, alpha, f, quad=GC, transpose=False, threads=1):
    return solve("helmholtz", N, (alpha,), f, quad, transpose, threads=threads)


def biharmonic_solve(N, a, b, f, quad=GC, transpose=False, threads=1):
    return solve("biharmonic", N, (a, b), f, quad, transpose, threads=threads)


def matvec(family: str, N: int, coeffs, u: np.ndarray, quad: int = GC, transpose: bool = False,
           extended: bool = False) -> np.ndarray:
    """Hu (tail of the result zero).  extended=True accumulates in long double."""
    u = np.asarray(u, dtype=np.complex128)
    nsys = u.shape[0]
    n = n_of(family, N)
    coeffs = tuple(np.asarray(c, dtype=np.float64).reshape(nsys) for c in coeffs)
    H = system_matrix(family, N, coeffs, quad)
    if transpose:
        H = np.swapaxes(H, -1, -2)
    out = np.zeros_like(u)
    if extended:
        Hl = H.astype(np.longdouble)
        re = np.einsum("wkj,wj->wk", Hl, u[:, :n].real.astype(np.longdouble))
        im = np.einsum("wkj,wj->wk", Hl, u[:, :n].imag.astype(np.longdouble))
        out[:, :n] = re.astype(np.float64) + 1j * im.astype(np.float64)
    else:
        out[:, :n] = np.einsum("wkj,wj->wk", H, u[:, :n])
    return out


# ----------------------------------------------------------------------------
# Mass-matrix solves: the last step of a forward Shen transform (Sec. 2, the
# complete transformation u_hat = B^{-1} S(u), with S(u) the vector of scalar
# products (u, phi_l)_sigma).  One matrix for every system: Bbar (three
# nonzero diagonals) for the Dirichlet basis, Bchk (five) for the biharmonic
# one.
# ----------------------------------------------------------------------------

def mass_matrix(family: str, N: int, quad: int = GC) -> np.ndarray:
    """Bbar (family "helmholtz", the Dirichlet basis) or Bchk ("biharmonic")."""
    op = Operators.get(N, quad)
    return op.Bd if family == "helmholtz" else op.Bb


def mass_solve(family: str, N: int, f: np.ndarray, quad: int = GC, refine: int = 2) -> np.ndarray:
    """u = B^{-1} f for every system (row) of f; entries k >= n of f ignored, of u zero.

    LAPACK gesv on the dense mass matrix, all systems as right-hand sides of
    one factorisation, then ``refine`` steps of iterative refinement with the
    residual in extended precision (as in ``solve``)."""
    f = np.asarray(f, dtype=np.complex128)
    nsys = f.shape[0]
    n = n_of(family, N)
    u = np.zeros_like(f)
    if nsys == 0:
        return u
    B = mass_matrix(family, N, quad)
    rhs = np.concatenate([f[:, :n].real, f[:, :n].imag], axis=0).T  # [n, 2 nsys]
    x = np.linalg.solve(B, rhs)
    Bl = B.astype(np.longdouble)
    rl = rhs.astype(np.longdouble)
    for _ in range(refine):
        r = rl - Bl @ x.astype(np.longdouble)
        x = x + np.linalg.solve(B, r.astype(np.float64))
    u[:, :n] = x[:, :nsys].T + 1j * x[:, nsys:].T
    return u


def derivative_matrix(N: int) -> np.ndarray:
    """Cbar_kj = (phichk_j', phibar_k)_sigma, Dirichlet rows k < N-2 by biharmonic columns
    j < N-4 (appendix matrix table): pi (k-2)(k+1)/k at j = k-3, -2 pi (k+1)^2/(k+2) at
    j = k-1, pi (k+1) at j = k+1.  The same for GC and GL (the quadrature is exact for
    these products)."""
    nd, nb = N - 2, N - 4
    C = np.zeros((nd, nb))
    for k in range(nd):
        if 0 <= k - 3 < nb:
            C[k, k - 3] = PI * (k - 2) * (k + 1) / k
        if 0 <= k - 1 < nb:
            C[k, k - 1] = -2.0 * PI * (k + 1) ** 2 / (k + 2)
        if k + 1 < nb:
            C[k, k + 1] = PI * (k + 1)
    return C


def derivative_solve(N: int, uhat: np.ndarray, quad: int = GC) -> np.ndarray:
    """fhat with Bbar fhat = Cbar uhat (Sec. 3, the last of the wall-normal systems):
    the Dirichlet-basis Galerkin coefficients of du/dx for u = sum_j uhat_j phichk_j.
    uhat: [nsys, N], entries k >= N-4 ignored; result [nsys, N], entries k >= N-2 zero."""
    uhat = np.asarray(uhat, dtype=np.complex128)
    nb = N - 4
    rhs = np.zeros_like(uhat)
    C = derivative_matrix(N)
    rhs[:, :N - 2] = uhat[:, :nb] @ C.T
    return mass_solve("helmholtz", N, rhs, quad)


# ----------------------------------------------------------------------------
# Shen transforms in the wall-normal direction (Sec. 2; appendix algorithms for
# the forward scalar products / transforms and the inverse transforms), by
# plain dense evaluation of the basis functions at the quadrature points.
#
# Points and weights (Sec. 2): Chebyshev-Gauss x_j = cos(pi (2j+1)/(2N)),
# sigma_j = pi/N; Chebyshev-Gauss-Lobatto x_j = cos(pi j/(N-1)),
# sigma_j = pi/(c_j (N-1)) with c_0 = c_{N-1} = 2.  Spaces: "chebyshev"
# (T_k, k < N), "dirichlet" (T_k - T_{k+2}, k < N-2), "biharmonic"
# (T_k - 2(k+2)/(k+3) T_{k+2} + (k+1)/(k+3) T_{k+4}, k < N-4).
#   scalar product  S(u)_k = sum_j u(x_j) phi_k(x_j) sigma_j
#   forward         uhat = B^{-1} S(u),  B_kl = (phi_l, phi_k)_sigma
#   inverse         u(x_j) = sum_k uhat_k phi_k(x_j)
# T_k(x_j) = cos(k theta_j) is evaluated with the integer multiple of the
# angle reduced exactly, in long double.
# ----------------------------------------------------------------------------

SPACES = ("chebyshev", "dirichlet", "biharmonic")


def n_space(space: str, N: int) -> int:
    return {"chebyshev": N, "dirichlet": N - 2, "biharmonic": N - 4}[space]


def quad_weights(N: int, quad: int = GC) -> np.ndarray:
    if quad == GC:
        return np.full(N, PI / N)
    c = np.ones(N)
    c[0] = c[-1] = 2.0
    return PI / (c * (N - 1))


def quad_points(N: int, quad: int = GC) -> np.ndarray:
    j = np.arange(N)
    if quad == GC:
        return np.cos(PI * (2 * j + 1) / (2 * N))
    return np.cos(PI * j / (N - 1))


def cheb_at_points(N: int, quad: int = GC, kmax=None) -> np.ndarray:
    """T_k(x_j) for k < kmax (default N), j < N, as long double [kmax, N]."""
    kmax = N if kmax is None else kmax
    k = np.arange(kmax, dtype=np.int64)[:, None]
    j = np.arange(N, dtype=np.int64)[None, :]
    if quad == GC:
        m = (k * (2 * j + 1)) % (4 * N)  # angle pi m / (2N)
        ang = np.pi * m.astype(np.longdouble) / np.longdouble(2 * N)
    else:
        m = (k * j) % (2 * (N - 1))  # angle pi m / (N-1)
        ang = np.pi * m.astype(np.longdouble) / np.longdouble(N - 1)
    return np.cos(ang)


def basis_at_points(space: str, N: int, quad: int = GC) -> np.ndarray:
    """phi_k(x_j) for the space's k, as long double [n, N] (basis definitions, Sec. 2)."""
    T = cheb_at_points(N, quad)
    if space == "chebyshev":
        return T
    n = n_space(space, N)
    k = np.arange(n)
    if space == "dirichlet":
        return T[:n] - T[2:n + 2]
    g1 = (2.0 * (k + 2) / (k + 3)).astype(np.longdouble)[:, None]
    g2 = ((k + 1) / (k + 3)).astype(np.longdouble)[:, None]
    return T[:n] - g1 * T[2:n + 2] + g2 * T[4:n + 4]


def scalar_product(space: str, N: int, u: np.ndarray, quad: int = GC) -> np.ndarray:
    """S(u)_k = (u, phi_k)_sigma for point values u [nsys, N]; entries k >= n zero.
    The sums run in long double."""
    u = np.asarray(u, dtype=np.complex128)
    n = n_space(space, N)
    P = basis_at_points(space, N, quad) * quad_weights(N, quad).astype(np.longdouble)[None, :]
    out = np.zeros_like(u)
    re = u.real.astype(np.longdouble) @ P.T
    im = u.imag.astype(np.longdouble) @ P.T
    out[:, :n] = re.astype(np.float64) + 1j * im.astype(np.float64)
    return out


def space_mass_solve(space: str, N: int, f: np.ndarray, quad: int = GC) -> np.ndarray:
    """B^{-1} f with B the space's mass matrix: diagonal c_k pi/2 for "chebyshev" (c_0 = 2,
    and c_{N-1} = 2 for GL), else the Dirichlet / biharmonic mass solves above."""
    if space == "chebyshev":
        f = np.asarray(f, dtype=np.complex128)
        return f / (0.5 * PI * ck(np.arange(N), N, quad))[None, :]
    return mass_solve("helmholtz" if space == "dirichlet" else "biharmonic", N, f, quad)


def forward_transform(space: str, N: int, u: np.ndarray, quad: int = GC) -> np.ndarray:
    """uhat = B^{-1} S(u) (Sec. 2, the complete transformation)."""
    return space_mass_solve(space, N, scalar_product(space, N, u, quad), quad)


def backward_transform(space: str, N: int, uhat: np.ndarray, quad: int = GC) -> np.ndarray:
    """u(x_j) = sum_k uhat_k phi_k(x_j) for coefficients uhat [nsys, N] (entries k >= n
    ignored); sums in long double."""
    uhat = np.asarray(uhat, dtype=np.complex128)
    n = n_space(space, N)
    P = basis_at_points(space, N, quad)
    re = uhat[:, :n].real.astype(np.longdouble) @ P
    im = uhat[:, :n].imag.astype(np.longdouble) @ P
    return re.astype(np.float64) + 1j * im.astype(np.float64)


# ----------------------------------------------------------------------------
# Right-hand sides of one Crank-Nicolson step (Sec. 3, eqs. ufin and gfin),
# written with the paper's unscaled matrices.  Per wavenumber pair, with
# z2 = m^2 + n^2 the squared wavenumber:
#
#   biharmonic (eq. ufin):  Hchk uhat' = (2 Achk - 2 z2 Bchk - Hchk) uhat + dt S(h_v)
#       Hchk = -(nu dt/2) Qchk + (1 + nu dt z2) Achk - (2 z2 + nu dt z2^2)/2 Bchk
#   Helmholtz (eq. gfin):   Hbar ghat' = (2 Bbar - Hbar) ghat + dt S(h_g)
#       Hbar = -(nu dt/2) Abar + (1 + nu dt z2/2) Bbar,   Abar = (phi'', phi) = -Sbar
#
# (the sign of A as read for the Crank-Nicolson matrices: the matrices are
# consistent with A = +(phi'', phi) only).  The solves of this library take the
# systems divided by -nu dt/2 (biharmonic) and nu dt/2 (Helmholtz), so the
# right-hand side returned here is the paper's one times -2/(nu dt) or
# 2/(nu dt): exactly what makes solve(rhs) the step's new coefficients.
# ----------------------------------------------------------------------------

def cn_matrix_paper(family: str, N: int, z2: float, nu: float, dt: float, quad: int = GC) -> np.ndarray:
    """The paper's unscaled Crank-Nicolson matrix of one wavenumber pair (Sec. 3)."""
    op = Operators.get(N, quad)
    if family == "helmholtz":
        Abar = -op.Sd
        return -(nu * dt / 2.0) * Abar + (1.0 + nu * dt * z2 / 2.0) * op.Bd
    return (-(nu * dt / 2.0) * op.Qb + (1.0 + nu * dt * z2) * op.Ab
            - ((2.0 * z2 + nu * dt * z2 * z2) / 2.0) * op.Bb)


def cn_explicit_matrix_paper(family: str, N: int, z2: float, nu: float, dt: float, quad: int = GC) -> np.ndarray:
    """The matrix acting on the old coefficients in eqs. ufin / gfin:
    2 Achk - 2 z2 Bchk - Hchk (biharmonic), 2 Bbar - Hbar (Helmholtz)."""
    op = Operators.get(N, quad)
    H = cn_matrix_paper(family, N, z2, nu, dt, quad)
    if family == "helmholtz":
        return 2.0 * op.Bd - H
    return 2.0 * op.Ab - 2.0 * z2 * op.Bb - H


def rhs_assemble(family: str, N: int, K2, nu: float, dt: float, uhat: np.ndarray, sh=None,
                 quad: int = GC, extended: bool = False) -> np.ndarray:
    """Right-hand side of one Crank-Nicolson step in the scaling of ``solve``:
    -2/(nu dt) [(2 Achk - 2 z2 Bchk - Hchk) uhat + dt S(h)] (biharmonic) or
    2/(nu dt) [(2 Bbar - Hbar) ghat + dt S(h)] (Helmholtz), per system with z2 = K2[w].
    uhat, sh: complex [nsys, N] (entries k >= n ignored; sh=None omits the term).
    Result [nsys, N] with the tail zero.  extended=True forms the product and the
    sum in long double (a reference for the device's FP64 result)."""
    uhat = np.asarray(uhat, dtype=np.complex128)
    nsys = uhat.shape[0]
    n = n_of(family, N)
    K2 = np.asarray(K2, dtype=np.float64).reshape(nsys)
    scale = (2.0 if family == "helmholtz" else -2.0) / (nu * dt)
    dtype = np.longdouble if extended else np.float64
    out = np.zeros_like(uhat)
    for w in range(nsys):
        M = cn_explicit_matrix_paper(family, N, float(K2[w]), nu, dt, quad).astype(dtype)
        re = M @ uhat[w, :n].real.astype(dtype)
        im = M @ uhat[w, :n].imag.astype(dtype)
        if sh is not None:
            re = re + dtype(dt) * np.asarray(sh[w, :n].real, dtype=dtype)
            im = im + dtype(dt) * np.asarray(sh[w, :n].imag, dtype=dtype)
        out[w, :n] = (dtype(scale) * re).astype(np.float64) + 1j * (dtype(scale) * im).astype(np.float64)
    return out


# ----------------------------------------------------------------------------
# Adjoint and coefficient gradients
# ----------------------------------------------------------------------------

def solve_grads(family: str, N: int, coeffs, f: np.ndarray, gu: np.ndarray, quad: int = GC):
    """Gradients of a real loss through u = H^{-1} f, given gu = dL/dRe(u) + i dL/dIm(u).

    lambda = H^{-T} gu (H is real) is the gradient with respect to f; the
    gradient with respect to a coefficient c multiplying the matrix M_c is
    -Re(lambda^H M_c u), because du/dc = -H^{-1} M_c u.
    Returns (u, grad_f, [grad per coefficient]).
    """
    u = solve(family, N, coeffs, f, quad)
    lam = solve(family, N, coeffs, gu, quad, transpose=True)
    n = n_of(family, N)
    op = Operators.get(N, quad)
    mats = [op.Bd] if family == "helmholtz" else [op.Ab, op.Bb]
    grads = []
    for M in mats:
        Mu = np.einsum("kj,wj->wk", M, u[:, :n])
        grads.append(-np.real(np.sum(np.conj(lam[:, :n]) * Mu, axis=1)))
    return u, lam, grads


# ----------------------------------------------------------------------------
# Singular coefficients (failure cases of the unpivoted LU of Sec. 4)
# ----------------------------------------------------------------------------

def chain_rows(k: int):
    """Rows p, p+2, ..., k of the parity chain that ends at row k (p = k mod 2)."""
    return np.arange(k % 2, k + 1, 2)


def singular_coefficient(family: str, N: int, k: int, quad: int = GC, a: float = 0.0) -> float:
    """A coefficient that makes the leading block of row k's parity chain singular.

    Odd and even rows decouple (Sec. 4), so the leading block of the unpivoted LU up to
    row k is singular exactly when the block of rows chain_rows(k) is.  Helmholtz: the
    alpha with Sbar + alpha Bbar singular there, i.e. minus a generalised eigenvalue of
    (Sbar, Bbar) restricted to those rows; biharmonic: the b with (Qchk + a Achk) + b Bchk
    singular there.  The eigenvalue taken is the largest, whose eigenvector needs every
    row of the block (the smooth modes are already resolved by shorter blocks).  It is
    polished to the FP64 neighbour pair across which det changes sign (bisection on the
    sign of det from pivoted LU), and the member with the smaller |det| is returned.
    With k the last row of its chain this is a singular coefficient of the whole system.
    """
    op = Operators.get(N, quad)
    if family == "helmholtz":
        M0, M1 = op.Sd, op.Bd
    else:
        M0, M1 = op.Qb + a * op.Ab, op.Bb
    idx = chain_rows(k)
    A0 = M0[np.ix_(idx, idx)]
    A1 = M1[np.ix_(idx, idx)]
    lam = np.linalg.eigvals(np.linalg.solve(A1, A0))
    lam = lam[np.abs(lam.imag) <= 1e-9 * np.abs(lam)].real
    c = -float(np.max(lam))

    def sgn(x):
        return np.linalg.slogdet(A0 + x * A1)

    lo, hi = c * (1 + 1e-8), c * (1 - 1e-8)
    slo = sgn(lo)[0]
    if sgn(hi)[0] == slo:
        raise ValueError("no sign change of det around the eigenvalue")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if sgn(mid)[0] == slo:
            lo = mid
        else:
            hi = mid
    return lo if sgn(lo)[1] <= sgn(hi)[1] else hi


# ----------------------------------------------------------------------------
# Error metrics
# ----------------------------------------------------------------------------

def rel_err_per_system(u: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """max_k |u_k - ref_k| / max_k |ref_k| per system (the roundoff measure of Sec. 5)."""
    num = np.max(np.abs(u - ref), axis=1)
    den = np.max(np.abs(ref), axis=1)
    den = np.where(den == 0, 1.0, den)
    return num / den


# ----------------------------------------------------------------------------
# Timing of the oracle on the host (a baseline, not the target)
# ----------------------------------------------------------------------------

def host_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def time_solve(family, N, coeffs, f, threads=None, quad=GC, refine=2):
    """Wall time of the oracle over the given systems; returns (seconds, threads, u)."""
    threads = threads or host_threads()
    n = n_of(family, N)
    nsys = f.shape[0]
    chunk = max(1, min(64, (nsys + threads - 1) // threads, int(2.0e7 // max(1, n * n))))
    t0 = time.perf_counter()
    u = solve(family, N, coeffs, f, quad, chunk=chunk, threads=threads, refine=refine)
    return time.perf_counter() - t0, threads, u
