"""Pins of the oracle's mass-matrix solves u = B^{-1} f (Sec. 2: the complete forward
transform is u_hat = B^{-1} S(u)).

* exact: the mass matrix from exact rational Chebyshev algebra (chebexact), the
  system solved in rational arithmetic, against the oracle;
* transform round trip: u = sum_q u_hat_q phi_q evaluated at the quadrature points
  with numpy.polynomial, its scalar products S_l(u) = sum_i u(x_i) phi_l(x_i) w_i
  formed by quadrature, and B^{-1} S(u) must give u_hat back;
* the chunked scheme of the mass-solve kernels (tests/chunkalg.py) against the
  oracle, within the bound that the conditioning of B allows.
"""
from fractions import Fraction

import numpy as np
import numpy.polynomial.chebyshev as Ch
import pytest

import chebexact as cx
import chunkalg as ca
from oracle import shen_oracle as so

FAMS = {"helmholtz": "dirichlet", "biharmonic": "biharmonic"}


def _solve_exact(M, b):
    """Gaussian elimination in rationals (M is symmetric positive definite)."""
    n = len(M)
    A = [list(row) + [b[i]] for i, row in enumerate(M)]
    for c in range(n):
        for r in range(c + 1, n):
            if A[r][c] != 0:
                f = A[r][c] / A[c][c]
                A[r] = [x - f * y for x, y in zip(A[r], A[c])]
    x = [Fraction(0)] * n
    for r in range(n - 1, -1, -1):
        x[r] = (A[r][n] - sum(A[r][j] * x[j] for j in range(r + 1, n))) / A[r][r]
    return x


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
@pytest.mark.parametrize("N", [9, 12])
@pytest.mark.parametrize("gl", [False, True])
def test_mass_solve_exact(family, N, gl):
    rng = np.random.default_rng(N + 10 * gl)
    M = cx.matrix_over_pi(FAMS[family], 0, N, gl=gl)  # B / pi, exact
    n = len(M)
    fr = rng.integers(-9, 10, size=n)
    fi = rng.integers(-9, 10, size=n)
    # B u = f  <=>  (B / pi) u = f / pi: solve with f' = f, then divide by pi
    xr = _solve_exact(M, [Fraction(int(v)) for v in fr])
    xi = _solve_exact(M, [Fraction(int(v)) for v in fi])
    exact = (np.array([float(v) for v in xr]) + 1j * np.array([float(v) for v in xi])) / np.pi
    f = np.zeros((1, N), complex)
    f[0, :n] = fr + 1j * fi
    f[0, n:] = 123.0  # ignored
    u = so.mass_solve(family, N, f, so.GL if gl else so.GC)
    assert np.all(u[0, n:] == 0)
    assert np.max(np.abs(u[0, :n] - exact)) <= 1e-14 * np.max(np.abs(exact))


def _quad(N, gl):
    i = np.arange(N)
    if gl:
        x = np.cos(i * np.pi / (N - 1))
        c = np.ones(N)
        c[0] = c[-1] = 2.0
        return x, np.pi / (c * (N - 1))
    return np.cos((2 * i + 1) * np.pi / (2 * N)), np.full(N, np.pi / N)


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
@pytest.mark.parametrize("N", [16, 33])
@pytest.mark.parametrize("gl", [False, True])
def test_transform_round_trip(family, N, gl):
    rng = np.random.default_rng(7 * N + gl)
    n = so.n_of(family, N)
    x, w = _quad(N, gl)
    Phi = np.array([Ch.chebval(x, np.array([float(v) for v in cx.basis(FAMS[family], k)])) for k in range(n)])  # [k, i]
    uhat = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    vals = uhat @ Phi                      # u(x_i)
    S = np.zeros((3, N), complex)
    S[:, :n] = (vals * w) @ Phi.T          # S_l(u) = (u, phi_l)_sigma by quadrature
    back = so.mass_solve(family, N, S, so.GL if gl else so.GC)
    kappa = np.linalg.cond(so.mass_matrix(family, N, so.GL if gl else so.GC))
    assert np.max(np.abs(back[:, :n] - uhat)) <= 50 * kappa * 2.2e-16 * np.max(np.abs(uhat))


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_mass_solve_is_symmetric(family):
    """B^{-1} is symmetric: <g, B^{-1} f> = <B^{-1} g, f> for real f, g."""
    N = 40
    rng = np.random.default_rng(3)
    n = so.n_of(family, N)
    f = np.zeros((1, N), complex)
    g = np.zeros((1, N), complex)
    f[0, :n] = rng.standard_normal(n)
    g[0, :n] = rng.standard_normal(n)
    a = np.vdot(g, so.mass_solve(family, N, f)).real
    b = np.vdot(so.mass_solve(family, N, g), f).real
    assert abs(a - b) <= 1e-12 * abs(a)


def mass_tol(family, N, gl=False):
    """Parity bar of a mass solve, relative to max |u| per system: the error of a
    plain FP64 factorisation of B is a small multiple of cond(B) times the unit
    roundoff (measured about 0.01 cond(B) eps), so 0.1 cond(B) eps, floor 1e-13."""
    kappa = np.linalg.cond(so.mass_matrix(family, N, so.GL if gl else so.GC))
    return max(1e-13, 0.1 * kappa * 2.2e-16)


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
@pytest.mark.parametrize("N,C,G", [(9, 8, 16), (64, 8, 16), (300, 8, 32), (512, 16, 16)])
def test_chunked_mass_scheme(family, N, C, G):
    rng = np.random.default_rng(N)
    f = rng.standard_normal((6, N)) + 1j * rng.standard_normal((6, N))
    ref = so.mass_solve(family, N, f)
    u = ca.mass_chunked(family, f, N, C, G)
    assert so.rel_err_per_system(u, ref).max() <= mass_tol(family, N)


# --------------------------------------------------------------- Bbar fhat = Cbar uhat

@pytest.mark.parametrize("N", [8, 9, 12, 17])
@pytest.mark.parametrize("gl", [False, True])
def test_derivative_matrix_exact(N, gl):
    """Cbar_kj = (phichk_j', phibar_k)_sigma from exact rational algebra."""
    ph_d = [cx.basis("dirichlet", k) for k in range(N - 2)]
    dph_b = [cx.nderiv(cx.basis("biharmonic", j), 1) for j in range(N - 4)]
    exact = np.array([[float(cx.inner_over_pi(dph_b[j], ph_d[k], N, gl)) for j in range(N - 4)]
                      for k in range(N - 2)]) * np.pi
    np.testing.assert_allclose(so.derivative_matrix(N), exact, rtol=1e-14, atol=1e-13)


@pytest.mark.parametrize("N", [16, 33])
@pytest.mark.parametrize("gl", [False, True])
def test_derivative_projection_by_quadrature(N, gl):
    """fhat solves Bbar fhat = ((u', phibar_k)_sigma)_k, the scalar products formed by
    quadrature of numpy.polynomial derivative values of u = sum_j uhat_j phichk_j."""
    rng = np.random.default_rng(11 * N + gl)
    nb, nd = N - 4, N - 2
    x, w = _quad(N, gl)
    Phi_d = np.array([Ch.chebval(x, np.array([float(v) for v in cx.basis("dirichlet", k)])) for k in range(nd)])
    dPhi_b = np.array([Ch.chebval(x, Ch.chebder(np.array([float(v) for v in cx.basis("biharmonic", j)])))
                       for j in range(nb)])
    uhat = np.zeros((2, N), complex)
    uhat[:, :nb] = rng.standard_normal((2, nb)) + 1j * rng.standard_normal((2, nb))
    du = uhat[:, :nb] @ dPhi_b                      # u'(x_i)
    S = np.zeros((2, N), complex)
    S[:, :nd] = (du * w) @ Phi_d.T                  # (u', phibar_k)_sigma
    ref = so.mass_solve("helmholtz", N, S, so.GL if gl else so.GC)
    got = so.derivative_solve(N, uhat, so.GL if gl else so.GC)
    assert np.all(got[:, nd:] == 0)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_derivative_of_a_dirichlet_function_is_reproduced():
    """u = (1 - x^2)^2 q(x) lies in the biharmonic space, and u' vanishes at both walls, so u'
    lies in the Dirichlet space and its Galerkin projection is u' itself: fhat must be the
    Dirichlet coefficients of u'."""
    N = 24
    q = np.array([0.3, -0.2, 0.5])                       # power series of q
    u_pow = np.polynomial.polynomial.polymul(np.polynomial.polynomial.polypow([1.0, 0.0, -1.0], 2), q)
    du_pow = np.polynomial.polynomial.polyder(u_pow)
    u_ch = np.polynomial.chebyshev.poly2cheb(u_pow)
    du_ch = np.polynomial.chebyshev.poly2cheb(du_pow)
    nb, nd = N - 4, N - 2
    # coefficients in the two bases by least squares on the Chebyshev coefficients (exact here)
    Bb = np.zeros((N, nb))
    for j in range(nb):
        c = np.array([float(v) for v in cx.basis("biharmonic", j)])
        Bb[:c.size, j] = c
    Bd = np.zeros((N, nd))
    for k in range(nd):
        c = np.array([float(v) for v in cx.basis("dirichlet", k)])
        Bd[:c.size, k] = c
    tgt = np.zeros(N)
    tgt[:u_ch.size] = u_ch
    uh = np.linalg.lstsq(Bb, tgt, rcond=None)[0]
    assert np.allclose(Bb @ uh, tgt, atol=1e-13)
    tgt_d = np.zeros(N)
    tgt_d[:du_ch.size] = du_ch
    fd = np.linalg.lstsq(Bd, tgt_d, rcond=None)[0]
    assert np.allclose(Bd @ fd, tgt_d, atol=1e-13)
    uhat = np.zeros((1, N), complex)
    uhat[0, :nb] = uh
    got = so.derivative_solve(N, uhat)
    np.testing.assert_allclose(got[0, :nd].real, fd, atol=1e-12)


@pytest.mark.parametrize("N", [16, 64, 512, 1024])
def test_dirichlet_mass_pivots_closed_form(N):
    """At Gauss points the Dirichlet mass matrix restricted to a parity chain is tridiagonal with
    off-diagonals -pi/2 and diagonal pi (3 pi/2 in row 0 of the even chain), so the unpivoted LU
    pivots are d_m = (pi/2)(2m+3)/(2m+1) (even chain) and (pi/2)(m+2)/(m+1) (odd chain): the
    closed form the one-pass Dirichlet forward transform uses.  Checked against the pivot
    recurrence of the oracle's matrix, and their product against its determinant."""
    B = so.mass_matrix("helmholtz", N, so.GC)
    n = N - 2
    for p in (0, 1):
        idx = np.arange(p, n, 2)
        Bc = B[np.ix_(idx, idx)]
        assert np.allclose(np.diag(Bc, 1), -np.pi / 2) and np.allclose(np.diag(Bc, -1), -np.pi / 2)
        assert np.count_nonzero(np.triu(Bc, 2)) == 0
        d = np.empty(len(idx))
        prev = None
        for m in range(len(idx)):  # the pivot recurrence of the unpivoted LU
            d[m] = Bc[m, m] if m == 0 else Bc[m, m] - Bc[m, m - 1] * Bc[m - 1, m] / prev
            prev = d[m]
        M = np.arange(len(idx), dtype=np.float64)
        closed = (np.pi / 2) * ((2 * M + 3) / (2 * M + 1) if p == 0 else (M + 2) / (M + 1))
        np.testing.assert_allclose(d, closed, rtol=1e-13)
        # and the product of the pivots is the determinant of the chain's matrix
        sign, logdet = np.linalg.slogdet(Bc)
        assert sign > 0 and abs(logdet - np.sum(np.log(closed))) <= 1e-10 * max(1.0, abs(logdet))
