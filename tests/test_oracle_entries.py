"""Pins of the oracle's closed-form Galerkin matrices.

Three independent routes to each entry (row k = test function, column j):
exact rational Chebyshev algebra, numerical Gauss-Chebyshev / Gauss-Lobatto
quadrature of the basis functions and their derivatives (numpy.polynomial),
and a handful of hand-computed values.
"""
from fractions import Fraction

import numpy as np
import numpy.polynomial.chebyshev as C
import pytest

import chebexact as cx
from oracle import shen_oracle as so

PI = np.pi


def _exact(family, p, N, gl=False, sign=1):
    M = cx.matrix_over_pi(family, p, N, gl=gl, sign=sign)
    return np.array([[float(v) for v in row] for row in M]) * PI


@pytest.mark.parametrize("N", [6, 7, 9, 12, 17, 24])
@pytest.mark.parametrize("gl", [False, True])
def test_dirichlet_exact(N, gl):
    quad = so.GL if gl else so.GC
    np.testing.assert_allclose(so.dirichlet_mass(N, quad), _exact("dirichlet", 0, N, gl), rtol=1e-14, atol=1e-13)
    np.testing.assert_allclose(so.dirichlet_stiffness(N), _exact("dirichlet", 2, N, gl, sign=-1), rtol=1e-14, atol=1e-12)


@pytest.mark.parametrize("N", [6, 7, 9, 12, 17, 24])
@pytest.mark.parametrize("gl", [False, True])
def test_biharmonic_exact(N, gl):
    quad = so.GL if gl else so.GC
    np.testing.assert_allclose(so.biharmonic_mass(N, quad), _exact("biharmonic", 0, N, gl), rtol=1e-14, atol=1e-13)
    np.testing.assert_allclose(so.biharmonic_laplacian(N), _exact("biharmonic", 2, N, gl), rtol=1e-14, atol=1e-11)
    np.testing.assert_allclose(so.biharmonic_bilaplacian(N), _exact("biharmonic", 4, N, gl), rtol=1e-14, atol=1e-9)


def _quad_points(N, gl):
    i = np.arange(N)
    if gl:
        x = np.cos(i * PI / (N - 1))
        c = np.ones(N)
        c[0] = c[-1] = 2.0
        w = PI / (c * (N - 1))
    else:
        x = np.cos((2 * i + 1) * PI / (2 * N))
        w = np.full(N, PI / N)
    return x, w


def _quad_matrix(family, p, N, gl, sign=1):
    n = N - 2 if family == "dirichlet" else N - 4
    x, w = _quad_points(N, gl)
    V = []
    D = []
    for k in range(n):
        c = np.array([float(v) for v in cx.basis(family, k)])
        V.append(C.chebval(x, c))
        D.append(C.chebval(x, C.chebder(c, p)) if p else C.chebval(x, c))
    V = np.array(V)
    D = np.array(D)
    return sign * (V * w) @ D.T  # [k, j] = sum_i phi_k(x_i) phi_j^(p)(x_i) w_i


@pytest.mark.parametrize("N", [8, 11, 16, 20])
@pytest.mark.parametrize("gl", [False, True])
def test_quadrature(N, gl):
    quad = so.GL if gl else so.GC
    chk = [
        (so.dirichlet_mass(N, quad), _quad_matrix("dirichlet", 0, N, gl)),
        (so.dirichlet_stiffness(N), _quad_matrix("dirichlet", 2, N, gl, sign=-1)),
        (so.biharmonic_mass(N, quad), _quad_matrix("biharmonic", 0, N, gl)),
        (so.biharmonic_laplacian(N), _quad_matrix("biharmonic", 2, N, gl)),
        (so.biharmonic_bilaplacian(N), _quad_matrix("biharmonic", 4, N, gl)),
    ]
    for mine, q in chk:
        scale = np.max(np.abs(q))
        assert np.max(np.abs(mine - q)) <= 1e-13 * scale


def test_hand_values():
    """Entries worked out by hand from T_n'' = sum n(n^2-m^2)/c_m T_m and T_n'''' of low degree."""
    N = 16
    S = so.dirichlet_stiffness(N)
    A = so.biharmonic_laplacian(N)
    Q = so.biharmonic_bilaplacian(N)
    B = so.biharmonic_mass(N)
    assert S[0, 0] == pytest.approx(4 * PI)
    assert S[0, 2] == pytest.approx(4 * PI) and S[0, 4] == pytest.approx(4 * PI)
    assert S[1, 1] == pytest.approx(12 * PI) and S[1, 3] == pytest.approx(8 * PI)
    assert A[0, 0] == pytest.approx(-16 * PI / 3)
    assert A[0, 2] == pytest.approx(4 * PI) and A[2, 0] == pytest.approx(8 * PI)
    assert Q[0, 0] == pytest.approx(64 * PI) and Q[1, 1] == pytest.approx(480 * PI)
    assert Q[2, 2] == pytest.approx(1728 * PI)
    assert Q[0, 2] == pytest.approx(768 * PI / 5) and Q[1, 3] == pytest.approx(640 * PI)
    assert B[0, 0] == pytest.approx(35 * PI / 18)


def test_printed_q_diagonal_is_not_the_definition():
    """The Sec. 4 printed diagonal -4(k+1)(k+2)^2 disagrees with the definition; the oracle
    follows the definition (exact value 64 pi at k = 0, forced by the clamped plate)."""
    exact00 = cx.matrix_over_pi("biharmonic", 4, 8)[0][0]
    assert exact00 == Fraction(64)
    assert so.biharmonic_bilaplacian(8)[0, 0] == pytest.approx(64 * PI)
    assert -4 * 1 * 2 ** 2 != 64


@pytest.mark.parametrize("N", [9, 16, 33])
def test_structure(N):
    """Bandwidths the fast solvers rely on (Sec. 4): Achk 3 diagonals, Bchk 5, Qchk and Sbar
    upper triangular, and the odd/even decoupling of every matrix."""
    op = so.Operators.get(N)
    k = np.arange(N - 4)
    off = np.abs(k[:, None] - k[None, :])
    assert np.all(op.Ab[off > 2] == 0)
    assert np.all(op.Bb[off > 4] == 0)
    assert np.all(np.tril(op.Qb, -1) == 0)
    assert np.all(np.tril(op.Sd, -1) == 0)
    for M in (op.Ab, op.Bb, op.Qb):
        assert np.all(M[(off % 2) == 1] == 0)
    kd = np.arange(N - 2)
    offd = np.abs(kd[:, None] - kd[None, :])
    for M in (op.Bd, op.Sd):
        assert np.all(M[(offd % 2) == 1] == 0)
