"""Pins of the oracle's wall-normal Shen transforms (Sec. 2; appendix algorithms for the
forward scalar products / transforms and the inverse transforms) against things it does
not compute itself:

* discrete orthogonality: (T_m, T_k)_sigma = c_k pi/2 delta_km at the N Gauss or
  Gauss-Lobatto points (c_0 = 2, and c_{N-1} = 2 for Gauss-Lobatto);
* the appendix's own route: SciPy's DCT of type 2 (Gauss) or 1 (Gauss-Lobatto) scaled by
  pi/(2N) or pi/(2(N-1)), then the Shen combination; and for the inverse the DCT of type 3
  (Gauss) or 1 (Gauss-Lobatto) with its end corrections, after the Shen -> Chebyshev map;
* round trips: forward(inverse(uhat)) = uhat and inverse(forward(u)) = u on the space;
* point values of known polynomials: phi_k(x) at the points from numpy's chebval.
"""
import numpy as np
import numpy.polynomial.chebyshev as C
import pytest
import scipy.fft as sf

from oracle import shen_oracle as so

PI = np.pi
QUADS = [so.GC, so.GL]


def rng(*tail):
    return np.random.default_rng([1701, 40, *tail])


def shen_combine(space, w):
    """Alg. forwardScalar: Shen combination of the Chebyshev scalar products w."""
    N = w.shape[-1]
    y = np.zeros_like(w)
    if space == "dirichlet":
        y[..., :N - 2] = w[..., :N - 2] - w[..., 2:]
    elif space == "biharmonic":
        k = np.arange(N - 4)
        y[..., :N - 4] = w[..., :N - 4] - 2 * (k + 2) / (k + 3) * w[..., 2:N - 2] + (k + 1) / (k + 3) * w[..., 4:]
    else:
        y = w.copy()
    return y


def scipy_scalar(space, u, quad):
    N = u.shape[-1]
    if quad == so.GC:
        w = sf.dct(u.real, type=2, axis=-1) * PI / (2 * N) + 1j * sf.dct(u.imag, type=2, axis=-1) * PI / (2 * N)
    else:
        w = sf.dct(u.real, type=1, axis=-1) * PI / (2 * (N - 1)) + 1j * sf.dct(u.imag, type=1, axis=-1) * PI / (2 * (N - 1))
    return shen_combine(space, w)


def shen_to_cheb(space, f):
    """Alg. inverseShenTransform: Shen coefficients -> Chebyshev coefficients."""
    N = f.shape[-1]
    z = np.zeros_like(f)
    if space == "chebyshev":
        return f.copy()
    if space == "dirichlet":
        z[..., :N - 2] += f[..., :N - 2]
        z[..., 2:] -= f[..., :N - 2]
        return z
    k = np.arange(N - 4)
    z[..., :N - 4] += f[..., :N - 4]
    z[..., 2:N - 2] -= 2 * (k + 2) / (k + 3) * f[..., :N - 4]
    z[..., 4:] += (k + 1) / (k + 3) * f[..., :N - 4]
    return z


def scipy_inverse_cheb(z, quad):
    """Alg. inverseChebTransform: Chebyshev coefficients -> point values."""
    def real(a):
        if quad == so.GC:
            return 0.5 * sf.dct(a, type=3, axis=-1) + 0.5 * a[..., :1]
        N = a.shape[-1]
        y = 0.5 * sf.dct(a, type=1, axis=-1) + 0.5 * a[..., :1]
        return y + 0.5 * (-1.0) ** np.arange(N) * a[..., -1:]
    return real(z.real) + 1j * real(z.imag)


@pytest.mark.parametrize("quad", QUADS)
@pytest.mark.parametrize("N", [8, 17, 64])
def test_discrete_orthogonality(quad, N):
    for m in (0, 1, N // 2, N - 1):
        u = np.zeros((1, N), complex)
        u[0] = np.cos(m * np.arccos(so.quad_points(N, quad)))  # T_m at the points
        s = so.scalar_product("chebyshev", N, u, quad)[0]
        ref = np.zeros(N)
        ref[m] = PI / 2 * (2.0 if (m == 0 or (quad == so.GL and m == N - 1)) else 1.0)
        np.testing.assert_allclose(s.real, ref, atol=1e-13)
        assert np.max(np.abs(s.imag)) == 0


@pytest.mark.parametrize("space", so.SPACES)
@pytest.mark.parametrize("quad", QUADS)
@pytest.mark.parametrize("N", [9, 32, 100, 512])
def test_scalar_product_vs_appendix_dct(space, quad, N):
    u = rng(N, quad).standard_normal((3, N)) + 1j * rng(N, quad, 1).standard_normal((3, N))
    got = so.scalar_product(space, N, u, quad)
    want = scipy_scalar(space, u, quad)
    n = so.n_space(space, N)
    assert np.max(np.abs(got[:, :n] - want[:, :n])) <= 1e-13 * np.max(np.abs(want))
    assert np.all(got[:, n:] == 0)


@pytest.mark.parametrize("space", so.SPACES)
@pytest.mark.parametrize("quad", QUADS)
@pytest.mark.parametrize("N", [9, 32, 100, 512])
def test_inverse_vs_appendix_dct(space, quad, N):
    n = so.n_space(space, N)
    uh = np.zeros((3, N), complex)
    uh[:, :n] = rng(N, quad, 2).standard_normal((3, n)) + 1j * rng(N, quad, 3).standard_normal((3, n))
    got = so.backward_transform(space, N, uh, quad)
    want = scipy_inverse_cheb(shen_to_cheb(space, uh), quad)
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want))


@pytest.mark.parametrize("space", so.SPACES)
@pytest.mark.parametrize("quad", QUADS)
def test_point_values_from_chebval(space, quad):
    N = 24
    x = so.quad_points(N, quad)
    n = so.n_space(space, N)
    for k in (0, 1, n // 2, n - 1):
        uh = np.zeros((1, N), complex)
        uh[0, k] = 1.0
        c = shen_to_cheb(space, uh)[0].real
        np.testing.assert_allclose(so.backward_transform(space, N, uh, quad)[0].real, C.chebval(x, c), atol=1e-13)


@pytest.mark.parametrize("space", so.SPACES)
@pytest.mark.parametrize("quad", QUADS)
@pytest.mark.parametrize("N", [12, 64, 257])
def test_round_trips(space, quad, N):
    n = so.n_space(space, N)
    uh = np.zeros((4, N), complex)
    uh[:, :n] = rng(N, quad, 4).standard_normal((4, n)) + 1j * rng(N, quad, 5).standard_normal((4, n))
    u = so.backward_transform(space, N, uh, quad)
    back = so.forward_transform(space, N, u, quad)
    # the rounding of the point values reaches the coefficients amplified by up to the
    # condition number of the space's mass matrix (the mass-solve bar, reading A16)
    if space == "chebyshev":
        kappa = 2.0
    else:
        kappa = np.linalg.cond(so.mass_matrix("helmholtz" if space == "dirichlet" else "biharmonic", N, quad))
    bar = max(1e-13, 0.1 * kappa * np.finfo(float).eps)
    assert np.max(np.abs(back - uh)) <= bar * np.max(np.abs(uh))
    assert np.all(back[:, n:] == 0)
    again = so.backward_transform(space, N, back, quad)
    assert np.max(np.abs(again - u)) <= bar * np.max(np.abs(u))
