"""Pins of the oracle's Crank-Nicolson right-hand sides (Sec. 3, eqs. ufin and gfin)
against the time-continuous problems they discretise, not against its own matrices.

The step solves  d/dt (grad^2 u) = h_u + nu grad^4 u  (biharmonic basis) and
d g/dt = h_g + nu grad^2 g  (Dirichlet basis) for one Fourier mode, grad^2 = D^2 - z2.
Everything here is computed from the basis definitions (Sec. 2), numpy's Chebyshev
derivatives and Gauss-Chebyshev quadrature:

* steady states: with h = -nu grad^4 v (resp. -nu grad^2 g) the step must leave the
  coefficients unchanged, i.e. solve(rhs) returns them;
* time convergence: a manufactured solution v = exp(-t) w(x) stepped to t = T with the
  exact forcing at the half step is reached with an error that falls as dt^2.

A wrong sign or factor on any term of either operator breaks one of these.
"""
import numpy as np
import numpy.polynomial.chebyshev as C
import pytest

from oracle import shen_oracle as so

PI = np.pi


def shen_to_cheb(family, N, uh):
    """Chebyshev coefficients (length N) of sum_k uh_k phi_k (basis definitions, Sec. 2)."""
    c = np.zeros(N)
    if family == "helmholtz":
        n = N - 2
        c[:n] += uh[:n]
        c[2:n + 2] -= uh[:n]
    else:
        n = N - 4
        k = np.arange(n)
        c[:n] += uh[:n]
        c[2:n + 2] -= 2.0 * (k + 2) / (k + 3) * uh[:n]
        c[4:n + 4] += (k + 1) / (k + 3) * uh[:n]
    return c


def gc_scalar_products(family, N, cheb):
    """(g, phi_k)_sigma for a Chebyshev series g: N-point Gauss-Chebyshev quadrature."""
    j = np.arange(N)
    x = np.cos(PI * (2 * j + 1) / (2 * N))
    gx = C.chebval(x, cheb)
    n = so.n_of(family, N)
    out = np.zeros(N)
    for k in range(n):
        e = np.zeros(k + 5)
        e[k] = 1.0
        if family == "helmholtz":
            e[k + 2] = -1.0
        else:
            e[k + 2] = -2.0 * (k + 2) / (k + 3)
            e[k + 4] = (k + 1) / (k + 3)
        out[k] = np.sum(gx * C.chebval(x, e)) * PI / N
    return out


def lap(cheb, z2, times=1):
    """(D^2 - z2)^times applied to a Chebyshev series."""
    c = np.array(cheb, dtype=float)
    for _ in range(times):
        d2 = C.chebder(c, 2)
        nxt = -z2 * c
        nxt[: len(d2)] += d2
        c = nxt
    return c


def coeffs_of(family, K2, nu, dt):
    inv = 2.0 / (nu * dt)
    if family == "helmholtz":
        return (np.array([K2 + inv]),)
    return (np.array([-(2.0 * K2 + inv)]), np.array([K2 * (K2 + inv)]))


def _sh(family, N, cheb_h):
    return gc_scalar_products(family, N, cheb_h)[None, :].astype(complex)


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
@pytest.mark.parametrize("K2", [0.0, 5.0, 130.0])
def test_steady_state_is_a_fixed_point(family, K2):
    N = 16
    nu, dt = 0.37, 0.021
    rng = np.random.default_rng([1701, 31, int(K2)])
    n = so.n_of(family, N)
    uh = np.zeros((1, N), complex)
    uh[0, :n] = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    sh = np.zeros((1, N), complex)
    for part, unit in ((uh[0].real, 1.0), (uh[0].imag, 1j)):
        c = shen_to_cheb(family, N, part)
        h = -nu * (lap(c, K2, 1) if family == "helmholtz" else lap(c, K2, 2))
        sh += unit * _sh(family, N, h)
    rhs = so.rhs_assemble(family, N, [K2], nu, dt, uh, sh)
    got = so.solve(family, N, coeffs_of(family, K2, nu, dt), rhs)
    assert np.max(np.abs(got - uh)) <= 1e-12 * np.max(np.abs(uh))
    assert np.all(rhs[:, n:] == 0)


def _cn_error(family, N, K2, nu, dt, T):
    """Step v = exp(-t) w from t=0 to T with the exact forcing at half steps."""
    n = so.n_of(family, N)
    # w: a fixed polynomial of the space (a few random Shen coefficients)
    rng = np.random.default_rng([1701, 32])
    what = np.zeros(N)
    what[: min(n, 6)] = rng.standard_normal(min(n, 6))
    w = shen_to_cheb(family, N, what)
    if family == "helmholtz":
        # dg/dt = h + nu lap g ; g = e^-t w  =>  h = e^-t (-w - nu lap w)
        base = -w - nu * lap(w, K2, 1)
    else:
        # d/dt lap v = h + nu lap^2 v ; v = e^-t w  =>  h = e^-t (-lap w - nu lap^2 w)
        base = -lap(w, K2, 1) - nu * lap(w, K2, 2)
    sbase = _sh(family, N, base)
    cs = coeffs_of(family, K2, nu, dt)
    u = np.zeros((1, N), complex)
    u[0, :n] = what[:n]
    steps = int(round(T / dt))
    for kappa in range(steps):
        th = (kappa + 0.5) * dt
        rhs = so.rhs_assemble(family, N, [K2], nu, dt, u, np.exp(-th) * sbase)
        u = so.solve(family, N, cs, rhs)
    exact = np.exp(-steps * dt) * what
    return np.max(np.abs(u[0, :n].real - exact[:n])) / np.max(np.abs(exact[:n]))


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_crank_nicolson_second_order(family):
    N, K2, nu, T = 14, 3.0, 0.3, 0.4
    e1 = _cn_error(family, N, K2, nu, 0.04, T)
    e2 = _cn_error(family, N, K2, nu, 0.02, T)
    assert e1 < 1e-2
    assert 3.5 < e1 / e2 < 4.5, (e1, e2)


def test_extended_matches_fp64():
    N = 40
    rng = np.random.default_rng([1701, 33])
    uh = rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N))
    sh = rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N))
    for fam in ("helmholtz", "biharmonic"):
        a = so.rhs_assemble(fam, N, [0.0, 7.0, 99.0], 5e-5, 5e-4, uh, sh)
        b = so.rhs_assemble(fam, N, [0.0, 7.0, 99.0], 5e-5, 5e-4, uh, sh, extended=True)
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
        c = so.rhs_assemble(fam, N, [0.0, 7.0, 99.0], 5e-5, 5e-4, uh, None)
        d = so.rhs_assemble(fam, N, [0.0, 7.0, 99.0], 5e-5, 5e-4, uh, np.zeros_like(sh))
        assert np.array_equal(c, d)
