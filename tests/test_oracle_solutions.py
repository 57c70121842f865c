"""Pins of the oracle's solves against answers it does not compute itself.

* closed-form problems (Poisson, clamped plate);
* manufactured solutions: random Shen coefficients -> Chebyshev series ->
  the continuous operator applied with numpy.polynomial.chebyshev.chebder ->
  right-hand side from discrete Chebyshev orthogonality; the oracle must
  return the coefficients (independent of its closed-form matrices);
* limits (alpha -> inf, b -> inf) against mass-matrix solves;
* the roundoff protocol of Sec. 5 against the paper's table (upper bound);
* adjoint identities.
"""
import os

import numpy as np
import numpy.polynomial.chebyshev as C
import pytest

from oracle import shen_oracle as so
from paper_1701_03787_amd import workloads as wl

PI = np.pi
HERE = os.path.dirname(os.path.abspath(__file__))


def test_poisson_closed_form():
    # u = (1-x^2)/2 = phi_0/4 solves -u'' = 1 with u(+-1) = 0; (1, phi_k) = pi delta_k0.
    for N in (8, 33, 64):
        f = np.zeros((1, N), complex)
        f[0, 0] = PI
        u = so.helmholtz_solve(N, [0.0], f)
        ref = np.zeros(N)
        ref[0] = 0.25
        np.testing.assert_allclose(u[0].real, ref, atol=1e-14)
        assert np.all(u[0].imag == 0)


def test_clamped_plate_closed_form():
    # u = (1-x^2)^2 = (3/8) phi_0 solves u'''' = 24 with u = u' = 0 at the walls.
    for N in (8, 33, 64):
        f = np.zeros((1, N), complex)
        f[0, 0] = 24 * PI + 24j * PI
        u = so.biharmonic_solve(N, [0.0], [0.0], f)
        ref = np.zeros(N)
        ref[0] = 3 / 8
        np.testing.assert_allclose(u[0].real, ref, atol=1e-14)
        np.testing.assert_allclose(u[0].imag, ref, atol=1e-14)


def _tm_products(g, N, gl):
    """(g, T_m)_sigma for a Chebyshev series g (coefficients), m = 0..N-1."""
    c = np.ones(N)
    c[0] = 2.0
    if gl:
        c[N - 1] = 2.0
    gg = np.zeros(N)
    gg[: min(N, len(g))] = g[:N]
    return gg * c * PI / 2


def manufactured_rhs(family, N, coeffs, uhat, gl=False):
    """f_k = (L u, phi_k)_sigma for u = sum uhat_k phi_k, L from the continuous operator."""
    nsys = uhat.shape[0]
    f = np.zeros((nsys, N), complex)
    for w in range(nsys):
        for part, unit in ((uhat[w].real, 1.0), (uhat[w].imag, 1j)):
            cheb = np.zeros(N)
            if family == "helmholtz":
                n = N - 2
                cheb[:n] += part[:n]
                cheb[2:n + 2] -= part[:n]
                Lu = coeffs[0][w] * cheb
                d2 = C.chebder(cheb, 2)
                Lu[: len(d2)] -= d2
                tm = _tm_products(Lu, N, gl)
                fk = tm[:n] - tm[2:n + 2]
            else:
                n = N - 4
                k = np.arange(n)
                cheb[:n] += part[:n]
                cheb[2:n + 2] -= 2 * (k + 2) / (k + 3) * part[:n]
                cheb[4:n + 4] += (k + 1) / (k + 3) * part[:n]
                Lu = coeffs[1][w] * cheb
                d2 = C.chebder(cheb, 2)
                d4 = C.chebder(cheb, 4)
                Lu[: len(d2)] += coeffs[0][w] * d2
                Lu[: len(d4)] += d4
                tm = _tm_products(Lu, N, gl)
                fk = tm[:n] - 2 * (k + 2) / (k + 3) * tm[2:n + 2] + (k + 1) / (k + 3) * tm[4:n + 4]
            f[w, :n] += unit * fk
    return f


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
@pytest.mark.parametrize("N", [12, 32, 65])
@pytest.mark.parametrize("gl", [False, True])
def test_manufactured(family, N, gl):
    g = wl.small_grid(N, 12, kmax=48)
    coeffs = g.coefficients(family)
    n = wl.n_unknowns(family, N)
    rng = np.random.default_rng([1701, 11, N, int(gl)])
    uhat = np.zeros((12, N), complex)
    uhat[:, :n] = rng.standard_normal((12, n)) + 1j * rng.standard_normal((12, n))
    uhat[1:4, :n] *= (np.arange(n) + 1.0) ** -3  # also a decaying spectrum
    f = manufactured_rhs(family, N, coeffs, uhat, gl)
    u = so.solve(family, N, coeffs, f, quad=so.GL if gl else so.GC)
    err = so.rel_err_per_system(u, uhat)
    assert err.max() < 1e-11, err.max()
    assert np.all(u[:, n:] == 0)


def test_manufactured_detects_planted_mistake():
    """A wrong sign on Achk (a plausible slip) must fail the manufactured check."""
    N = 32
    g = wl.small_grid(N, 4, kmax=48)
    a, b = g.coefficients("biharmonic")
    rng = np.random.default_rng(5)
    uhat = np.zeros((4, N), complex)
    uhat[:, : N - 4] = rng.standard_normal((4, N - 4))
    f = manufactured_rhs("biharmonic", N, (a, b), uhat)
    op = so.Operators.get(N)
    H = op.Qb - a[:, None, None] * op.Ab + b[:, None, None] * op.Bb
    x = np.linalg.solve(H, f[:, : N - 4].real[..., None])[..., 0]
    assert np.max(np.abs(x - uhat[:, : N - 4].real)) > 1e-6


def test_large_coefficient_limits():
    N = 40
    rng = np.random.default_rng(3)
    f = np.zeros((2, N), complex)
    f[:, : N - 2] = rng.standard_normal((2, N - 2))
    big = 1e18  # ||Bbar^-1|| ||Sbar|| ||Bbar^-1|| / big << 1
    u = so.helmholtz_solve(N, [big, big], f)
    ref = np.linalg.solve(so.dirichlet_mass(N), f[:, : N - 2].T).T
    np.testing.assert_allclose(big * u[:, : N - 2], ref, rtol=1e-6, atol=1e-9)
    fb = np.zeros((2, N), complex)
    fb[:, : N - 4] = rng.standard_normal((2, N - 4))
    ub = so.biharmonic_solve(N, [0.0, 0.0], [big, big], fb)
    refb = np.linalg.solve(so.biharmonic_mass(N), fb[:, : N - 4].T).T
    np.testing.assert_allclose(big * ub[:, : N - 4], refb, rtol=1e-5, atol=1e-9)


def _roundoff_table():
    rows = {}
    with open(os.path.join(HERE, "golden", "roundoff_table.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            fam, z, *vals = line.split()
            rows[(fam, int(z))] = dict(zip((64, 128, 256, 512, 1024, 2048, 4096), map(float, vals)))
    return rows


def roundoff_protocol(solver, family, N, z, runs, seed=0):
    """Sec. 5: u ~ U(0,1), f = H u formed accurately, v = solve(f), mean of max|u-v|/max|u|."""
    inv = 2.0 / ((1.0 / 5200.0) * 1e-5)
    K2 = float(z) ** 2
    coeffs = (np.full(runs, K2 + inv),) if family == "helmholtz" else (
        np.full(runs, -(2 * K2 + inv)), np.full(runs, K2 * (K2 + inv)))
    n = wl.n_unknowns(family, N)
    rng = np.random.default_rng([1701, 55, N, z, seed])
    u = np.zeros((runs, N), complex)
    u[:, :n] = rng.uniform(0.0, 1.0, (runs, n))
    f = so.matvec(family, N, coeffs, u, extended=True)
    v = solver(family, N, coeffs, f)
    return float(np.mean(so.rel_err_per_system(v, u)))


@pytest.mark.parametrize("family", ["biharmonic", "helmholtz"])
def test_roundoff_vs_paper_table(family):
    """In the Sec. 5 protocol the (refined) oracle is at least as accurate as the paper's
    O(N) solver; plain partially pivoted gesv is not, on the biharmonic matrices."""
    table = _roundoff_table()
    worst_plain = 0.0
    for N in (64, 128, 256):
        for z in (0, 200, 1800, 5400):
            e = roundoff_protocol(lambda fam, N_, c, f: so.solve(fam, N_, c, f), family, N, z, runs=8)
            assert e <= table[(family, z)][N], (family, N, z, e, table[(family, z)][N])
            ep = roundoff_protocol(lambda fam, N_, c, f: so.solve(fam, N_, c, f, refine=0), family, N, z, runs=8)
            worst_plain = max(worst_plain, ep / table[(family, z)][N])
    if family == "biharmonic":
        assert worst_plain > 5.0  # why the oracle refines


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_adjoint_identity(family):
    N = 48
    g = wl.small_grid(N, 6)
    coeffs = g.coefficients(family)
    n = wl.n_unknowns(family, N)
    rng = np.random.default_rng(9)
    gvec = np.zeros((6, N), complex)
    v = np.zeros((6, N), complex)
    gvec[:, :n] = rng.standard_normal((6, n)) + 1j * rng.standard_normal((6, n))
    v[:, :n] = rng.standard_normal((6, n)) + 1j * rng.standard_normal((6, n))
    lam = so.solve(family, N, coeffs, gvec, transpose=True)
    lhs = np.sum(so.matvec(family, N, coeffs, lam, transpose=True) * v, axis=1)
    rhs = np.sum(lam * so.matvec(family, N, coeffs, v), axis=1)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12)
    np.testing.assert_allclose(so.matvec(family, N, coeffs, lam, transpose=True), gvec, rtol=0, atol=1e-9 * np.abs(gvec).max())


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_gradients_finite_difference(family):
    """Coefficient and RHS gradients of L = Re<w,u> + |u|^2/2 vs central differences."""
    N = 24
    g = wl.small_grid(N, 3)
    coeffs = [c.copy() for c in g.coefficients(family)]
    f = g.rhs(family)
    rng = np.random.default_rng(4)
    wv = rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N))

    def loss(cs, ff):
        u = so.solve(family, N, cs, ff)
        return np.real(np.sum(np.conj(wv) * u)) + 0.5 * np.sum(np.abs(u) ** 2)

    u = so.solve(family, N, coeffs, f)
    gu = wv + u
    _, lam, grads = so.solve_grads(family, N, coeffs, f, gu)
    for ci, gc in enumerate(grads):
        for w in range(3):
            h = 1e-6 * max(1.0, abs(coeffs[ci][w]))
            cp = [c.copy() for c in coeffs]
            cm = [c.copy() for c in coeffs]
            cp[ci][w] += h
            cm[ci][w] -= h
            fd = (loss(cp, f) - loss(cm, f)) / (2 * h)
            assert abs(fd - gc[w]) <= 1e-6 * max(1.0, abs(gc[w])) + 1e-9, (ci, w, fd, gc[w])
    n = wl.n_unknowns(family, N)
    d = np.zeros((3, N), complex)
    d[:, :n] = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    h = 1e-6
    fd = (loss(coeffs, f + h * d) - loss(coeffs, f - h * d)) / (2 * h)
    an = np.real(np.sum(np.conj(lam) * d))
    assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
