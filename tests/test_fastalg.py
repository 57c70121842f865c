"""The O(N) recurrences (NumPy prototype) against the oracle.

These fix, on the CPU, the arithmetic the HIP kernels implement: if a
recurrence were wrong here the GPU parity tests would be chasing it blind.
"""
import numpy as np
import pytest

import fastalg as fa
from oracle import shen_oracle as so
from paper_1701_03787_amd import workloads as wl
from test_oracle_solutions import _roundoff_table, roundoff_protocol


def _grid(N, nsys=16, kmax=200):
    return wl.small_grid(N, nsys, kmax=kmax)


@pytest.mark.parametrize("N", [6, 7, 8, 9, 10, 11, 16, 33, 64, 129, 256])
@pytest.mark.parametrize("gl", [False, True])
def test_helmholtz_recurrence(N, gl):
    g = _grid(N)
    alpha = g.alpha()
    f = g.rhs("helmholtz")
    u = fa.helmholtz_solve(alpha, f, N, gl)
    ref = so.helmholtz_solve(N, alpha, f, quad=so.GL if gl else so.GC)
    assert so.rel_err_per_system(u, ref).max() < 1e-13


@pytest.mark.parametrize("N", [6, 7, 8, 9, 10, 11, 12, 16, 33, 64, 129, 256])
@pytest.mark.parametrize("gl", [False, True])
def test_biharmonic_recurrence(N, gl):
    g = _grid(N)
    a, b = g.a(), g.b()
    f = g.rhs("biharmonic")
    u = fa.biharmonic_solve(a, b, f, N, gl)
    ref = so.biharmonic_solve(N, a, b, f, quad=so.GL if gl else so.GC)
    assert so.rel_err_per_system(u, ref).max() < 1e-12


@pytest.mark.parametrize("N", [8, 9, 33, 128])
def test_transposed(N):
    g = _grid(N, 8)
    gv = g.rhs("helmholtz")
    lam = fa.helmholtz_solve_T(g.alpha(), gv, N)
    ref = so.helmholtz_solve(N, g.alpha(), gv, transpose=True)
    assert so.rel_err_per_system(lam, ref).max() < 1e-13
    gv = g.rhs("biharmonic")
    lam = fa.biharmonic_solve_T(g.a(), g.b(), gv, N)
    ref = so.biharmonic_solve(N, g.a(), g.b(), gv, transpose=True)
    assert so.rel_err_per_system(lam, ref).max() < 1e-12


@pytest.mark.parametrize("N", [8, 33, 128])
def test_matvec(N):
    g = _grid(N, 6)
    u = g.rhs("helmholtz")
    np.testing.assert_allclose(fa.helm_matvec(g.alpha(), u, N), so.matvec("helmholtz", N, (g.alpha(),), u), rtol=1e-13, atol=1e-9)
    u = g.rhs("biharmonic")
    ref = so.matvec("biharmonic", N, (g.a(), g.b()), u)
    got = fa.bih_matvec(g.a(), g.b(), u, N)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
@pytest.mark.parametrize("N", [64, 256, 512])
def test_mixed_refinement(family, N):
    g = wl.small_grid(N, 8, kmax=256)
    coeffs = g.coefficients(family)
    f = g.rhs(family)
    u, u0, iters, conv = fa.refine_solve(family, coeffs, f, N)
    ref = so.solve(family, N, coeffs, f)
    e0 = so.rel_err_per_system(u0, ref).max()
    e = so.rel_err_per_system(u, ref).max()
    assert e < 1e-12, (e0, e, iters)
    assert conv.all()
    assert iters.max() <= 6


@pytest.mark.parametrize("family", ["biharmonic", "helmholtz"])
def test_roundoff_like_paper(family):
    """Sec. 5 protocol with the O(N) algorithm: within 4x of the paper's table (N <= 256)."""
    table = _roundoff_table()
    solver = {
        "helmholtz": lambda fam, N, c, f: fa.helmholtz_solve(c[0], f, N),
        "biharmonic": lambda fam, N, c, f: fa.biharmonic_solve(c[0], c[1], f, N),
    }[family]
    for N in (64, 128, 256):
        for z in (0, 200, 1800, 5400):
            e = roundoff_protocol(solver, family, N, z, runs=16)
            assert e <= 4 * table[(family, z)][N], (N, z, e)
