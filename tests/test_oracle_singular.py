"""Pins of oracle.singular_coefficient: the coefficients that make a leading block of the
unpivoted LU of Sec. 4 singular (the failure cases the solvers report per system).

The oracle takes minus a generalised eigenvalue of the block pair and polishes it by
bisection on the sign of det; these tests check it against what fixes it independently:
the determinant itself changes sign across it (pivoted LU of the dense block), scipy's QZ
generalised eigenvalues of the same block, and the O(N) recurrences of Sec. 4 (the CPU
prototype of the kernels), whose pivot at row k collapses there while every earlier pivot
stays of the order of its row.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import fastalg as fa
from oracle import shen_oracle as so

TINY = 2.0 ** -40  # the solvers' numerically-zero pivot threshold, relative to the row


def _helm_ratios(N, alpha):
    n = N - 2
    _, d, _, _, _ = fa.helm_factor_forward(np.array([alpha]), np.zeros((1, n), complex), N)
    hm, h0, _, _ = fa.helm_entries(np.arange(n), np.array([alpha]), N)
    return np.abs(d[0]) / (np.abs(h0[0]) + np.abs(hm[0]))


def _bih_ratios(N, a, b):
    n = N - 4
    U0 = fa.bih_factor_forward(np.array([a]), np.array([b]), np.zeros((1, n), complex), N)[0]
    sc = np.array([sum(abs(x[0]) for x in fa.bih_entries(k, np.array([a]), np.array([b]), N)[:3]) for k in range(n)])
    return np.abs(U0[0]) / sc


CASES = [("helmholtz", 40, 10, 0.0), ("helmholtz", 40, 11, 0.0), ("helmholtz", 40, 37, 0.0), ("helmholtz", 64, 60, 0.0),
         ("biharmonic", 40, 10, 0.0), ("biharmonic", 40, 13, -1000.0), ("biharmonic", 40, 35, 0.0),
         ("biharmonic", 40, 34, -1000.0)]


@pytest.mark.parametrize("family,N,k,a", CASES)
def test_singular_coefficient_pins(family, N, k, a):
    c = so.singular_coefficient(family, N, k, a=a)
    op = so.Operators.get(N)
    M0, M1 = (op.Sd, op.Bd) if family == "helmholtz" else (op.Qb + a * op.Ab, op.Bb)
    idx = so.chain_rows(k)
    A0, A1 = M0[np.ix_(idx, idx)], M1[np.ix_(idx, idx)]
    # det changes sign within 1e-13 (relative) of c (closer in, the computed sign is rounding)
    s_lo = np.linalg.slogdet(A0 + c * (1 - 1e-13) * A1)[0]
    s_hi = np.linalg.slogdet(A0 + c * (1 + 1e-13) * A1)[0]
    assert s_lo * s_hi < 0
    # minus the largest real QZ eigenvalue of the same block
    w = sla.eigvals(A0, A1)
    lam = np.max(w[np.abs(w.imag) < 1e-9 * np.abs(w)].real)
    assert abs(c + lam) <= 1e-9 * abs(lam)
    # the Sec. 4 recurrences: pivot k collapses, every earlier pivot is of the order of its row
    r = _helm_ratios(N, c) if family == "helmholtz" else _bih_ratios(N, a, c)
    assert r[k] <= TINY * 1e-1, r[k]
    assert r[:k].min() >= 1e-3, r[:k].min()


def test_singular_coefficient_full_system_is_singular():
    """With k the last row of its chain the whole matrix is singular: the smallest singular
    value of the dense system matrix is at rounding level."""
    for family, N in (("helmholtz", 40), ("biharmonic", 40)):
        n = so.n_of(family, N)
        c = so.singular_coefficient(family, N, n - 1)
        H = (so.helmholtz_matrix(N, np.array([c]))[0] if family == "helmholtz"
             else so.biharmonic_matrix(N, np.array([0.0]), np.array([c]))[0])
        sv = np.linalg.svd(H, compute_uv=False)
        assert sv[-1] <= 1e-13 * sv[0], (family, sv[-1] / sv[0])
