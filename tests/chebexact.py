"""Exact (rational) Chebyshev-series algebra, used to pin the oracle's matrices.

Every entry of the Galerkin matrices is pi times a rational number, so they
can be computed exactly from the basis definitions: a basis function is a
short Chebyshev series with rational coefficients, differentiation maps
Chebyshev coefficients to Chebyshev coefficients by the textbook recurrence,
and the discrete weighted inner product of two Chebyshev series reduces to
sum_m a_m b_m c_m pi/2 as long as quadrature is exact for the product (true
for every matrix here; for Gauss-Lobatto the single inexact product
T_{N-1} T_{N-1} is what c_{N-1} = 2 accounts for).

Independent of the oracle: nothing here reads its closed forms.
"""
from fractions import Fraction


def basis(family, k):
    """Chebyshev coefficients of the Dirichlet / biharmonic basis function k."""
    if family == "dirichlet":
        c = [Fraction(0)] * (k + 3)
        c[k] = Fraction(1)
        c[k + 2] = Fraction(-1)
        return c
    c = [Fraction(0)] * (k + 5)
    c[k] = Fraction(1)
    c[k + 2] = Fraction(-2 * (k + 2), k + 3)
    c[k + 4] = Fraction(k + 1, k + 3)
    return c


def deriv(a):
    """Coefficients of d/dx of sum a_m T_m (exact)."""
    m = len(a) - 1
    if m <= 0:
        return [Fraction(0)]
    b = [Fraction(0)] * (m + 2)
    for k in range(m, 0, -1):
        b[k - 1] = b[k + 1] + 2 * k * a[k]
    b[0] = b[0] / 2
    return b[:m]


def nderiv(a, p):
    for _ in range(p):
        a = deriv(a)
    return a


def inner_over_pi(a, b, N, gl=False):
    """(sum a_m T_m, sum b_m T_m)_sigma / pi for the N-point GC (or GL) rule."""
    s = Fraction(0)
    for m in range(min(len(a), len(b))):
        if a[m] == 0 or b[m] == 0:
            continue
        c = 2 if m == 0 else 1
        if gl and m == N - 1:
            c = 2
        s += a[m] * b[m] * Fraction(c, 2)
    return s


def matrix_over_pi(family, p, N, gl=False, sign=1):
    """Exact [k][j] = sign * (phi_j^{(p)}, phi_k)_sigma / pi."""
    n = N - 2 if family == "dirichlet" else N - 4
    phis = [basis(family, k) for k in range(n)]
    dphis = [nderiv(ph, p) for ph in phis]
    return [[sign * inner_over_pi(dphis[j], phis[k], N, gl) for j in range(n)] for k in range(n)]
