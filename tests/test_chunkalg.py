"""The chunked / scanned reformulation (what the wave kernels compute) against the oracle."""
import numpy as np
import pytest

import chunkalg as ca
from oracle import shen_oracle as so
from paper_1701_03787_amd import workloads as wl


@pytest.mark.parametrize("N,C,G", [(64, 4, 8), (130, 8, 8), (512, 16, 16), (512, 8, 32), (1024, 16, 32)])
def test_chunked_helmholtz(N, C, G):
    g = wl.small_grid(N, 6, kmax=256)
    f = g.rhs("helmholtz")
    u = ca.helm_chunked(g.alpha(), f, N, C, G)
    ref = so.helmholtz_solve(N, g.alpha(), f)
    assert so.rel_err_per_system(u, ref).max() < 1e-13


@pytest.mark.parametrize("N,C,G", [(64, 4, 8), (130, 8, 8), (512, 16, 16), (512, 8, 32), (1024, 16, 32)])
def test_chunked_biharmonic(N, C, G):
    g = wl.small_grid(N, 6, kmax=256)
    f = g.rhs("biharmonic")
    u = ca.bih_chunked(g.a(), g.b(), f, N, C, G)
    ref = so.biharmonic_solve(N, g.a(), g.b(), f)
    assert so.rel_err_per_system(u, ref).max() < 1e-12


def test_chunked_roundoff_protocol():
    """Sec. 5 protocol at z = 0 and 5400 (the extremes), N = 512."""
    from test_oracle_solutions import _roundoff_table, roundoff_protocol
    table = _roundoff_table()
    for z in (0, 1800, 5400):
        e = roundoff_protocol(lambda fam, N, c, f: ca.bih_chunked(c[0], c[1], f, N, 16, 16), "biharmonic", 512, z, 4)
        assert e <= 1.5 * table[("biharmonic", z)][512], (z, e)
        e = roundoff_protocol(lambda fam, N, c, f: ca.helm_chunked(c[0], f, N, 16, 16), "helmholtz", 512, z, 4)
        assert e <= 4 * table[("helmholtz", z)][512], (z, e)
