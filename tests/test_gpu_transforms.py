"""GPU parity of the wall-normal Shen transforms (Sec. 2; appendix transform algorithms)
against the oracle's dense long-double evaluation of the basis at the points.

Bars (per system):
* scalar products: |S - S_ref|_inf <= (N + 64) eps pi max|u| -- the rounding bound of an
  N-term sum whose terms are at most max|u| pi/N times |phi| <= 4 (the FFT path's error
  is far below it);
* inverse: |u - u_ref|_inf <= (N + 64) eps 4 sum_k |uhat_k|, the same bound for the sum
  over coefficients;
* forward transform = scalar products, then the mass solve: the error of S(u), a few
  ulps relative, reaches uhat amplified by at most cond(B) (reading A16), so
  |uhat - ref|_inf <= max(1e-13, 8 log2(N) cond(B) eps) max|ref|.
"""
import numpy as np
import pytest

from oracle import shen_oracle as so
from paper_1701_03787_amd import workloads as wl

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps
SPACES = ("chebyshev", "dirichlet", "biharmonic")

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1701_03787_amd import _lib
    _lib.lib()
    return torch.device("cuda:0")


def T(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def case(**kw):
    print("CASE " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def qo(quad):
    return so.GL if quad == "gl" else so.GC


def mass_cond(space, N, quad):
    if space == "chebyshev":
        return 2.0
    return np.linalg.cond(so.mass_matrix("helmholtz" if space == "dirichlet" else "biharmonic", N, qo(quad)))


def check_scalar(got, ref, u, N):
    bound = (N + 64) * EPS * np.pi * np.max(np.abs(u), axis=1)
    err = np.max(np.abs(got - ref), axis=1)
    assert np.all(err <= bound), float(np.max(err / bound))


def check_inverse(got, ref, uh, N):
    bound = (N + 64) * EPS * 4.0 * np.sum(np.abs(uh), axis=1)
    err = np.max(np.abs(got - ref), axis=1)
    assert np.all(err <= bound), float(np.max(err / bound))


# Gauss points: powers of two take the FFT kernel, the others the direct sums;
# Gauss-Lobatto points always take the direct sums.
SIZES = {"gc": (8, 9, 16, 64, 100, 256, 512, 1024, 2048), "gl": (9, 16, 64, 100, 257)}


@pytest.mark.parametrize("quad", ["gc", "gl"])
@pytest.mark.parametrize("space", SPACES)
def test_scalar_product_and_inverse(dev, space, quad):
    from paper_1701_03787_amd import api
    for N in SIZES[quad]:
        if N < 5:
            continue
        for nsys in (1, 37):
            case(test="transform", space=space, quad=quad, N=N, nsys=nsys)
            rng = np.random.default_rng([1701, 50, N, nsys])
            u = rng.standard_normal((nsys, N)) + 1j * rng.standard_normal((nsys, N))
            got = api.scalar_product(T(u, dev), space, quad=quad).cpu().numpy()
            ref = so.scalar_product(space, N, u, qo(quad))
            check_scalar(got, ref, u, N)
            n = so.n_space(space, N)
            assert np.all(got[:, n:] == 0)
            uh = np.zeros((nsys, N), complex)
            uh[:, :n] = rng.standard_normal((nsys, n)) + 1j * rng.standard_normal((nsys, n))
            uh_in = uh.copy()
            uh_in[:, n:] = np.nan  # entries k >= n must not be read
            got = api.backward_transform(T(uh_in, dev), space, quad=quad).cpu().numpy()
            check_inverse(got, so.backward_transform(space, N, uh, qo(quad)), uh, N)


@pytest.mark.parametrize("quad", ["gc", "gl"])
@pytest.mark.parametrize("space", SPACES)
def test_forward_transform_and_round_trip(dev, space, quad):
    """Point values of a series with a decaying spectrum (the channel recipe) -> coefficients
    (scalar products then the mass solve), against the oracle; then back to the points."""
    from paper_1701_03787_amd import api
    for N in ((9, 64, 100, 256, 512, 1024) if quad == "gc" else (9, 64, 100)):
        n = so.n_space(space, N)
        g = wl.small_grid(N, 21, index=N + 7)
        uh = np.zeros((g.nsys, N), complex)
        uh[:, :n] = g.rhs("helmholtz")[:, :n]  # spectrum decaying as (k+1)^-3
        u = so.backward_transform(space, N, uh, qo(quad))
        case(test="forward", space=space, quad=quad, N=N)
        got = api.forward_transform(T(u, dev), space, quad=quad).cpu().numpy()
        ref = so.forward_transform(space, N, u, qo(quad))
        m = 8 * np.log2(N)
        bar = max(1e-13, m * mass_cond(space, N, quad) * EPS)
        err = np.max(np.abs(got - ref), axis=1) / np.max(np.abs(ref), axis=1)
        assert err.max() <= bar, (N, err.max(), bar)
        assert np.all(got[:, n:] == 0)
        back = api.backward_transform(T(got, dev), space, quad=quad).cpu().numpy()
        assert np.max(np.abs(back - u)) <= bar * np.max(np.abs(u))


@pytest.mark.parametrize("space", ["dirichlet", "biharmonic"])
def test_transforms_config3_full_size_sampled(dev, space):
    """The bench workload's shape (N=512, 131,584 systems, Gauss points): scalar products and
    inverse transforms in one launch each, sampled rows against the oracle."""
    from paper_1701_03787_amd import api
    g = wl.config_grids(3)[0]
    N, nsys = g.N, g.nsys
    case(test="transform_config3", space=space, nsys=nsys)
    fam = "helmholtz" if space == "dirichlet" else "biharmonic"
    uh = g.rhs(fam)
    ut = T(uh, dev)
    phys = api.backward_transform(ut, space)
    s = api.scalar_product(phys, space)
    torch.cuda.synchronize()
    rng = np.random.default_rng([1701, 3, 13])
    rows = np.unique(np.concatenate([[0, nsys - 1], rng.choice(nsys, 30, replace=False)]))
    idx = torch.from_numpy(rows).to(dev)
    p = phys[idx].cpu().numpy()
    check_inverse(p, so.backward_transform(space, N, uh[rows]), uh[rows], N)
    check_scalar(s[idx].cpu().numpy(), so.scalar_product(space, N, p), p, N)


def test_transform_argument_errors(dev):
    from paper_1701_03787_amd import api, _lib
    u = T(np.zeros((3, 16), complex), dev)
    with pytest.raises(ValueError):
        api.scalar_product(u, "fourier")
    with pytest.raises(ValueError):
        api.forward_transform(u, "dirichlet", out=u)  # output may not be the input
    with pytest.raises(_lib.ShenError):
        api.forward_transform(T(np.zeros((2, 2048), complex), dev), "biharmonic")  # mass solve limit N <= 1024
    with pytest.raises(_lib.ShenError):
        api.scalar_product(T(np.zeros((2, 4096), complex), dev), "chebyshev")
