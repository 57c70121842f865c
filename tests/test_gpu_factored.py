"""GPU parity of the factor-once / solve-many form: the restart states are computed once per
set of coefficients, then every solve runs only the wave kernel.  The result must be bitwise
that of the one-call solve (same kernels, same states), and within the FP64 bar of the oracle."""
import numpy as np
import pytest

from oracle import shen_oracle as so
from paper_1701_03787_amd import workloads as wl

pytestmark = pytest.mark.gpu
TOL = 1e-12
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


def _factor(api, family, N, cs, quad, chunk):
    if family == "helmholtz":
        return api.helmholtz_factor(cs[0], N, quad=quad, chunk=chunk)
    return api.biharmonic_factor(cs[0], cs[1], N, quad=quad, chunk=chunk)


def _solve_fac(api, family, f, cs, fac, **kw):
    if family == "helmholtz":
        return api.helmholtz_solve_factored(f, cs[0], fac, **kw)
    return api.biharmonic_solve_factored(f, cs[0], cs[1], fac, **kw)


def _solve(api, family, f, cs, **kw):
    fn = api.helmholtz_solve if family == "helmholtz" else api.biharmonic_solve
    return fn(f, *cs, **kw)


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
@pytest.mark.parametrize("N", [40, 65, 130, 257, 512, 1024])
@pytest.mark.parametrize("quad", ["gc", "gl"])
def test_factored_matches_one_call_and_oracle(dev, family, N, quad):
    from paper_1701_03787_amd import api
    g = wl.small_grid(N, 29, kmax=300, index=N + 3)
    csn = g.coefficients(family)
    cs = [T(c, dev) for c in csn]
    case(test="factored", family=family, N=N, quad=quad)
    fac = _factor(api, family, N, cs, quad, 0)
    ref = so.solve(family, N, csn, g.rhs(family), quad=so.GL if quad == "gl" else so.GC)
    # solve-many: three right-hand sides against one factor
    for r in range(3):
        fn = g.rhs(family) if r == 0 else wl.random_vector((g.nsys, N), (N, 40 + r))
        if r:
            fn[:, wl.n_unknowns(family, N):] = 0
            ref = so.solve(family, N, csn, fn, quad=so.GL if quad == "gl" else so.GC)
        f = T(fn, dev)
        u, info = _solve_fac(api, family, f, cs, fac, quad=quad, info=True)
        u1 = _solve(api, family, f, cs, quad=quad)
        torch.cuda.synchronize()
        assert torch.equal(u, u1), (N, r)
        assert np.all(info.cpu().numpy() == 0)
        un = u.cpu().numpy()
        assert so.rel_err_per_system(un, ref).max() <= TOL
        assert np.all(un[:, wl.n_unknowns(family, N):] == 0)


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_factored_in_place_and_chunk(dev, family):
    """u may alias f in the factored solve; the chunk knob of the factor call is honoured."""
    from paper_1701_03787_amd import api
    N = 512
    g = wl.small_grid(N, 40, kmax=362, index=11, nu=5e-5, dt=5e-4)
    csn = g.coefficients(family)
    cs = [T(c, dev) for c in csn]
    fn = g.rhs(family)
    ref = so.solve(family, N, csn, fn)
    for chunk in (0, 8):
        case(test="factored_inplace", family=family, chunk=chunk)
        fac = _factor(api, family, N, cs, "gc", chunk)
        f = T(fn, dev)
        u = _solve_fac(api, family, f, cs, fac, out=f, chunk=chunk)
        torch.cuda.synchronize()
        assert u.data_ptr() == f.data_ptr()
        assert so.rel_err_per_system(f.cpu().numpy(), ref).max() <= TOL


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_factored_full_size_sampled(dev, family):
    """The bench workload (N=512, 512x257 wavenumbers): bitwise equal to the one-call solve on
    every system, and sampled systems against the oracle."""
    from paper_1701_03787_amd import api
    g = wl.config_grids(3)[0]
    N = g.N
    case(test="factored_full", family=family, nsys=g.nsys)
    csn = g.coefficients(family)
    cs = [T(c, dev) for c in csn]
    fn = g.rhs(family)
    f = T(fn, dev)
    fac = _factor(api, family, N, cs, "gc", 0)
    u = _solve_fac(api, family, f, cs, fac)
    u1 = _solve(api, family, f, cs)
    torch.cuda.synchronize()
    assert torch.equal(u, u1)
    del u1
    rng = np.random.default_rng([1701, 3, 17])
    rows = np.unique(np.concatenate([[0, g.nsys - 1, int(np.argmin(g.K2))], rng.choice(g.nsys, 60, replace=False)]))
    ref = so.solve(family, N, tuple(c[rows] for c in csn), fn[rows])
    assert so.rel_err_per_system(u.cpu().numpy()[rows], ref).max() <= TOL


def test_factored_rejects_mismatched_state(dev):
    from paper_1701_03787_amd import api, _lib
    # no wave configuration for the smallest N: the factor-once form is refused
    g = wl.small_grid(33, 3)
    cs = [T(c, dev) for c in g.coefficients("biharmonic")]
    with pytest.raises(_lib.ShenError):
        api.biharmonic_factor(cs[0], cs[1], 33)
    g = wl.small_grid(64, 5)
    cs = [T(c, dev) for c in g.coefficients("biharmonic")]
    fac = api.biharmonic_factor(cs[0], cs[1], 64)
    with pytest.raises(ValueError):
        api.biharmonic_solve_factored(T(g.rhs("biharmonic"), dev), cs[0], cs[1], fac[:, :-1].contiguous())
