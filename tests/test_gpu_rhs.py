"""GPU parity of the Crank-Nicolson right-hand sides (Sec. 3, eqs. gfin and ufin) against
the oracle, which forms them from the paper's unscaled matrices in extended precision.

Bar: elementwise |rhs - ref| <= (4n + 64) eps ((|M| |uhat|)_k + |sigma S(h)_k|), the
rounding bound of an n-term FP64 product with entries formed to a few ulps (M the
scaled explicit matrix, so |M| |uhat| is the size of the terms that are summed); and
normwise <= 1e-12 of max |ref| per system.  The step as a whole (right-hand side, then
the solve) is checked against the oracle's step at the solves' 1e-12 bar.
"""
import numpy as np
import pytest

from oracle import shen_oracle as so
from paper_1701_03787_amd import workloads as wl

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps

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


def gpu_rhs(family, uh, K2, nu, dt, sh, dev, **kw):
    from paper_1701_03787_amd import api
    fn = api.helmholtz_rhs if family == "helmholtz" else api.biharmonic_rhs
    out = fn(T(uh, dev), T(K2, dev), nu, dt, T(sh, dev) if sh is not None else None, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check(family, N, K2, nu, dt, uh, sh, got, quad=so.GC):
    n = so.n_of(family, N)
    ref = so.rhs_assemble(family, N, K2, nu, dt, uh, sh, quad=quad, extended=True)
    scale = (2.0 if family == "helmholtz" else -2.0) / (nu * dt)
    sigma = scale * dt
    for w in range(uh.shape[0]):
        M = np.abs(scale * so.cn_explicit_matrix_paper(family, N, float(K2[w]), nu, dt, quad))
        size = M @ np.abs(uh[w, :n])
        if sh is not None:
            size = size + abs(sigma) * np.abs(sh[w, :n])
        bound = (4 * n + 64) * EPS * size
        err = np.abs(got[w, :n] - ref[w, :n])
        assert np.all(err <= bound), (w, float(np.max(err / np.maximum(bound, 1e-300))))
        assert np.max(err) <= 1e-12 * np.max(np.abs(ref[w, :n]))
    assert np.all(got[:, n:] == 0)


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
@pytest.mark.parametrize("quad", ["gc", "gl"])
def test_rhs_vs_oracle_sizes(dev, family, quad):
    """Small and ragged N (the chain kernels) and the tiled N (wave layout), with and
    without the S(h) term, at the channel coefficient law (negative alpha', sign-changing
    a', b')."""
    nu, dt = 5e-5, 5e-4
    qo = so.GL if quad == "gl" else so.GC
    for N in (9, 64, 130, 257, 512, 1024):
        g = wl.small_grid(N, 11, kmax=362, index=N + 3)
        uh = g.rhs(family)
        sh = wl.random_vector((g.nsys, N), (N, 61))
        for with_sh in (False, True):
            case(test="rhs", family=family, N=N, quad=quad, sh=with_sh)
            got = gpu_rhs(family, uh, g.K2, nu, dt, sh if with_sh else None, dev, quad=quad)
            check(family, N, g.K2, nu, dt, uh, sh if with_sh else None, got, quad=qo)


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_rhs_chain_and_wave_agree(dev, family):
    """The two kernel families on the same N (512: both have it) to the same bar."""
    nu, dt, N = 5e-5, 5e-4, 512
    g = wl.small_grid(N, 9, kmax=362, index=77)
    uh = g.rhs(family)
    sh = wl.random_vector((g.nsys, N), (62,))
    case(test="rhs_variants", family=family)
    a = gpu_rhs(family, uh, g.K2, nu, dt, sh, dev, variant="chain")
    b = gpu_rhs(family, uh, g.K2, nu, dt, sh, dev, variant="auto")
    check(family, N, g.K2, nu, dt, uh, sh, a)
    check(family, N, g.K2, nu, dt, uh, sh, b)


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_rhs_in_place_on_sh(dev, family):
    """out = sh accumulates the result into the S(h) buffer."""
    from paper_1701_03787_amd import api
    nu, dt, N = 5e-5, 5e-4, 256
    g = wl.small_grid(N, 13, kmax=200, index=5)
    uh = g.rhs(family)
    sh = wl.random_vector((g.nsys, N), (63,))
    case(test="rhs_inplace", family=family)
    st = T(sh, dev)
    fn = api.helmholtz_rhs if family == "helmholtz" else api.biharmonic_rhs
    fn(T(uh, dev), T(g.K2, dev), nu, dt, st, out=st)
    torch.cuda.synchronize()
    check(family, N, g.K2, nu, dt, uh, sh, st.cpu().numpy())


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_rhs_config3_full_size_sampled(dev, family):
    """The bench workload (N=512, 512x257): all 131,584 systems in one launch, sampled rows
    (first, last, K2 = 0, the largest K2, random) against the oracle."""
    g = wl.config_grids(3)[0]
    uh = g.rhs(family)
    sh = wl.random_vector((g.nsys, g.N), (64,))
    case(test="rhs_config3", family=family, nsys=g.nsys)
    from paper_1701_03787_amd import api
    fn = api.helmholtz_rhs if family == "helmholtz" else api.biharmonic_rhs
    out = fn(T(uh, dev), T(g.K2, dev), g.nu, g.dt, T(sh, dev))
    torch.cuda.synchronize()
    rng = np.random.default_rng([1701, 3, 12])
    rows = np.unique(np.concatenate([[0, g.nsys - 1, int(np.argmin(g.K2)), int(np.argmax(g.K2))],
                                     rng.choice(g.nsys, 24, replace=False)]))
    got = out[torch.from_numpy(rows).to(dev)].cpu().numpy()
    check(family, g.N, g.K2[rows], g.nu, g.dt, uh[rows], sh[rows], got)
    n = wl.n_unknowns(family, g.N)
    assert torch.all(out[:, n:] == 0).item()


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_one_time_step(dev, family):
    """Right-hand side then solve on the GPU, against the oracle's step (its right-hand side
    from the paper's matrices, then its dense solve), at the solves' 1e-12 bar."""
    from paper_1701_03787_amd import api
    nu, dt, N = 5e-5, 5e-4, 512
    g = wl.small_grid(N, 17, kmax=362, index=88, nu=nu, dt=dt)
    uh = so.solve(family, N, g.coefficients(family), g.rhs(family))  # a solution-like state
    sh = wl.random_vector((g.nsys, N), (65,)) * ((np.arange(N) + 1.0) ** -3)
    case(test="rhs_step", family=family)
    rhs = (api.helmholtz_rhs if family == "helmholtz" else api.biharmonic_rhs)(T(uh, dev), T(g.K2, dev), nu, dt,
                                                                                 T(sh, dev))
    cs = [T(c, dev) for c in g.coefficients(family)]
    u1 = (api.helmholtz_solve(rhs, *cs) if family == "helmholtz" else api.biharmonic_solve(rhs, *cs))
    torch.cuda.synchronize()
    ref = so.solve(family, N, g.coefficients(family), so.rhs_assemble(family, N, g.K2, nu, dt, uh, sh))
    assert so.rel_err_per_system(u1.cpu().numpy(), ref).max() <= 1e-12
