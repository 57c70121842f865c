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
def test_one_call_in_place_with_workspace(dev, family):
    """An in-place one-call solve given a workspace (opts.work) runs on the wave kernels (a factor
    call into the workspace, then the factored solve in place): bitwise the out-of-place result,
    at ragged and tiled N, GC and GL.  A workspace too small is refused before any launch; without
    one the in-place call takes the lane-per-chain kernels and meets the same bar."""
    from paper_1701_03787_amd import api, _lib
    fn = api.helmholtz_solve if family == "helmholtz" else api.biharmonic_solve
    for N, quad in ((130, "gc"), (512, "gc"), (512, "gl"), (1024, "gc")):
        g = wl.small_grid(N, 37, kmax=362, index=N + 12, nu=5e-5, dt=5e-4)
        csn = g.coefficients(family)
        cs = [T(c, dev) for c in csn]
        fh = g.rhs(family)
        case(test="inplace_work", family=family, N=N, quad=quad)
        ref = fn(T(fh, dev), *cs, quad=quad)
        work = torch.empty(g.nsys * api.factor_bytes(family, N) // 8, dtype=torch.float64, device=dev)
        f = T(fh, dev)
        u = fn(f, *cs, out=f, quad=quad, work=work)
        torch.cuda.synchronize()
        assert u.data_ptr() == f.data_ptr()
        assert torch.equal(f, ref)
        qo = so.GL if quad == "gl" else so.GC
        assert so.rel_err_per_system(f.cpu().numpy(), so.solve(family, N, csn, fh, quad=qo)).max() <= TOL
        with pytest.raises(_lib.ShenError):
            fn(f, *cs, out=f, quad=quad, work=work[: work.numel() // 2])
        f2 = T(fh, dev)
        fn(f2, *cs, out=f2, quad=quad)  # no workspace: lane-per-chain kernels
        torch.cuda.synchronize()
        assert so.rel_err_per_system(f2.cpu().numpy(), so.solve(family, N, csn, fh, quad=qo)).max() <= TOL


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
    f = T(g.rhs("biharmonic"), dev)
    with pytest.raises(ValueError):  # a bare state tensor carries no configuration
        api.biharmonic_solve_factored(f, cs[0], cs[1], fac.data)
    with pytest.raises(ValueError):  # a truncated state
        api.biharmonic_solve_factored(f, cs[0], cs[1], api.ShenFactor(fac.data[:, :-1].contiguous(), "biharmonic", 64,
                                                                      "gc", 0))
    with pytest.raises(ValueError):  # made for GC, asked for GL
        api.biharmonic_solve_factored(f, cs[0], cs[1], fac, quad="gl")
    with pytest.raises(ValueError):  # made with the automatic chunk, asked for another
        api.biharmonic_solve_factored(f, cs[0], cs[1], fac, chunk=8)
    fh = api.helmholtz_factor(cs[0], 64)
    with pytest.raises(ValueError):  # another family
        api.biharmonic_solve_factored(f, cs[0], cs[1], fh)


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_factored_info_codes(dev, family):
    """A non-finite coefficient: the factored solve reports the same per-system status as the
    one-call solve (pivot row + 1) and leaves the other systems of the wavefront intact."""
    from paper_1701_03787_amd import api
    N, nsys = 512, 6
    g = wl.small_grid(N, nsys, kmax=362, index=9)
    csn = [c.copy() for c in g.coefficients(family)]
    csn[0][2] = np.nan
    cs = [T(c, dev) for c in csn]
    fn = g.rhs(family)
    f = T(fn, dev)
    case(test="factored_info", family=family)
    fac = _factor(api, family, N, cs, "gc", 0)
    u, info = _solve_fac(api, family, f, cs, fac, info=True)
    u1, info1 = _solve(api, family, f, cs, info=True)
    torch.cuda.synchronize()
    expect = np.zeros(nsys, np.int32)
    expect[2] = 1
    assert np.array_equal(info.cpu().numpy(), expect)
    assert np.array_equal(info1.cpu().numpy(), expect)
    ok = np.arange(nsys) != 2
    ref = so.solve(family, N, tuple(c[ok] for c in csn), fn[ok])
    assert so.rel_err_per_system(u.cpu().numpy()[ok], ref).max() <= TOL


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
@pytest.mark.parametrize("N", [65, 512, 1024])
def test_adjoint_factored_matches_walking_adjoint(dev, family, N):
    """The adjoint from the forward factor's states is bitwise the adjoint that walks itself, and
    may run in place (lambda = gbar)."""
    from paper_1701_03787_amd import api
    g = wl.small_grid(N, 31, kmax=300, index=N + 5)
    csn = g.coefficients(family)
    cs = [T(c, dev) for c in csn]
    n = wl.n_unknowns(family, N)
    gun = wl.random_vector((g.nsys, N), (N, 3))
    gun[:, n:] = 0
    case(test="adjoint_factored", family=family, N=N)
    u_ref, lam_ref, grads_ref = so.solve_grads(family, N, csn, g.rhs(family), gun)
    u = T(u_ref, dev)
    gu = T(gun, dev)
    fac = _factor(api, family, N, cs, "gc", 0)
    adj = api.helmholtz_adjoint if family == "helmholtz" else api.biharmonic_adjoint
    r0 = adj(u, gu, *cs)
    r1 = adj(u, gu, *cs, fac=fac)
    torch.cuda.synchronize()
    for a, b in zip(r0, r1):
        assert torch.equal(a, b)
    assert so.rel_err_per_system(r1[0].cpu().numpy(), lam_ref).max() <= TOL
    # a coefficient gradient -Re sum_k conj(lam_k) (M u)_k can cancel: its attainable accuracy is
    # relative to sum_k |lam_k| |(M u)_k|
    op = so.Operators.get(N)
    mats = [op.Bd] if family == "helmholtz" else [op.Ab, op.Bb]
    for gg, gr, M in zip(r1[1:], grads_ref, mats):
        scale = np.sum(np.abs(lam_ref[:, :n]) * np.abs(np.einsum("kj,wj->wk", M, u_ref[:, :n])), axis=1)
        assert np.max(np.abs(gg.cpu().numpy() - gr) / scale) <= 1e-12
    # in place: lambda overwrites gbar (the binding allocates lambda, so call the ABI directly)
    import ctypes as C
    from paper_1701_03787_amd import _lib as L
    g2 = gu.clone()
    o = api._opts(dev)
    nsys = g.nsys
    if family == "helmholtz":
        rc = L.lib().helmholtz_adjoint_factored(N, nsys, cs[0].data_ptr(), fac.data_ptr(), None, g2.data_ptr(),
                                                g2.data_ptr(), None, C.byref(o))
    else:
        rc = L.lib().biharmonic_adjoint_factored(N, nsys, cs[0].data_ptr(), cs[1].data_ptr(), fac.data_ptr(), None,
                                                 g2.data_ptr(), g2.data_ptr(), None, None, C.byref(o))
    assert rc == 0
    torch.cuda.synchronize()
    assert torch.equal(g2, r0[0])
