"""GPU parity of the large-N wave solves (1024 < N <= 8192: chains spread over the wavefronts of
one work group, the scans carried across them through LDS; both parity chains of a system per work
group up to N = 4096, one chain per work group past it) against the oracle, and against the
lane-per-chain kernels where those serve the same N.

Bars: per-system relative max-norm error <= 1e-12 against the oracle (the solves' bar), zero
tail and info bit-exact; the Sec. 5 roundoff protocol within 4x of the paper's table at its
largest columns (N = 2048, 4096), where no other kernel of this library reaches the biharmonic.
"""
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


def solve(family, coeffs, f, dev, **kw):
    from paper_1701_03787_amd import api
    fn = api.helmholtz_solve if family == "helmholtz" else api.biharmonic_solve
    out = fn(T(f, dev), *[T(c, dev) for c in coeffs], **kw)
    torch.cuda.synchronize()
    if isinstance(out, tuple):
        return tuple(x.cpu().numpy() for x in out)
    return out.cpu().numpy()


# two parities per work group: 2, 3 and 4 wavefronts, ragged and exact fills of the last one;
# one parity per work group: 3 and 4 wavefronts (6 and 8 segments), ragged and exact
SIZES = (1025, 1537, 2048, 2049, 3001, 4096, 4097, 6143, 8192)


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_large_n_vs_oracle(dev, family):
    for N in SIZES:
        nsys = 3 if N <= 2049 else 2
        for quad in ("gc", "gl") if N in (1537, 4096, 8192) else ("gc",):
            case(test="large_n", family=family, N=N, nsys=nsys, quad=quad)
            g = wl.small_grid(N, nsys, kmax=362, index=N, nu=5e-5, dt=5e-4)
            cs = g.coefficients(family)
            f = g.rhs(family)
            qo = so.GL if quad == "gl" else so.GC
            ref = so.solve(family, N, cs, f, quad=qo)
            u, info = solve(family, cs, f, dev, quad=quad, info=True)
            assert np.all(info == 0)
            n = wl.n_unknowns(family, N)
            assert np.all(u[:, n:] == 0)
            e = so.rel_err_per_system(u, ref)
            assert e.max() <= TOL, (N, quad, e.max())


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_large_n_vs_chain_kernels(dev, family):
    """Many systems (K2 over the whole channel range, 0 included) on both paths; where the
    lane-per-chain kernels also serve N, the two agree to twice the bar (each is within the bar
    of the exact solution), and sampled rows match the oracle."""
    from paper_1701_03787_amd import _lib
    for N in (1100, 2000, 2900, 4500):
        g = wl.small_grid(N, 97, kmax=362, index=N + 1, nu=5e-5, dt=5e-4)
        cs = g.coefficients(family)
        f = g.rhs(family)
        case(test="large_n_chain", family=family, N=N, nsys=g.nsys)
        a = solve(family, cs, f, dev)
        try:
            b = solve(family, cs, f, dev, variant="chain")
        except _lib.ShenError:
            continue  # N past the chain kernels on this device
        # two results each within TOL of the exact solution differ by at most 2 TOL
        assert so.rel_err_per_system(a, b).max() <= 2 * TOL
        rows = np.array([0, int(np.argmax(g.K2)), g.nsys - 1])
        ref = so.solve(family, N, tuple(c[rows] for c in cs), f[rows])
        assert so.rel_err_per_system(a[rows], ref).max() <= TOL


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
@pytest.mark.parametrize("N", [2049, 4500])
def test_large_n_info(dev, family, N):
    """info in both large-N layouts (N = 4500: written by the walk, which checks every pivot).
    System 1 is singular in the leading block of row 11's chain, an odd row (oracle: minus a
    generalised eigenvalue, polished), so its pivot at row 11 is unusable: info 12, the lower of
    the two chains' first bad rows.  System 2 has a non-finite coefficient: row 0, info 1.  The
    others solve to the bar."""
    g = wl.small_grid(N, 4, kmax=200, index=9)
    cs = [c.copy() for c in g.coefficients(family)]
    if family == "helmholtz":
        cs[0][1] = so.singular_coefficient(family, N, 11)
    else:
        cs[0][1] = -1000.0
        cs[1][1] = so.singular_coefficient(family, N, 11, a=-1000.0)
    cs[0][2] = np.nan
    f = g.rhs(family)
    case(test="large_n_info", family=family, N=N)
    u, info = solve(family, cs, f, dev, info=True)
    assert list(info) == [0, 12, 1, 0]
    ok = np.array([0, 3])
    ref = so.solve(family, N, tuple(c[ok] for c in cs), f[ok])
    assert so.rel_err_per_system(u[ok], ref).max() <= TOL


@pytest.mark.parametrize("family", ["biharmonic", "helmholtz"])
def test_roundoff_protocol_large_n(dev, family):
    """Sec. 5 protocol at the table's largest columns (N = 2048, 4096): within 4x of the paper."""
    from test_oracle_solutions import _roundoff_table, roundoff_protocol
    table = _roundoff_table()

    def solver(fam, N, c, f):
        return solve(fam, c, f, dev)

    worst = []
    for N in (2048, 4096):
        for z in (0, 200, 1800, 5400):
            case(test="roundoff_large", family=family, N=N, z=z)
            e = roundoff_protocol(solver, family, N, z, runs=8)
            worst.append((e / table[(family, z)][N], N, z, e))
    print("roundoff ratios to the paper:", sorted(worst)[-4:], flush=True)
    assert max(w[0] for w in worst) <= 4.0, sorted(worst)[-3:]


def test_large_n_refusals(dev):
    """Past 8192 the biharmonic has no kernel here (the lane-per-chain kernels stop earlier);
    a chunk length is not a knob of the large-N path; the other forms stay on the lane-per-chain
    kernels there (no FP32 + refinement biharmonic at 4500)."""
    from paper_1701_03787_amd import _lib, api
    g = wl.small_grid(8193, 1, index=3)
    with pytest.raises(_lib.ShenError):
        api.biharmonic_solve(T(g.rhs("biharmonic"), dev), *[T(c, dev) for c in g.coefficients("biharmonic")])
    g = wl.small_grid(4500, 1, index=3)
    with pytest.raises(_lib.ShenError):
        api.biharmonic_solve(T(g.rhs("biharmonic"), dev), *[T(c, dev) for c in g.coefficients("biharmonic")],
                             precision="fp32_refine")
    g = wl.small_grid(2048, 1, index=4)
    with pytest.raises(_lib.ShenError):
        api.helmholtz_solve(T(g.rhs("helmholtz"), dev), T(g.coefficients("helmholtz")[0], dev), chunk=16)


def test_batched_with_large_n_grids(dev):
    """The batched form with grids past N = 1024 next to one-wavefront grids: the large-N grids
    take their own walk and solve; eager result against the oracle on sampled rows, and three
    graph replays equal to it bit for bit."""
    from paper_1701_03787_amd.batched import BatchedProblem, BatchedSolver
    grids = [wl.small_grid(N, ns, index=20 + i, kmax=200)
             for i, (N, ns) in enumerate([(4096, 3), (512, 40), (2050, 5), (5000, 2)])]
    case(test="batched_large_n")
    probs, host = [], []
    for g in grids:
        for fam in ("helmholtz", "biharmonic"):
            f = g.rhs(fam)
            cs = g.coefficients(fam)
            probs.append(BatchedProblem(fam, T(f, dev), [T(c, dev) for c in cs]))
            rows = np.array([0, g.nsys - 1])
            host.append((g, fam, f[rows], tuple(c[rows] for c in cs), rows))
    s = BatchedSolver(probs)
    cfg = s.configurations()
    assert cfg["biharmonic|4096"]["C"] is None  # no wave configuration to tune there
    s.run()
    torch.cuda.synchronize()
    for p, (g, fam, f, cs, rows) in zip(probs, host):
        ref = so.solve(fam, g.N, cs, f)
        assert so.rel_err_per_system(p.u.cpu().numpy()[rows], ref).max() <= TOL, (g.name, fam)
        assert np.all(p.u.cpu().numpy()[:, wl.n_unknowns(fam, g.N):] == 0)
    eager = [p.u.clone() for p in probs]
    s.capture()
    for r in range(3):
        for p in probs:
            p.u.zero_()
        torch.cuda.synchronize()
        s.replay()
        torch.cuda.synchronize()
        for p, e in zip(probs, eager):
            assert torch.equal(p.u, e), r


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_large_n_factored_and_in_place(dev, family):
    """Factor once / solve many past N = 1024 in both layouts (N = 2049: two parity chains per work
    group; N = 4500 and 8192: one per work group, info parked by the factor call): the factored solve,
    out of place and in place, and the one-call in-place solve through a workspace are bitwise the
    one-call out-of-place solve, info included (a singular system at odd row 11, a non-finite one).
    The adjoint has no factored form there and says so."""
    from paper_1701_03787_amd import _lib, api
    for N in (2049, 4500, 8192):
        g = wl.small_grid(N, 4, kmax=200, index=N + 7)
        cs = [c.copy() for c in g.coefficients(family)]
        if family == "helmholtz":
            cs[0][1] = so.singular_coefficient(family, N, 11)
        else:
            cs[0][1] = -1000.0
            cs[1][1] = so.singular_coefficient(family, N, 11, a=-1000.0)
        cs[0][2] = np.inf
        case(test="large_n_factored", family=family, N=N)
        f = T(g.rhs(family), dev)
        ct = [T(c, dev) for c in cs]
        solve = api.helmholtz_solve if family == "helmholtz" else api.biharmonic_solve
        ref, rinfo = solve(f, *ct, info=True)
        if family == "helmholtz":
            fac = api.helmholtz_factor(ct[0], N)
            u, info = api.helmholtz_solve_factored(f, ct[0], fac, info=True)
            x = f.clone()
            _, info2 = api.helmholtz_solve_factored(x, ct[0], fac, out=x, info=True)
        else:
            fac = api.biharmonic_factor(*ct, N)
            u, info = api.biharmonic_solve_factored(f, *ct, fac, info=True)
            x = f.clone()
            _, info2 = api.biharmonic_solve_factored(x, *ct, fac, out=x, info=True)
        y = f.clone()
        work = torch.empty(g.nsys * api.factor_bytes(family, N) // 8, dtype=torch.float64, device=dev)
        _, info3 = solve(y, *ct, out=y, work=work, info=True)
        torch.cuda.synchronize()
        assert list(rinfo.cpu().numpy()) == [0, 12, 1, 0]
        for got, gi in ((u, info), (x, info2), (y, info3)):
            assert torch.equal(gi, rinfo)
            ok = torch.tensor([0, 3], device=dev)
            assert torch.equal(got[ok], ref[ok])
        adj = api.helmholtz_adjoint if family == "helmholtz" else api.biharmonic_adjoint
        with pytest.raises(_lib.ShenError) as ei:
            adj(ref, f, *ct, fac=fac)
        assert ei.value.code == _lib.SHEN_ENOTSUP


@pytest.mark.parametrize("family,N", [("helmholtz", 2049), ("helmholtz", 4500), ("biharmonic", 2049)])
def test_large_n_autograd(dev, family, N):
    """The differentiable solves past N = 1024: the forward solve on the large-N wave kernels (no
    factor there), the backward pass on the lane-per-chain adjoint, against the oracle's gradients
    (lambda = H^-T gu to the solves' bar, the coefficient gradients to 1e-10 relative)."""
    from paper_1701_03787_amd import api
    g = wl.small_grid(N, 2, kmax=200, index=N + 11)
    cs = g.coefficients(family)
    f = g.rhs(family)
    gu = wl.random_vector((g.nsys, N), (N, 3))
    gu[:, wl.n_unknowns(family, N):] = 0
    case(test="large_n_autograd", family=family, N=N)
    u_ref, lam_ref, grads_ref = so.solve_grads(family, N, cs, f, gu)
    ft = T(f, dev).requires_grad_(True)
    ct = [T(c, dev).requires_grad_(True) for c in cs]
    u = api.helmholtz(ft, *ct) if family == "helmholtz" else api.biharmonic(ft, *ct)
    torch.autograd.backward([torch.view_as_real(u)], [torch.view_as_real(T(gu, dev))])
    torch.cuda.synchronize()
    assert so.rel_err_per_system(u.detach().cpu().numpy(), u_ref).max() <= TOL
    assert so.rel_err_per_system(ft.grad.cpu().numpy(), lam_ref).max() <= TOL
    for c, gr in zip(ct, grads_ref):
        np.testing.assert_allclose(c.grad.cpu().numpy(), gr, rtol=1e-10, atol=1e-300)
