"""GPU parity: the HIP library (through the C-ABI) against the CPU oracle.

Bar: per-system relative max-norm error <= 1e-12 (the accuracy target of the
plain and refined paths); bit-exact for integer outputs (info codes) and for
the zero tail.
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


def gpu_solve(family, N, coeffs, f, dev, **kw):
    from paper_1701_03787_amd import api
    ft = T(f, dev)
    cs = [T(c, dev) for c in coeffs]
    if family == "helmholtz":
        out = api.helmholtz_solve(ft, cs[0], **kw)
    else:
        out = api.biharmonic_solve(ft, cs[0], cs[1], **kw)
    torch.cuda.synchronize()
    if isinstance(out, tuple):
        return tuple(x.cpu().numpy() for x in out)
    return out.cpu().numpy()


def _print_case(**kw):
    print("CASE " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


SMALL_N = {
    "helmholtz": [3, 4, 5, 6, 7, 8, 9, 10, 17, 33, 64, 65, 128, 255, 256, 257, 512, 1024],
    "biharmonic": [5, 6, 7, 8, 9, 10, 11, 12, 17, 33, 64, 65, 128, 255, 256, 257, 512, 1024],
}


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
@pytest.mark.parametrize("gl", [False, True])
@pytest.mark.parametrize("variant", ["auto", "chain"])
def test_parity_sizes(dev, family, gl, variant):
    """Every small and ragged N, tiles that do not divide nsys, GC and GL, both kernel families."""
    for N in SMALL_N[family]:
        for nsys in (1, 3, 37):
            _print_case(test="sizes", family=family, N=N, nsys=nsys, gl=gl, variant=variant)
            g = wl.small_grid(N, nsys, kmax=200, index=N)
            coeffs = g.coefficients(family)
            f = g.rhs(family)
            quad = so.GL if gl else so.GC
            ref = so.solve(family, N, coeffs, f, quad=quad)
            u = gpu_solve(family, N, coeffs, f, dev, quad="gl" if gl else "gc", variant=variant)
            n = wl.n_unknowns(family, N)
            assert np.all(u[:, n:] == 0)
            e = so.rel_err_per_system(u, ref)
            assert e.max() <= TOL, (N, nsys, e.max())


def test_config1_full(dev):
    g = wl.config_grids(1)[0]
    _print_case(test="config1", N=g.N, nsys=g.nsys)
    f = g.rhs("helmholtz")
    ref = so.helmholtz_solve(g.N, g.alpha(), f)
    u = gpu_solve("helmholtz", g.N, (g.alpha(),), f, dev)
    assert so.rel_err_per_system(u, ref).max() <= TOL


@pytest.mark.parametrize("config", [2, 3, 5])
@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
@pytest.mark.parametrize("variant", ["auto", "chain"])
def test_config_full_size_sampled(dev, config, family, variant):
    """Full-size launch (the bench's launch configuration for config 3); the oracle checks a
    sample of systems (first, last, K2 = 0, the largest K2, and random rows)."""
    g = wl.config_grids(config)[0]
    _print_case(test="config", config=config, family=family, N=g.N, nsys=g.nsys, variant=variant)
    coeffs = g.coefficients(family)
    f = g.rhs(family)
    u = gpu_solve(family, g.N, coeffs, f, dev, variant=variant)
    rng = np.random.default_rng([1701, config, 3])
    K2 = g.K2
    rows = np.unique(np.concatenate([[0, g.nsys - 1, int(np.argmin(K2)), int(np.argmax(K2))],
                                     rng.choice(g.nsys, 60, replace=False)]))
    ref = so.solve(family, g.N, tuple(c[rows] for c in coeffs), f[rows])
    e = so.rel_err_per_system(u[rows], ref)
    assert e.max() <= TOL, e.max()
    n = wl.n_unknowns(family, g.N)
    assert np.all(u[:, n:] == 0)
    assert np.all(np.isfinite(u))


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_in_place_tail_and_determinism(dev, family):
    from paper_1701_03787_amd import api
    N, nsys = 130, 45
    g = wl.small_grid(N, nsys)
    coeffs = g.coefficients(family)
    f = g.rhs(family)
    n = wl.n_unknowns(family, N)
    fbad = f.copy()
    fbad[:, n:] = np.nan  # entries k >= n must not be read
    ref = so.solve(family, N, coeffs, f)
    _print_case(test="inplace", family=family, N=N, nsys=nsys)
    ft = T(fbad, dev)
    cs = [T(c, dev) for c in coeffs]
    if family == "helmholtz":
        u1 = api.helmholtz_solve(ft, cs[0])
        api.helmholtz_solve(ft, cs[0], out=ft)  # in place
        u2 = api.helmholtz_solve(T(fbad, dev), cs[0])
    else:
        u1 = api.biharmonic_solve(ft, cs[0], cs[1])
        api.biharmonic_solve(ft, cs[0], cs[1], out=ft)
        u2 = api.biharmonic_solve(T(fbad, dev), cs[0], cs[1])
    torch.cuda.synchronize()
    u1, u2, u3 = u1.cpu().numpy(), u2.cpu().numpy(), ft.cpu().numpy()
    assert np.all(u1[:, n:] == 0) and np.all(u3[:, n:] == 0)
    assert so.rel_err_per_system(u1, ref).max() <= TOL
    assert np.array_equal(u1.view(np.uint64), u2.view(np.uint64))  # bitwise rerun
    assert so.rel_err_per_system(u3, ref).max() <= TOL  # in place (chain kernels)


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_info_codes(dev, family):
    N, nsys = 40, 6
    g = wl.small_grid(N, nsys)
    coeffs = [c.copy() for c in g.coefficients(family)]
    coeffs[0][2] = np.nan  # first pivot of system 2 is NaN
    f = g.rhs(family)
    _print_case(test="info", family=family)
    u, info = gpu_solve(family, N, coeffs, f, dev, info=True)
    expect = np.zeros(nsys, np.int32)
    expect[2] = 1
    assert np.array_equal(info, expect)
    ok = np.arange(nsys) != 2
    ref = so.solve(family, N, tuple(c[ok] for c in coeffs), f[ok])
    assert so.rel_err_per_system(u[ok], ref).max() <= TOL


def _singular_batch(family, N):
    """Six regular channel systems, with system 2 made singular in the leading block of row 10's
    chain (a mid-chain zero pivot) and system 4 singular as a whole (its last odd or even row);
    the coefficients come from the oracle (minus a generalised eigenvalue, polished)."""
    g = wl.small_grid(N, 6, kmax=64, index=41)
    coeffs = [c.copy() for c in g.coefficients(family)]
    n = wl.n_unknowns(family, N)
    rows = {2: 10, 4: n - 1}
    for w, k in rows.items():
        if family == "helmholtz":
            coeffs[0][w] = so.singular_coefficient(family, N, k)
        else:
            coeffs[0][w] = -1000.0 if w == 2 else 0.0
            coeffs[1][w] = so.singular_coefficient(family, N, k, a=coeffs[0][w])
    expect = np.zeros(6, np.int32)
    for w, k in rows.items():
        expect[w] = k + 1
    return g, coeffs, g.rhs(family), expect


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
@pytest.mark.parametrize("variant", ["auto", "chain"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_info_singular(dev, family, variant, precision):
    """A coefficient at minus a generalised eigenvalue (oracle): the unpivoted LU meets a
    numerically zero pivot at the last row of the singular block; info reports that row + 1
    (FP32 + refinement: after its FP64 re-solve), the kernel exits normally, and the regular
    systems of the batch still match the oracle.

    FP32 + refinement and the mid-chain case (system 2, whose whole matrix is regular): FP32
    rounding moves that pivot off zero, so the FP32 LU may not meet it as unusable; the
    FP64-residual refinement then either converges to the solution of the regular system
    (info 0, and the result must meet the bar) or stalls and the FP64 re-solve reports the
    pivot (info 11)."""
    N = 40
    g, coeffs, f, expect = _singular_batch(family, N)
    _print_case(test="info_singular", family=family, variant=variant, precision=precision)
    u, info = gpu_solve(family, N, coeffs, f, dev, info=True, variant=variant, precision=precision)
    ok = expect == 0
    if precision == "fp32_refine":
        assert info[2] in (0, expect[2]), info
        if info[2] == 0:
            ok[2] = True
        keep = np.ones(6, bool)
        keep[2] = False
        assert np.array_equal(info[keep], expect[keep]), (info, expect)
    else:
        assert np.array_equal(info, expect), (info, expect)
    ref = so.solve(family, N, tuple(c[ok] for c in coeffs), f[ok])
    assert so.rel_err_per_system(u[ok], ref).max() <= TOL


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_info_singular_factored(dev, family):
    """The same per-system status from the factor-once form (the pivots are re-derived from the
    factor call's restart states)."""
    from paper_1701_03787_amd import api
    N = 40
    g, coeffs, f, expect = _singular_batch(family, N)
    cs = [T(c, dev) for c in coeffs]
    _print_case(test="info_singular_factored", family=family)
    if family == "helmholtz":
        fac = api.helmholtz_factor(cs[0], N)
        u, info = api.helmholtz_solve_factored(T(f, dev), cs[0], fac, info=True)
    else:
        fac = api.biharmonic_factor(cs[0], cs[1], N)
        u, info = api.biharmonic_solve_factored(T(f, dev), cs[0], cs[1], fac, info=True)
    torch.cuda.synchronize()
    assert np.array_equal(info.cpu().numpy(), expect)


def test_empty_batch(dev):
    from paper_1701_03787_amd import api
    f = torch.zeros((0, 32), dtype=torch.complex128, device=dev)
    a = torch.zeros((0,), dtype=torch.float64, device=dev)
    assert api.helmholtz_solve(f, a).shape == (0, 32)
    assert api.biharmonic_solve(f, a, a).shape == (0, 32)


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_wave_variant_rules(dev, family):
    """The register-resident path refuses in-place calls (it parks restart states in u)
    and the two kernel families give the same answers to the 1e-12 bar."""
    from paper_1701_03787_amd import api, _lib
    N, nsys = 512, 9
    g = wl.small_grid(N, nsys)
    coeffs = g.coefficients(family)
    f = g.rhs(family)
    ft = T(f, dev)
    cs = [T(c, dev) for c in coeffs]
    fn = api.helmholtz_solve if family == "helmholtz" else api.biharmonic_solve
    with pytest.raises(_lib.ShenError):
        fn(ft, *cs, out=ft, variant="wave")
    uw = fn(ft, *cs, variant="wave")
    uc = fn(ft, *cs, variant="chain")
    torch.cuda.synchronize()
    e = so.rel_err_per_system(uw.cpu().numpy(), uc.cpu().numpy())
    assert e.max() <= TOL


# chunk lengths the wave kernels are built with, per family: (chunk, the N it covers)
# (restart states must fit in one output row, so short rows take short chunks only)
CHUNK_CASES = {
    "helmholtz": [(4, (16, 33, 64)), (8, (17, 65, 130, 257, 512)), (16, (33, 130, 257, 512, 1024))],
    "biharmonic": [(8, (64, 100, 128, 512)), (16, (65, 130, 257, 512, 1024))],
}


@pytest.mark.parametrize("family,ci", [(fam, i) for fam, cases in CHUNK_CASES.items() for i in range(len(cases))])
def test_wave_chunk_knob(dev, family, ci):
    """Every chunk length the wave kernels offer gives the oracle's answer, over ragged N and at the
    channel size (the knob only changes the lane/chunk split)."""
    chunk, Ns = CHUNK_CASES[family][ci]
    for N in Ns:
        nsys = 37
        _print_case(test="chunk", family=family, N=N, nsys=nsys, chunk=chunk)
        g = wl.small_grid(N, nsys, kmax=200, index=N)
        coeffs = g.coefficients(family)
        f = g.rhs(family)
        ref = so.solve(family, N, coeffs, f)
        u = gpu_solve(family, N, coeffs, f, dev, variant="wave", chunk=chunk)
        assert np.all(u[:, wl.n_unknowns(family, N):] == 0)
        e = so.rel_err_per_system(u, ref)
        assert e.max() <= TOL, (N, chunk, e.max())


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_wave_chunk_refused(dev, family):
    """A chunk length no configuration of (family, N) is built with is refused (SHEN_EINVAL)
    instead of silently replaced, by the solve and by the factor call."""
    from paper_1701_03787_amd import _lib, api
    cases = ([(512, 4), (9, 4), (1024, 8), (64, 12)] if family == "helmholtz"
             else [(512, 4), (65, 8), (1024, 8), (128, 12)])
    for N, chunk in cases:
        g = wl.small_grid(N, 3)
        cs = [T(c, dev) for c in g.coefficients(family)]
        f = T(g.rhs(family), dev)
        fn = api.helmholtz_solve if family == "helmholtz" else api.biharmonic_solve
        with pytest.raises(_lib.ShenError) as ei:
            fn(f, *cs, chunk=chunk)
        assert ei.value.code == _lib.SHEN_EINVAL, (N, chunk)
        with pytest.raises(_lib.ShenError) as ei:
            api.factor_bytes(family, N, chunk=chunk)
        assert ei.value.code == _lib.SHEN_EINVAL, (N, chunk)


def test_streams(dev):
    """Calls enqueue on torch's current stream: two solves on two side streams (default
    priority) overlap with each other and with host work, and each matches the oracle."""
    N = 512
    g = wl.small_grid(N, 48, kmax=362, index=77, nu=5e-5, dt=5e-4)
    from paper_1701_03787_amd import api
    fams = ("helmholtz", "biharmonic")
    host = {fam: (g.rhs(fam), g.coefficients(fam)) for fam in fams}
    dev_in = {fam: (T(host[fam][0], dev), [T(c, dev) for c in host[fam][1]]) for fam in fams}
    torch.cuda.synchronize()
    streams = {fam: torch.cuda.Stream(device=dev) for fam in fams}
    out = {}
    _print_case(test="streams", N=N, nsys=g.nsys)
    for fam in fams:
        with torch.cuda.stream(streams[fam]):
            f, cs = dev_in[fam]
            fn = api.helmholtz_solve if fam == "helmholtz" else api.biharmonic_solve
            out[fam] = fn(f, *cs)
    for fam in fams:
        streams[fam].synchronize()
        ref = so.solve(fam, N, host[fam][1], host[fam][0])
        assert so.rel_err_per_system(out[fam].cpu().numpy(), ref).max() <= TOL


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
def test_maximum_n(dev, family):
    """The largest N the library accepts on this device (shen_max_n: the chain kernels beyond the
    wave kernels' 1024) solves to the FP64 bar; one more is refused before any launch."""
    from paper_1701_03787_amd import _lib, api
    fam = _lib.SHEN_HELMHOLTZ if family == "helmholtz" else _lib.SHEN_BIHARMONIC
    nmax = int(_lib.lib().shen_max_n(fam, _lib.SHEN_FP64))
    assert nmax > 1024
    nsys = 3
    _print_case(test="max_n", family=family, N=nmax, nsys=nsys)
    g = wl.small_grid(nmax, nsys, kmax=200, index=5)
    coeffs = g.coefficients(family)
    f = g.rhs(family)
    ref = so.solve(family, nmax, coeffs, f)
    u = gpu_solve(family, nmax, coeffs, f, dev)
    assert so.rel_err_per_system(u, ref).max() <= TOL
    assert np.all(u[:, wl.n_unknowns(family, nmax):] == 0)
    g1 = wl.small_grid(nmax + 1, 1, index=6)
    fn = api.helmholtz_solve if family == "helmholtz" else api.biharmonic_solve
    with pytest.raises(_lib.ShenError):
        fn(T(g1.rhs(family), dev), *[T(c, dev) for c in g1.coefficients(family)])
