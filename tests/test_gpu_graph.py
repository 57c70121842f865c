"""One solver step of every form in one hipGraph.

Every entry point enqueues kernels only, on the caller's stream: no allocation, no memset, no
host synchronisation.  So one graph can capture all of them together:
* the FP64 solves: one-wavefront, large-N in both layouts (N = 2049, two parity chains per work
  group; N = 4500, one per work group, with info from the walk), transposed, and in place through
  a workspace;
* the FP32 + refinement solves, with info and iteration counts;
* the factored solves and the adjoints;
* the right-hand sides and the transforms.
There are three replays, with eager work and synchronisations between them.  The inputs of the
in-place solves are restored inside the graph.  Every output of every replay must equal the
eager result bit for bit.
"""
import numpy as np
import pytest

from paper_1701_03787_amd import workloads as wl

pytestmark = pytest.mark.gpu
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


def test_every_form_in_one_graph(dev):
    from paper_1701_03787_amd import api
    print("CASE test=graph_all_forms", flush=True)
    g = wl.small_grid(512, 37, index=71)
    gl1 = wl.small_grid(2049, 3, index=72)
    gl2 = wl.small_grid(4500, 2, index=73)
    H = {fam: (T(g.rhs(fam), dev), [T(c, dev) for c in g.coefficients(fam)]) for fam in ("helmholtz", "biharmonic")}
    L1 = {fam: (T(gl1.rhs(fam), dev), [T(c, dev) for c in gl1.coefficients(fam)]) for fam in ("helmholtz", "biharmonic")}
    L2 = {fam: (T(gl2.rhs(fam), dev), [T(c, dev) for c in gl2.coefficients(fam)]) for fam in ("helmholtz", "biharmonic")}
    K2 = T(g.K2, dev)
    pts = T(wl.random_vector((g.nsys, g.N), (74,)), dev)
    fac = {"helmholtz": api.helmholtz_factor(H["helmholtz"][1][0], g.N),
           "biharmonic": api.biharmonic_factor(*H["biharmonic"][1], g.N)}
    work = torch.empty(g.nsys * max(api.factor_bytes(fam, g.N) for fam in H) // 8, dtype=torch.float64, device=dev)
    outs = {}

    def buf(name, like, dtype=None):
        if name not in outs:
            outs[name] = torch.empty(like.shape, dtype=dtype or like.dtype, device=dev)
        return outs[name]

    def ints(name, n):
        if name not in outs:
            outs[name] = torch.empty(n, dtype=torch.int32, device=dev)
        return outs[name]

    def step():
        for fam, solve in (("helmholtz", api.helmholtz_solve), ("biharmonic", api.biharmonic_solve)):
            f, cs = H[fam]
            solve(f, *cs, out=buf(f"{fam}.u", f), info=ints(f"{fam}.info", g.nsys))
            solve(f, *cs, out=buf(f"{fam}.uT", f), transpose=True)
            solve(f, *cs, out=buf(f"{fam}.mixed", f), precision="fp32_refine", info=ints(f"{fam}.minfo", g.nsys),
                  iters=ints(f"{fam}.iters", g.nsys))
            x = buf(f"{fam}.inplace", f)
            x.copy_(f)
            solve(x, *cs, out=x, work=work)
            if fam == "helmholtz":
                api.helmholtz_solve_factored(f, cs[0], fac[fam], out=buf(f"{fam}.fac", f))
                lam, ga = api.helmholtz_adjoint(outs[f"{fam}.u"], f, cs[0])
                outs[f"{fam}.lam"], outs[f"{fam}.ga"] = lam, ga
                api.helmholtz_rhs(f, K2, 5e-5, 5e-4, f, out=buf(f"{fam}.rhs", f))
            else:
                api.biharmonic_solve_factored(f, *cs, fac[fam], out=buf(f"{fam}.fac", f))
                lam, ga, gb = api.biharmonic_adjoint(outs[f"{fam}.u"], f, *cs)
                outs[f"{fam}.lam"], outs[f"{fam}.ga"], outs[f"{fam}.gb"] = lam, ga, gb
                api.biharmonic_rhs(f, K2, 5e-5, 5e-4, f, out=buf(f"{fam}.rhs", f))
            for tag, grid, data in (("l1", gl1, L1), ("l2", gl2, L2)):
                fl, csl = data[fam]
                solve(fl, *csl, out=buf(f"{fam}.{tag}", fl), info=ints(f"{fam}.{tag}info", grid.nsys))
        for space in ("dirichlet", "biharmonic"):
            api.forward_transform(pts, space, out=buf(f"fwd.{space}", pts))
            api.backward_transform(outs[f"fwd.{space}"], space, out=buf(f"bwd.{space}", pts))

    step()
    torch.cuda.synchronize()
    eager = {k: v.clone() for k, v in outs.items()}
    assert all(int(eager[f"{fam}.info"].abs().sum()) == 0 for fam in H)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for r in range(3):
        for v in outs.values():
            v.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k, v in outs.items():
            assert torch.equal(v, eager[k]), (r, k)
        junk = api.biharmonic_solve(*[H["biharmonic"][0]], *H["biharmonic"][1])  # eager work between replays
        torch.cuda.synchronize()
        del junk
