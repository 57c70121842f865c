"""batched_solve_static (the batched launch with the library's own counter array, for
callers that cannot allocate) against batched_solve with a caller work buffer, through
the C-ABI: two calls in a row, the second on a smaller batch, each equal to the
work-buffer call and to the oracle on sampled rows.

Same descriptors and kernels on both sides, so the results must agree bit for bit;
the oracle bar is the solves' 1e-12 per-system relative error.
"""
import ctypes as C

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


def _batch(dev, shapes, seed):
    """Problems of the given (family, N, nsys) with the channel coefficient law and RHS recipe."""
    from paper_1701_03787_amd.batched import BatchedProblem
    probs, host = [], []
    for i, (fam, N, nsys) in enumerate(shapes):
        g = wl.small_grid(N, nsys, kmax=362, index=seed * 100 + i, nu=5e-5, dt=5e-4)
        f = g.rhs(fam)
        cs = g.coefficients(fam)
        info = torch.full((nsys,), -7, dtype=torch.int32, device=dev)
        probs.append(BatchedProblem(fam, torch.from_numpy(f).to(dev), [torch.from_numpy(c).to(dev) for c in cs],
                                    info=info))
        host.append((fam, N, cs, f))
    return probs, host


def _run_both(dev, shapes, seed):
    from paper_1701_03787_amd import _lib as L
    from paper_1701_03787_amd.batched import BatchedSolver
    probs, host = _batch(dev, shapes, seed)
    solver = BatchedSolver(probs)
    print(f"CASE no_alloc seed={seed} problems={len(probs)} tiles={solver.tiles_total}", flush=True)
    # reference: the work-buffer entry point
    solver.run(static=False)
    torch.cuda.synchronize()
    ref = {id(p): (p.u.cpu().numpy().copy(), p.info.cpu().numpy().copy()) for p in solver.problems}
    for p in solver.problems:
        p.u.fill_(float("nan"))
        p.info.fill_(-7)
    # the entry point under test, called through the C-ABI directly
    o = solver._opts()
    rc = L.lib().batched_solve_static(solver.desc, len(solver.problems), C.byref(o))
    assert rc == L.SHEN_OK, L.lib().shen_status_string(rc)
    torch.cuda.synchronize()
    rng = np.random.default_rng([1701, seed])
    order = {id(p): i for i, p in enumerate(probs)}
    for p in solver.problems:
        u, inf = p.u.cpu().numpy(), p.info.cpu().numpy()
        ru, rinf = ref[id(p)]
        assert np.array_equal(inf, rinf) and np.all(inf == 0)
        assert np.array_equal(u.view(np.float64), ru.view(np.float64)), "static and work-buffer launches differ"
        fam, N, cs, f = host[order[id(p)]]
        rows = np.unique(np.concatenate([[0, f.shape[0] - 1], rng.choice(f.shape[0], min(6, f.shape[0]), replace=False)]))
        want = so.solve(fam, N, tuple(c[rows] for c in cs), f[rows])
        assert so.rel_err_per_system(u[rows], want).max() <= TOL
        assert np.all(u[:, wl.n_unknowns(fam, N):] == 0)


def test_static_batched_two_calls(dev):
    """First a larger mixed batch, then a smaller one: the static counters are cleared by
    each launch, so the second call does not see the first call's counts."""
    first = [("helmholtz", 512, 300), ("biharmonic", 256, 257), ("biharmonic", 1024, 65), ("helmholtz", 64, 900),
             ("biharmonic", 128, 129), ("helmholtz", 1024, 70)]
    second = [("biharmonic", 64, 40), ("helmholtz", 256, 33)]
    _run_both(dev, first, 1)
    _run_both(dev, second, 2)


def test_static_scratch_limit(dev):
    """The static buffer covers the work buffer of up to 512 descriptors; a larger batch is refused
    with SHEN_ESCRATCH before anything is read or launched."""
    from paper_1701_03787_amd import _lib as L
    cap = L.lib().shen_batched_static_bytes()
    assert cap == 4096
    for nd in (1, 48, 512):
        assert 0 < L.lib().shen_batched_work_bytes(nd) <= cap
    assert L.lib().shen_batched_work_bytes(513) > cap
    host = (L.ShenProblem * 600)()
    o = L.default_opts()
    assert L.lib().batched_solve_static(host, 600, C.byref(o)) == L.SHEN_ESCRATCH
