"""Benchmark: batched wall-normal Helmholtz + biharmonic solves on one MI355X.

One step = the FP64 Helmholtz solve and the FP64 biharmonic solve over every
(kx, kz) of the channel-scale workload (N = 512 wall-normal modes, 512 x 257
rfft wavenumber grid, 131,584 systems per family), inputs resident in HBM.
The FP32 + FP64-refinement form is timed beside it on the same inputs.

Prints ONE JSON line (rank 0).  `value` = wall-normal systems x N solved per
second over the whole step (both families).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "wall-normal solves·N/s + HBM GB/s, FP32+refine vs FP64 at 1e-12 rel err, 1 GPU"
HBM_PEAK_GBS = 8000.0


KERNEL_SOURCES = ("wave_kernels.hip", "shen_rows.hpp", "shen_launch.hpp")  # the solve kernels and their launchers


def kernel_source_hash() -> str:
    """sha256 over the sources of the FP64 solve kernels (identifies the code the counters were taken on)."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1701_03787_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, family: str):
    """HBM bytes per solve call from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary of this workload,
    or None when there is none or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith(("kernel_source_sha256", "traffic_bytes_")):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    v = vals.get(f"traffic_bytes_{family}")
    return int(v) if v else None


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def alg_bytes(family: str, N: int, nsys: int) -> int:
    """Algorithmic HBM bytes of one solve: read f[k<n], write u[0:N], read coefficients."""
    if family == "helmholtz":
        return nsys * (16 * (N - 2) + 16 * N + 8)
    return nsys * (16 * (N - 4) + 16 * N + 16)


def _sampled_err(fam, N, cs_host, f_host, u_dev, rows, transpose=False):
    """max per-system relative error of the device result on the given rows (oracle on the CPU)."""
    import numpy as np
    import torch
    from oracle import shen_oracle as so
    u = u_dev[torch.from_numpy(rows).to(u_dev.device)].cpu().numpy()
    ref = so.solve(fam, N, tuple(c[rows] for c in cs_host), f_host[rows], transpose=transpose)
    return float(so.rel_err_per_system(u, ref).max())


def measure_batched(dev, args):
    """Batching form: the 48 grids of uneven N (both families) in one persistent launch,
    captured in a hipGraph; replays are timed with HIP events."""
    import numpy as np
    import torch
    from paper_1701_03787_amd import workloads as wl
    from paper_1701_03787_amd.batched import BatchedProblem, BatchedSolver
    grids = wl.config_grids(4)
    probs, checks, units, nbytes = [], [], 0, 0
    rng = np.random.default_rng([1701, 4, 4])
    for g in grids:
        for fam in ("helmholtz", "biharmonic"):
            f = g.rhs(fam)
            cs = g.coefficients(fam)
            p = BatchedProblem(fam, torch.from_numpy(f).to(dev), [torch.from_numpy(c).to(dev) for c in cs])
            probs.append(p)
            rows = np.unique(np.concatenate([[0, g.nsys - 1], rng.choice(g.nsys, 2, replace=False)]))
            checks.append((fam, g.N, tuple(c[rows] for c in cs), f[rows], rows))
            units += g.nsys * g.N
            nbytes += alg_bytes(fam, g.N, g.nsys)
            del f
    solver = BatchedSolver(probs)  # autotuned (chunk, systems per work item) per (family, N)
    solver.capture()
    for _ in range(max(1, args.warmup)):
        solver.replay()
    torch.cuda.synchronize()
    reps = max(3, min(args.steps, 10))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        solver.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    err = 0.0
    for p, (fam, N, cs, f, rows) in zip(probs, checks):
        u = p.u[torch.from_numpy(rows).to(dev)].cpu().numpy()
        from oracle import shen_oracle as so
        err = max(err, float(so.rel_err_per_system(u, so.solve(fam, N, cs, f)).max()))
    out = {"workload": "48 grids, N in {64..1024}, both families", "problems": len(probs), "ms_per_launch": round(ms, 4),
           "value": round(units / (ms * 1e-3), 2), "unit": "system·N/s",
           "hbm_gbps": round(nbytes / (ms * 1e-3) / 1e9, 2), "frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "bytes_per_launch": int(nbytes), "max_rel_err_sampled": err, "graph_replays": reps,
           "autotuned": solver.configurations()}
    del solver, probs
    torch.cuda.empty_cache()
    return out


def measure_adjoint(dev, args):
    """Differentiation form: forward solve + hand-written adjoint (torch.autograd) on the
    N=512, 256x129 workload, per family; the gradient w.r.t. f is checked on sampled rows."""
    import numpy as np
    import torch
    from paper_1701_03787_amd import api
    from paper_1701_03787_amd import workloads as wl
    g = wl.config_grids(5)[0]
    out = {"workload": g.name}
    rng = np.random.default_rng([1701, 5, 5])
    rows = np.unique(np.concatenate([[0, g.nsys - 1], rng.choice(g.nsys, 14, replace=False)]))
    for fam in ("helmholtz", "biharmonic"):
        fh = g.rhs(fam)
        csh = g.coefficients(fam)
        f = torch.from_numpy(fh).to(dev).requires_grad_(True)
        cs = [torch.from_numpy(c).to(dev).requires_grad_(True) for c in csh]
        gbar = torch.from_numpy(wl.random_vector((g.nsys, g.N), (5, 2))).to(dev)

        def step():
            f.grad = None
            for c in cs:
                c.grad = None
            u = api.helmholtz(f, *cs) if fam == "helmholtz" else api.biharmonic(f, *cs)
            u.backward(gbar)
            return u

        for _ in range(max(1, args.warmup)):
            step()
        torch.cuda.synchronize()
        reps = max(3, min(args.steps, 10))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gb = gbar.cpu().numpy()
        n = wl.n_unknowns(fam, g.N)
        gb[:, n:] = 0
        err = _sampled_err(fam, g.N, csh, gb, f.grad, rows, transpose=True)
        # algorithmic bytes of forward + backward per system: the solve reads f[k<n] and the
        # coefficients and writes u; the adjoint reads gbar[k<n], u[k<n] and the coefficients and
        # writes lambda and one gradient per coefficient
        nc = len(csh)
        per = (16 * n + 16 * g.N + 8 * nc) + (16 * n + 16 * n + 16 * g.N + 8 * nc + 8 * nc)
        gbs = g.nsys * per / (ms * 1e-3) / 1e9
        out[fam] = {"ms_forward_backward": round(ms, 4), "value": round(g.nsys * g.N / (ms * 1e-3), 2),
                    "unit": "system·N/s", "bytes_per_step": int(g.nsys * per), "hbm_gbps": round(gbs, 2),
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "max_rel_err_grad_f_sampled": err}
        del f, cs, gbar
    torch.cuda.empty_cache()
    return out


def measure_factored(dev, args, grid, data, host, rows):
    """Factor-once / solve-many form on the bench workload: the restart states are computed
    once per family (timed on its own), then a step is the two factored solves; the state
    slots read by each solve are reported beside the algorithmic bytes."""
    import numpy as np
    import torch
    from paper_1701_03787_amd import api
    N, nsys = grid.N, grid.nsys
    out = {"workload": grid.name}
    facs, fac_ms = {}, {}
    for fam, (f, cs, u) in data.items():
        for _ in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            facs[fam] = (api.helmholtz_factor(cs[0], N, chunk=args.chunk) if fam == "helmholtz"
                         else api.biharmonic_factor(cs[0], cs[1], N, chunk=args.chunk))
            e1.record()
            torch.cuda.synchronize()
            fac_ms[fam] = e0.elapsed_time(e1)

    def launch(fam):
        f, cs, u = data[fam]
        if fam == "helmholtz":
            api.helmholtz_solve_factored(f, cs[0], facs[fam], out=u, chunk=args.chunk)
        else:
            api.biharmonic_solve_factored(f, cs[0], cs[1], facs[fam], out=u, chunk=args.chunk)

    for _ in range(max(1, args.warmup)):
        for fam in data:
            launch(fam)
    torch.cuda.synchronize()
    ev = {fam: [] for fam in data}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for fam in data:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            launch(fam)
            e1.record()
            ev[fam].append((e0, e1))
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    kms = {fam: float(np.mean([a.elapsed_time(b) for a, b in ev[fam]])) for fam in data}
    out.update({"ms_per_step": round(ms, 4), "value": round(len(data) * nsys * N / (ms * 1e-3), 2),
                "unit": "system·N/s", "kernel_ms": {k: round(v, 4) for k, v in kms.items()},
                "factor_ms": {k: round(v, 4) for k, v in fac_ms.items()}})
    for fam in data:
        state = facs[fam].data.numel() * 8
        out[fam] = {"hbm_gbps_algorithmic": round(alg_bytes(fam, N, nsys) / (kms[fam] * 1e-3) / 1e9, 2),
                    "state_bytes": int(state),
                    "hbm_gbps_with_states": round((alg_bytes(fam, N, nsys) + state) / (kms[fam] * 1e-3) / 1e9, 2),
                    "max_rel_err_sampled": _sampled_err(fam, N, host[fam][1], host[fam][0], data[fam][2], rows)}
    del facs
    torch.cuda.empty_cache()
    return out


def measure_matvec(dev, args, grid, data, host, rows):
    """O(N) products H u on the bench workload (the residual / right-hand-side assembly kernel):
    one read of u, one write of Hu per system; sampled rows against the oracle's dense product."""
    import numpy as np
    import torch
    from oracle import shen_oracle as so
    from paper_1701_03787_amd import api
    N, nsys = grid.N, grid.nsys
    out = {"workload": grid.name}
    for fam, (f, cs, u) in data.items():
        fn = api.helmholtz_matvec if fam == "helmholtz" else api.biharmonic_matvec
        hu = torch.empty_like(f)
        for _ in range(max(1, args.warmup)):
            fn(f, *cs, out=hu)
        torch.cuda.synchronize()
        reps = max(3, min(args.steps, 10))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn(f, *cs, out=hu)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        nbytes = nsys * (16 * N + 16 * N + 8 * len(cs))
        fh, csh = host[fam]
        ref = so.matvec(fam, N, tuple(c[rows] for c in csh), fh[rows], extended=True)
        got = hu[torch.from_numpy(rows).to(dev)].cpu().numpy()
        err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        out[fam] = {"ms": round(ms, 4), "hbm_gbps": round(nbytes / (ms * 1e-3) / 1e9, 2), "max_rel_err_sampled": err}
        del hu
    return out


def measure_rhs(dev, args, grid, data, host, rows):
    """Crank-Nicolson right-hand sides (Sec. 3, eqs. gfin / ufin) on the bench workload, with the
    S(h) term fused in: read uhat and S(h), write rhs per system (K2 per system); sampled rows
    against the oracle's extended-precision right-hand side from the paper's matrices."""
    import numpy as np
    import torch
    from oracle import shen_oracle as so
    from paper_1701_03787_amd import api
    from paper_1701_03787_amd import workloads as wl
    N, nsys = grid.N, grid.nsys
    K2h = grid.K2
    K2 = torch.from_numpy(K2h).to(dev)
    out = {"workload": grid.name, "nu": grid.nu, "dt": grid.dt}
    for fam, (f, cs, u) in data.items():
        fn = api.helmholtz_rhs if fam == "helmholtz" else api.biharmonic_rhs
        shh = wl.random_vector((len(rows), N), (66,))
        sh = torch.empty_like(f)
        sh.copy_(f)  # any resident S(h) rows of the workload's shape
        r = torch.empty_like(f)
        for _ in range(max(1, args.warmup)):
            fn(f, K2, grid.nu, grid.dt, sh, out=r)
        torch.cuda.synchronize()
        reps = max(3, min(args.steps, 10))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn(f, K2, grid.nu, grid.dt, sh, out=r)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        n = wl.n_unknowns(fam, N)
        nbytes = nsys * (16 * n + 16 * n + 16 * N + 8)
        # accuracy on sampled rows, with distinct S(h) rows for them
        idx = torch.from_numpy(rows).to(dev)
        shs = torch.from_numpy(shh).to(dev)
        got = fn(f[idx].contiguous(), K2[idx].contiguous(), grid.nu, grid.dt, shs).cpu().numpy()
        fh = host[fam][0]
        ref = so.rhs_assemble(fam, N, K2h[rows], grid.nu, grid.dt, fh[rows], shh, extended=True)
        err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        key = "helmholtz_gfin" if fam == "helmholtz" else "biharmonic_ufin"
        out[key] = {"ms": round(ms, 4), "hbm_gbps": round(nbytes / (ms * 1e-3) / 1e9, 2),
                    "frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "bytes_per_launch": int(nbytes),
                    "max_rel_err_sampled": err}
        del sh, r
    return out


def measure_transforms(dev, args, grid, data, host, rows):
    """Wall-normal Shen transforms (Sec. 2) on the bench workload's shape, Gauss points: the inverse
    (coefficients -> point values: one read, one write per system), the scalar products (point values ->
    S(u)) and the forward transform (scalar products, then the mass solve in place), per space; sampled
    rows against the oracle."""
    import numpy as np
    import torch
    from oracle import shen_oracle as so
    from paper_1701_03787_amd import api
    N, nsys = grid.N, grid.nsys
    out = {"workload": grid.name, "quad": "GC"}
    reps = max(3, min(args.steps, 10))
    for fam, (f, cs, u) in data.items():
        space = "dirichlet" if fam == "helmholtz" else "biharmonic"
        n = so.n_space(space, N)
        phys = torch.empty_like(f)
        coef = torch.empty_like(f)
        ops = {"backward": (lambda: api.backward_transform(f, space, out=phys), 16 * n + 16 * N),
               "scalar_product": (lambda: api.scalar_product(phys, space, out=coef), 16 * N + 16 * N),
               "forward": (lambda: api.forward_transform(phys, space, out=coef), 16 * N + 16 * N)}
        res = {}
        for name, (fn, per) in ops.items():
            for _ in range(max(1, args.warmup)):
                fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            gbs = nsys * per / (ms * 1e-3) / 1e9
            res[name] = {"ms": round(ms, 4), "hbm_gbps": round(gbs, 2), "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "bytes_per_launch": int(nsys * per)}
        idx = torch.from_numpy(rows).to(dev)
        api.backward_transform(f, space, out=phys)
        p = phys[idx].cpu().numpy()
        fh = host[fam][0][rows]
        ref = so.backward_transform(space, N, fh)
        res["backward"]["max_rel_err_sampled"] = float(np.max(np.abs(p - ref)) / np.max(np.abs(ref)))
        api.scalar_product(phys, space, out=coef)
        refs = so.scalar_product(space, N, p)
        got = coef[idx].cpu().numpy()
        res["scalar_product"]["max_rel_err_sampled"] = float(np.max(np.abs(got - refs)) / np.max(np.abs(refs)))
        api.forward_transform(phys, space, out=coef)
        got = coef[idx].cpu().numpy()
        res["forward"]["max_rel_err_sampled"] = float(so.rel_err_per_system(got, so.forward_transform(space, N, p)).max())
        out[space] = res
        del phys, coef
    return out


def measure_large_n(dev, args):
    """Large N (chains spread over the wavefronts of a work group): N=4096 on the 128x65 rfft
    grid (8,320 systems per family), the paper's largest roundoff-table column, and N=8192 on
    the 64x33 grid of the paper's 64x64 timing mesh (its largest timing-table column; one parity
    chain per work group there); ms, GB/s and sampled errors against the oracle (one row per
    family: the dense oracle is O(N^3)), and the factored solve (restart states computed once
    beforehand, as the paper times its solves).  At N=4096 the Helmholtz solve is also timed on the
    lane-per-chain kernels, which served it before."""
    import numpy as np
    import torch
    from paper_1701_03787_amd import api
    from paper_1701_03787_amd import workloads as wl
    reps = max(3, min(args.steps, 10))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def one_grid(N, nk, chain):
        kx, kz = wl.rfft_grid(nk, nk)
        g = wl.Grid(N, kx, kz, 5e-5, 5e-4, 3.0, 6, name=f"N{N}_{nk}x{nk // 2 + 1}")
        out = {"workload": g.name}
        rows = np.array([int(np.argmax(g.K2))])
        for fam in ("helmholtz", "biharmonic"):
            fh = g.rhs(fam)
            csh = g.coefficients(fam)
            f = torch.from_numpy(fh).to(dev)
            cs = [torch.from_numpy(c).to(dev) for c in csh]
            u = torch.empty_like(f)
            solve = api.helmholtz_solve if fam == "helmholtz" else api.biharmonic_solve
            ms = timed(lambda: solve(f, *cs, out=u))
            nbytes = alg_bytes(fam, g.N, g.nsys)
            gbs = nbytes / (ms * 1e-3) / 1e9
            rec = {"ms": round(ms, 4), "value": round(g.nsys * g.N / (ms * 1e-3), 2), "unit": "system·N/s",
                   "hbm_gbps": round(gbs, 2), "frac": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_launch": int(nbytes),
                   "max_rel_err_sampled": _sampled_err(fam, g.N, csh, fh, u, rows)}
            if chain and fam == "helmholtz":
                rec["chain_kernels_ms"] = round(timed(lambda: solve(f, *cs, out=u, variant="chain")), 4)
            # the solve with the factorisation done once beforehand (the paper's timed configuration)
            if fam == "helmholtz":
                fac = api.helmholtz_factor(cs[0], g.N)
                fms = timed(lambda: api.helmholtz_solve_factored(f, cs[0], fac, out=u))
            else:
                fac = api.biharmonic_factor(cs[0], cs[1], g.N)
                fms = timed(lambda: api.biharmonic_solve_factored(f, cs[0], cs[1], fac, out=u))
            rec["factored_ms"] = round(fms, 4)
            rec["factored_hbm_gbps"] = round(nbytes / (fms * 1e-3) / 1e9, 2)
            del fac
            out[fam] = rec
            del f, cs, u
        torch.cuda.empty_cache()
        return out

    out = one_grid(4096, 128, True)
    out["paper_max_n"] = one_grid(8192, 64, False)
    return out


def measure_mass(dev, args, grid, data, host, rows):
    """Mass-matrix solves u = B^{-1} f (forward Shen transforms, Sec. 2) on the bench
    workload, f standing in for the scalar products S(u): one read of f, one write of u
    per system; sampled rows against the oracle."""
    import numpy as np
    import torch
    from oracle import shen_oracle as so
    from paper_1701_03787_amd import api
    N, nsys = grid.N, grid.nsys
    out = {"workload": grid.name}
    for fam, (f, cs, u) in data.items():
        fn = api.dirichlet_mass_solve if fam == "helmholtz" else api.biharmonic_mass_solve
        v = torch.empty_like(f)
        for _ in range(max(1, args.warmup)):
            fn(f, out=v)
        torch.cuda.synchronize()
        reps = max(3, min(args.steps, 10))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn(f, out=v)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        n = N - 2 if fam == "helmholtz" else N - 4
        nbytes = nsys * (16 * n + 16 * N)
        ref = so.mass_solve(fam, N, host[fam][0][rows])
        got = v[torch.from_numpy(rows).to(dev)].cpu().numpy()
        err = float(so.rel_err_per_system(got, ref).max())
        key = "dirichlet" if fam == "helmholtz" else "biharmonic"
        out[key] = {"ms": round(ms, 4), "hbm_gbps": round(nbytes / (ms * 1e-3) / 1e9, 2), "max_rel_err_sampled": err}
        if fam == "biharmonic":
            # Bbar fhat = Cbar uhat, uhat = these biharmonic-basis rows
            for _ in range(max(1, args.warmup)):
                api.dirichlet_derivative_solve(f, out=v)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                api.dirichlet_derivative_solve(f, out=v)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            nbytes = nsys * (16 * (N - 4) + 16 * N)
            ref = so.derivative_solve(N, host[fam][0][rows])
            got = v[torch.from_numpy(rows).to(dev)].cpu().numpy()
            out["derivative"] = {"ms": round(ms, 4), "hbm_gbps": round(nbytes / (ms * 1e-3) / 1e9, 2),
                                 "max_rel_err_sampled": float(so.rel_err_per_system(got, ref).max())}
        del v
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the factored, batched (48 grids) and adjoint measurements")
    ap.add_argument("--variant", default="auto")
    ap.add_argument("--chunk", type=int, default=0, help="wave kernels: preferred chunk length (0 = automatic)")
    ap.add_argument("--probe-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU (asked for --gpus {args.gpus}); the systems are "
              "independent and would shard by wavenumber range, with no exchange", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1701_03787_amd import api
    from paper_1701_03787_amd import workloads as wl

    dev = torch.device("cuda:0")
    grid = wl.config_grids(args.config)[0]
    N, nsys = grid.N, grid.nsys
    fams = [f for f in ("helmholtz", "biharmonic") if f in grid.families]
    print(f"# workload {grid.name}: N={N} nsys={nsys} per family, families={fams}", file=sys.stderr, flush=True)

    host = {}
    data = {}
    for fam in fams:
        f = grid.rhs(fam)
        cs = grid.coefficients(fam)
        host[fam] = (f, cs)
        data[fam] = (torch.from_numpy(f).to(dev), [torch.from_numpy(c).to(dev) for c in cs],
                     torch.empty((nsys, N), dtype=torch.complex128, device=dev))
    torch.cuda.synchronize()

    def launch(fam, precision="fp64"):
        f, cs, u = data[fam]
        if fam == "helmholtz":
            api.helmholtz_solve(f, cs[0], out=u, precision=precision, variant=args.variant, chunk=args.chunk)
        else:
            api.biharmonic_solve(f, cs[0], cs[1], out=u, precision=precision, variant=args.variant, chunk=args.chunk)

    def timed(precision):
        for _ in range(args.warmup):
            for fam in fams:
                launch(fam, precision)
        torch.cuda.synchronize()
        ev = {fam: [] for fam in fams}
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for fam in fams:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                launch(fam, precision)
                e1.record()
                ev[fam].append((e0, e1))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms = {fam: float(np.mean([a.elapsed_time(b) for a, b in ev[fam]])) for fam in fams}
        return wall, kms

    wall, kms = timed("fp64")
    ms_per_step = 1e3 * wall / args.steps
    units = sum(nsys * N for _ in fams)
    value = units / (ms_per_step / 1e3)
    step_bytes = sum(alg_bytes(fam, N, nsys) for fam in fams)

    # accuracy of the timed outputs on a sample of systems (oracle, CPU)
    from oracle import shen_oracle as so
    rng = np.random.default_rng([1701, 77])
    rows = np.unique(np.concatenate([[0, nsys - 1, int(np.argmin(grid.K2)), int(np.argmax(grid.K2))],
                                     rng.choice(nsys, 28, replace=False)]))
    acc = {}
    for fam in fams:
        launch(fam, "fp64")
        torch.cuda.synchronize()
        u = data[fam][2][torch.from_numpy(rows).to(dev)].cpu().numpy()
        f, cs = host[fam]
        ref = so.solve(fam, N, tuple(c[rows] for c in cs), f[rows])
        acc[fam] = float(so.rel_err_per_system(u, ref).max())

    dom = max(fams, key=lambda fm: kms[fm])
    achieved = alg_bytes(dom, N, nsys) / (kms[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(grid.name, dom),
                "kernel": f"{dom}_solve fp64", "kernel_ms": round(kms[dom], 4),
                "bytes_per_launch": alg_bytes(dom, N, nsys)}

    mixed = None
    if not args.no_mixed:
        wall_m, kms_m = timed("fp32_refine")
        acc_m = {}
        for fam in fams:
            launch(fam, "fp32_refine")
            torch.cuda.synchronize()
            u = data[fam][2][torch.from_numpy(rows).to(dev)].cpu().numpy()
            f, cs = host[fam]
            ref = so.solve(fam, N, tuple(c[rows] for c in cs), f[rows])
            acc_m[fam] = float(so.rel_err_per_system(u, ref).max())
        ms_m = 1e3 * wall_m / args.steps
        # Per-system status and corrections of one full mixed launch (outside the timed
        # region), and the error of the uncorrected FP32 solve (refine_max = 0) on the
        # sampled rows: the pre-refinement error.
        status, pre = {}, {}
        for fam in fams:
            f, cs, u = data[fam]
            fn = api.helmholtz_solve if fam == "helmholtz" else api.biharmonic_solve
            _, inf, its = fn(f, *cs, out=u, precision="fp32_refine", variant=args.variant, chunk=args.chunk,
                             info=True, iters=True)
            torch.cuda.synchronize()
            iv, it = inf.cpu().numpy(), its.cpu().numpy()
            vals, cnts = np.unique(iv, return_counts=True)
            status[fam] = {"info_histogram": {str(int(v)): int(c) for v, c in zip(vals, cnts)},
                           "fp64_fallbacks": int(np.count_nonzero(iv == -2)),
                           "iters_mean": round(float(it.mean()), 4), "iters_max": int(it.max()),
                           "iters_histogram": {str(int(v)): int(c) for v, c in zip(*np.unique(it, return_counts=True))}}
            fn(f, *cs, out=u, precision="fp32_refine", variant=args.variant, chunk=args.chunk, refine_max=0)
            torch.cuda.synchronize()
            got = u[torch.from_numpy(rows).to(dev)].cpu().numpy()
            fh, csh = host[fam]
            ref = so.solve(fam, N, tuple(c[rows] for c in csh), fh[rows])
            pre[fam] = float(so.rel_err_per_system(got, ref).max())
            del inf, its
        mixed = {"value": units / (ms_m / 1e3), "ms_per_step": round(ms_m, 4),
                 "kernel_ms": {k: round(v, 4) for k, v in kms_m.items()},
                 "speedup_vs_fp64": round(ms_per_step / ms_m, 4), "max_rel_err": acc_m,
                 "pre_refine_err": pre, "status": status}

    forms = None
    if not args.no_forms:
        forms = {"factored": measure_factored(dev, args, grid, data, host, rows),
                 "matvec": measure_matvec(dev, args, grid, data, host, rows),
                 "rhs": measure_rhs(dev, args, grid, data, host, rows),
                 "transforms": measure_transforms(dev, args, grid, data, host, rows),
                 "mass": measure_mass(dev, args, grid, data, host, rows),
                 "batched": measure_batched(dev, args), "adjoint": measure_adjoint(dev, args),
                 "large_n": measure_large_n(dev, args)}

    cpu = None
    if not args.no_cpu:
        from threadpoolctl import threadpool_limits
        threads = so.host_threads()
        per_fam = min(nsys, max(256, 1024 * threads))
        sample = rng.choice(nsys, per_fam, replace=False)
        t_cpu = 0.0
        with threadpool_limits(limits=1):
            for fam in fams:
                f, cs = host[fam]
                dt, used, _ = so.time_solve(fam, N, tuple(c[sample] for c in cs), f[sample], threads=threads)
                t_cpu += dt
        cpu = {"value": round(len(fams) * per_fam * N / t_cpu, 2), "unit": "system·N/s", "cores": threads,
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"{per_fam} random systems per family of {grid.name} (same inputs), dense LU + refinement, "
                         f"{t_cpu:.1f} s on {threads} threads"}

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "system·N/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": grid.name, "N": N, "nsys_per_family": nsys, "families": fams,
                   "precision": "fp64", "quadrature": "GC"},
        "hbm_gbps_step": round(step_bytes / (ms_per_step * 1e-3) / 1e9, 2),
        "kernel_ms": {k: round(v, 4) for k, v in kms.items()},
        "max_rel_err": acc,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "mixed_fp32_refine": mixed,
        "forms": forms,
    }
    if args.probe_copy:
        x = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = int(x.numel() * 8)
    out["kernel_source_sha256"] = kernel_source_hash()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
