"""Batched form: many independent grids (uneven N, both families) in one
persistent launch, optionally captured once in a hipGraph and replayed.

Per (family, N) an autotuner picks the two knobs of the launch: the chunk
length of the wave kernels, which fixes their configuration (C rows per lane
and parity chain, G lanes per chain, hence systems per wavefront), and the
number of systems per work item of the dynamic queue.  It times every offered
combination on the device and caches the winners in a JSON file (env
SHENHIP_AUTOTUNE_CACHE, default ~/.cache/shenhip/autotune.json).
"""
from __future__ import annotations

import ctypes as C
import itertools
import json
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from . import _lib as L
from .api import _QUAD

TILE_CANDIDATES = (8, 16, 32, 64, 128)
CHUNK_CANDIDATES = (4, 8, 16)
DEFAULT_TILE = 32


def wave_config(family: str, N: int, chunk: int = 0):
    """(C, G) of the wave kernels for (family, N) at this chunk length, or None if not offered."""
    c, g = C.c_int32(0), C.c_int32(0)
    fam = L.SHEN_HELMHOLTZ if family == "helmholtz" else L.SHEN_BIHARMONIC
    rc = L.lib().shen_wave_config(fam, int(N), int(chunk), C.byref(c), C.byref(g))
    return (int(c.value), int(g.value)) if rc == L.SHEN_OK else None


def chunk_candidates(family: str, N: int):
    """The chunk lengths offered for (family, N), one per distinct configuration."""
    out, seen = [], set()
    for ch in CHUNK_CANDIDATES:
        cfg = wave_config(family, N, ch)
        if cfg is not None and cfg[0] == ch and cfg not in seen:
            seen.add(cfg)
            out.append(ch)
    return out or [0]


@dataclass
class BatchedProblem:
    """One grid: family "helmholtz" (coeffs = (alpha,)) or "biharmonic" (coeffs = (a, b)).
    f and u are complex128 [nsys, N] device tensors (u must not alias f)."""

    family: str
    f: torch.Tensor
    coeffs: Sequence[torch.Tensor]
    u: Optional[torch.Tensor] = None
    info: Optional[torch.Tensor] = None
    tile: int = 0
    chunk: int = 0

    def __post_init__(self):
        if self.family not in ("helmholtz", "biharmonic"):
            raise ValueError(self.family)
        f = self.f
        if (not isinstance(f, torch.Tensor) or f.dtype != torch.complex128 or f.dim() != 2 or not f.is_contiguous()
                or not f.is_cuda):
            raise ValueError("f must be a contiguous complex128 [nsys, N] device tensor")
        need = 1 if self.family == "helmholtz" else 2
        if len(self.coeffs) != need:
            raise ValueError(f"{self.family} needs {need} coefficient arrays")
        for c in self.coeffs:
            if (not isinstance(c, torch.Tensor) or c.dtype != torch.float64 or tuple(c.shape) != (f.shape[0],)
                    or not c.is_contiguous() or c.device != f.device):
                raise ValueError(f"coefficients must be contiguous float64 [nsys] tensors on {f.device}")
        if self.u is None:
            self.u = torch.empty_like(f)
        u = self.u
        if (not isinstance(u, torch.Tensor) or u.dtype != torch.complex128 or tuple(u.shape) != tuple(f.shape)
                or not u.is_contiguous() or u.device != f.device):
            raise ValueError(f"u must be a contiguous complex128 tensor of shape {tuple(f.shape)} on {f.device}")
        if self.info is not None:
            i = self.info
            if (not isinstance(i, torch.Tensor) or i.dtype != torch.int32 or tuple(i.shape) != (f.shape[0],)
                    or not i.is_contiguous() or i.device != f.device):
                raise ValueError(f"info must be a contiguous int32 [nsys] tensor on {f.device}")

    @property
    def N(self) -> int:
        return int(self.f.shape[1])

    @property
    def nsys(self) -> int:
        return int(self.f.shape[0])


def _cache_path() -> str:
    return os.environ.get("SHENHIP_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "shenhip", "autotune.json"))


def _arch(device) -> str:
    p = torch.cuda.get_device_properties(device)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


class Autotuner:
    """Per (arch, family, N, quadrature) choice of the chunk length and the systems per work item."""

    def __init__(self, path: Optional[str] = None):
        self.path = path or _cache_path()
        self.table = {}
        if os.path.exists(self.path):
            try:
                with open(self.path) as fh:
                    self.table = json.load(fh)
            except (OSError, ValueError):
                self.table = {}

    def key(self, device, family, N, quad="gc") -> str:
        return f"{_arch(device)}|{family}|{N}|{quad}"

    def get(self, device, family, N, quad="gc"):
        """(chunk, tile) from the cache, or None."""
        v = self.table.get(self.key(device, family, N, quad))
        if not v or "chunk" not in v:
            return None
        return int(v["chunk"]), int(v["tile"])

    def tune(self, device, family: str, N: int, nsys: int = 16384, reps: int = 5, quad="gc"):
        """Time every offered (chunk, tile) on a synthetic grid of the given shape (HIP events on
        the launching stream, best of reps); store and return the fastest."""
        g = torch.Generator(device="cpu").manual_seed(1701 + N)
        f = torch.randn((nsys, N), dtype=torch.complex128, generator=g).to(device)
        K2 = torch.arange(nsys, dtype=torch.float64) % 4096
        inv = 8e7
        if family == "helmholtz":
            coeffs = [(K2 + inv).to(device)]
        else:
            coeffs = [(-(2 * K2 + inv)).to(device), (K2 * (K2 + inv)).to(device)]
        best, best_t = (0, DEFAULT_TILE), float("inf")
        timings = {}
        stream = torch.cuda.current_stream(device)
        for chunk, tile in itertools.product(chunk_candidates(family, N), TILE_CANDIDATES):
            solver = BatchedSolver([BatchedProblem(family, f, coeffs, tile=tile, chunk=chunk)], quad=quad, autotune=False)
            solver.run()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            for a, b in ev:
                a.record(stream)
                solver.run()
                b.record(stream)
            torch.cuda.synchronize(device)
            dt = min(a.elapsed_time(b) for a, b in ev) * 1e-3
            timings[f"{chunk},{tile}"] = dt
            if dt < best_t:
                best, best_t = (chunk, tile), dt
            del solver
        self.table[self.key(device, family, N, quad)] = {"chunk": best[0], "tile": best[1], "seconds": timings}
        self.save()
        return best

    def save(self):
        try:
            os.makedirs(os.path.dirname(self.path), exist_ok=True)
            tmp = self.path + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(self.table, fh, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
        except OSError:
            pass


class BatchedSolver:
    """Plans a batch of problems once; run() enqueues its launches (one walk and one persistent
    solve per class of grids with the same family, N and wave configuration)."""

    def __init__(self, problems: List[BatchedProblem], quad: str = "gc", autotune: bool = True,
                 tuner: Optional[Autotuner] = None):
        """autotune: pick (chunk, tile) per (family, N) with the tuner where a problem leaves them
        at 0 (cached per device); otherwise chunk 0 (automatic) and DEFAULT_TILE."""
        if not problems:
            raise ValueError("empty batch")
        self.device = problems[0].f.device
        if any(p.f.device != self.device for p in problems):
            raise ValueError(f"every problem of a batch must be on {self.device}")
        # largest work first: better balance of the dynamic work queue
        self.problems = sorted(problems, key=lambda p: -p.N)
        self.quad = quad
        tuner = tuner or (Autotuner() if autotune else None)
        n = len(self.problems)
        host = (L.ShenProblem * n)()
        for i, p in enumerate(self.problems):
            d = host[i]
            d.family = L.SHEN_HELMHOLTZ if p.family == "helmholtz" else L.SHEN_BIHARMONIC
            d.N = p.N
            d.nsys = p.nsys
            d.c0 = p.coeffs[0].data_ptr()
            d.c1 = p.coeffs[1].data_ptr() if p.family == "biharmonic" else None
            d.f = p.f.data_ptr()
            d.u = p.u.data_ptr()
            d.info = p.info.data_ptr() if p.info is not None else None
            tile, chunk = p.tile, p.chunk
            # past N = 1024 the large-N solves have no knob to tune
            if tuner is not None and (tile <= 0 or chunk <= 0) and wave_config(p.family, p.N) is not None:
                got = tuner.get(self.device, p.family, p.N, quad) or tuner.tune(self.device, p.family, p.N, quad=quad)
                chunk = chunk if chunk > 0 else got[0]
                tile = tile if tile > 0 else got[1]
            d.sys_per_tile = tile if tile > 0 else DEFAULT_TILE
            d.chunk = max(0, chunk)
        o = self._opts()
        total = L.lib().shen_batched_plan(host, n, C.byref(o))
        if total < 0:
            raise L.ShenError(int(total), "shen_batched_plan")
        self.tiles_total = int(total)
        self.maxN = max(p.N for p in self.problems)
        self.desc = host  # the planned HOST descriptors, read by the library at every call
        nbytes = int(L.lib().shen_batched_work_bytes(n))
        self.work = torch.zeros((nbytes + 7) // 8, dtype=torch.int64, device=self.device)
        self.tiles = [host[i].sys_per_tile for i in range(n)]
        self.chunks = [host[i].chunk for i in range(n)]
        self.graph = None

    def configurations(self):
        """The chosen knobs per (family, N): chunk, the (C, G) it gives, systems per work item."""
        out = {}
        for p, tile, chunk in zip(self.problems, self.tiles, self.chunks):
            cfg = wave_config(p.family, p.N, chunk)
            out[f"{p.family}|{p.N}"] = {"chunk": chunk, "C": cfg[0] if cfg else None, "G": cfg[1] if cfg else None,
                                        "sys_per_tile": tile}
        return out

    def _opts(self):
        o = L.default_opts()
        o.stream = torch.cuda.current_stream(self.device).cuda_stream
        o.quad = _QUAD[self.quad]
        return o

    def run(self, static: bool = False):
        """Enqueue the launch.  static=True uses batched_solve_static (the library's own
        counter array instead of this solver's work buffer: nothing is allocated)."""
        o = self._opts()
        if static:
            L.check(L.lib().batched_solve_static(self.desc, len(self.problems), C.byref(o)), "batched_solve_static")
            return
        L.check(L.lib().batched_solve(self.desc, len(self.problems), self.work.data_ptr(), C.byref(o)), "batched_solve")

    def capture(self):
        """Capture run() in a hipGraph once (warm up first); replay() re-launches it."""
        s = torch.cuda.Stream(self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):
            self.run()
        torch.cuda.current_stream(self.device).wait_stream(s)
        torch.cuda.synchronize(self.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()
        return self.graph

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()
