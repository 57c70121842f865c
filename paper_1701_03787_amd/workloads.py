"""Seeded synthetic workloads for the wall-normal Shen-Galerkin solves.

This module only draws inputs: wavenumber grids, the per-wavenumber
coefficients of the Crank-Nicolson Helmholtz / biharmonic operators, and
complex right-hand sides.  It holds none of the solver arithmetic and imports
neither the GPU library nor the oracle, so both sides can share it.

Coefficient laws (Sec. 3, eqs. for the Helmholtz and biharmonic matrices):
dividing the paper's Helmholtz matrix by nu*dt/2 gives ``S + alpha*B`` with
``alpha = K2 + 2/(nu*dt)``; dividing its biharmonic matrix by -nu*dt/2 gives
``Q + a*A + b*B`` with ``a = -(2*K2 + 2/(nu*dt))`` and
``b = K2*(K2 + 2/(nu*dt))``, where ``K2 = kx^2 + kz^2`` is the squared
periodic wavenumber (2*pi-periodic box, integer wavenumbers).

Right-hand sides: real and imaginary parts i.i.d. N(0,1), scaled by
``(k+1)^-p`` along the wall-normal mode index k (p=2 for the small
Helmholtz-only case, p=3 otherwise); entries k >= n (the unknown count of the
family) are zero.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED = 1701
FAMILIES = ("helmholtz", "biharmonic")
_FAMILY_ID = {"helmholtz": 0, "biharmonic": 1}


def n_unknowns(family: str, N: int) -> int:
    """Number of Shen coefficients of a length-N array (Dirichlet: N-2, biharmonic: N-4)."""
    return N - 2 if family == "helmholtz" else N - 4


@dataclass(frozen=True)
class Grid:
    """One wall-normal batch: N modes and a flattened (kx, kz) wavenumber list."""

    N: int
    kx: np.ndarray
    kz: np.ndarray
    nu: float
    dt: float
    rhs_power: float
    config: int
    index: int = 0
    families: tuple = FAMILIES
    name: str = field(default="")

    @property
    def nsys(self) -> int:
        return int(self.kx.size)

    @property
    def K2(self) -> np.ndarray:
        return (self.kx.astype(np.float64) ** 2 + self.kz.astype(np.float64) ** 2)

    @property
    def inv(self) -> float:
        return 2.0 / (self.nu * self.dt)

    def alpha(self) -> np.ndarray:
        return self.K2 + self.inv

    def a(self) -> np.ndarray:
        return -(2.0 * self.K2 + self.inv)

    def b(self) -> np.ndarray:
        K2 = self.K2
        return K2 * (K2 + self.inv)

    def coefficients(self, family: str):
        if family == "helmholtz":
            return (self.alpha(),)
        return (self.a(), self.b())

    def rhs(self, family: str, rows=None) -> np.ndarray:
        """complex128 [nsys, N] (or [len(rows), N]); tail k >= n is zero.

        The full grid is drawn from one generator so that a row subset is
        bit-identical to the same rows of the full draw.
        """
        n = n_unknowns(family, self.N)
        rng = np.random.default_rng([SEED, self.config, self.index, _FAMILY_ID[family]])
        x = rng.standard_normal((self.nsys, n))
        y = rng.standard_normal((self.nsys, n))
        scale = (np.arange(n, dtype=np.float64) + 1.0) ** (-self.rhs_power)
        f = np.zeros((self.nsys, self.N), dtype=np.complex128)
        f[:, :n] = (x + 1j * y) * scale
        if rows is not None:
            f = np.ascontiguousarray(f[rows])
        return f


def rfft_grid(nkx: int, nkz_full: int):
    """Wavenumbers of an rfft mesh: kx = fftfreq(nkx)*nkx, kz = 0..nkz_full/2 (row-major)."""
    kx = np.rint(np.fft.fftfreq(nkx) * nkx).astype(np.int64)
    kz = np.arange(nkz_full // 2 + 1, dtype=np.int64)
    KX, KZ = np.meshgrid(kx, kz, indexing="ij")
    return KX.ravel(), KZ.ravel()


def config_grids(config: int):
    """The seeded grids of one workload configuration (1..5)."""
    if config == 1:
        k = np.arange(16, dtype=np.int64)
        KX, KZ = np.meshgrid(k, k, indexing="ij")  # w = 16*kx + kz
        return [Grid(64, KX.ravel(), KZ.ravel(), 1e-3, 1e-3, 2.0, 1,
                     families=("helmholtz",), name="N64_16x16")]
    if config == 2:
        kx, kz = rfft_grid(128, 128)
        return [Grid(256, kx, kz, 5e-5, 5e-4, 3.0, 2, name="N256_128x65")]
    if config == 3:
        kx, kz = rfft_grid(512, 512)
        return [Grid(512, kx, kz, 5e-5, 5e-4, 3.0, 3, name="N512_512x257")]
    if config == 5:
        kx, kz = rfft_grid(256, 256)
        return [Grid(512, kx, kz, 5e-5, 5e-4, 3.0, 5, name="N512_256x129")]
    if config == 4:
        rng = np.random.default_rng([SEED, 4])
        Ns = rng.choice([64, 128, 256, 512, 1024], size=48)
        ns = rng.choice([32, 64, 128, 256], size=48)
        grids = []
        for g in range(48):
            kx, kz = rfft_grid(int(ns[g]), int(ns[g]))
            grids.append(Grid(int(Ns[g]), kx, kz, 5e-5, 5e-4, 3.0, 4, index=g,
                              name=f"g{g}_N{int(Ns[g])}_{int(ns[g])}x{int(ns[g]) // 2 + 1}"))
        return grids
    raise ValueError(f"unknown config {config}")


def small_grid(N: int, nsys: int, config: int = 90, nu: float = 5e-5, dt: float = 5e-4,
               kmax: int = 64, index: int = 0) -> Grid:
    """A reduced channel-shaped grid (random integer wavenumbers up to kmax) for tests."""
    rng = np.random.default_rng([SEED, config, index, 7])
    kx = rng.integers(-kmax, kmax, size=nsys)
    kz = rng.integers(0, kmax + 1, size=nsys)
    if nsys > 0:
        kx[0] = 0
        kz[0] = 0
    return Grid(N, kx.astype(np.int64), kz.astype(np.int64), nu, dt, 3.0, config, index=index,
                name=f"small_N{N}_{nsys}")


def random_vector(shape, seed_tail, complex_=True) -> np.ndarray:
    """Seeded standard-normal array (complex by default), for adjoint/gradient probes."""
    rng = np.random.default_rng([SEED, 99, *seed_tail])
    if complex_:
        return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return rng.standard_normal(shape)
