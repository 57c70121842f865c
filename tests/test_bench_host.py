"""Host logic of bench.py, without a GPU.

* More than one GPU is refused with exit status 2 before anything touches a device.
* The algorithmic bytes of one solve (the numerator of the roofline's achieved rate) equal what the
  solve must move by its contract: the significant right-hand-side coefficients it reads (the Shen
  Dirichlet space has N - 2 functions, the biharmonic space N - 4; Sec. 2), the N complex values per
  system it writes, and the float64 coefficients it reads.  Counted here from the arrays the workload
  generator produces, not from the formula in bench.py.
* The measured HBM traffic is taken from the committed counter summary only while its kernel-source
  hash matches the sources; otherwise it is null.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import bench
from paper_1701_03787_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("family", ["helmholtz", "biharmonic"])
@pytest.mark.parametrize("N", [16, 37, 512])
def test_algorithmic_bytes_match_the_solve_contract(family, N):
    g = wl.small_grid(N, 9, index=5)
    f = g.rhs(family)
    read_cols = int(np.count_nonzero(np.any(f != 0, axis=0)))
    assert read_cols == N - (2 if family == "helmholtz" else 4)
    out_row = np.empty(N, dtype=np.complex128)
    per_system = read_cols * f.itemsize + out_row.nbytes + sum(c.itemsize for c in g.coefficients(family))
    assert bench.alg_bytes(family, N, g.nsys) == g.nsys * per_system


def test_algorithmic_bytes_of_the_bench_workload():
    # N = 512 on the 512 x 257 rfft grid: 131,584 systems per family
    grid = wl.config_grids(3)[0]
    assert (grid.N, grid.nsys) == (512, 131584)
    assert bench.alg_bytes("helmholtz", grid.N, grid.nsys) == 131584 * (510 * 16 + 512 * 16 + 8)
    assert bench.alg_bytes("biharmonic", grid.N, grid.nsys) == 131584 * (508 * 16 + 512 * 16 + 16)


def _summary_hash(workload):
    with open(os.path.join(ROOT, "profiles", f"traffic_{workload}.md")) as fh:
        for line in fh:
            if line.startswith("kernel_source_sha256"):
                return line.split(":", 1)[1].strip().strip("`")
    return None


def test_measured_traffic_follows_the_kernel_hash(monkeypatch):
    workload = "N512_512x257"
    recorded = _summary_hash(workload)
    assert recorded and len(recorded) == 64
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: recorded)
    for family in ("helmholtz", "biharmonic"):
        t = bench.measured_traffic(workload, family)
        assert isinstance(t, int) and t > 0
        # at least the algorithmic bytes cross HBM
        assert t >= bench.alg_bytes(family, 512, 131584)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.measured_traffic(workload, "biharmonic") is None
    assert bench.measured_traffic("no_such_workload", "biharmonic") is None
