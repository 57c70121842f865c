"""Host-only checks of the C-ABI library: it loads, exports every declared entry
point, and rejects bad arguments before touching a device (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_1701_03787_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "shenhip.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in {"if", "defined"}))


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    declared = _declared()
    assert len(declared) >= 13
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == {s[0] for s in L.SIGNATURES}


def test_version_and_strings():
    lib = L.lib()
    assert lib.shen_abi_version() == 4
    for code in (0, -1, -2, -3, -4, 7):
        assert isinstance(lib.shen_status_string(code), bytes)
    o = L.default_opts()
    assert o.precision == 0 and o.quad == 0 and o.transpose == 0 and o.refine_max == 8
    assert o.refine_tol == pytest.approx(1e-14)
    assert C.sizeof(L.ShenOpts) == 72
    assert C.sizeof(L.ShenProblem) == 72


ALIGNED = 1 << 20  # never dereferenced: validation fails first or there is no device


@pytest.mark.parametrize("args,code", [
    ((2, 4, ALIGNED, ALIGNED, ALIGNED), L.SHEN_EINVAL),           # N < 3
    ((16, -1, ALIGNED, ALIGNED, ALIGNED), L.SHEN_EINVAL),         # nsys < 0
    ((16, 4, None, ALIGNED, ALIGNED), L.SHEN_EINVAL),             # NULL alpha
    ((16, 4, ALIGNED, None, ALIGNED), L.SHEN_EINVAL),             # NULL f
    ((16, 4, ALIGNED, ALIGNED + 8, ALIGNED + 4096), L.SHEN_EINVAL),  # misaligned f
    ((16, 4, ALIGNED + 4, ALIGNED, ALIGNED + 4096), L.SHEN_EINVAL),  # misaligned alpha
    ((16, 4, ALIGNED, ALIGNED, ALIGNED + 16), L.SHEN_EINVAL),     # partial overlap f/u
    ((16, 0, None, None, None), L.SHEN_OK),                       # empty batch: nothing to do
])
def test_helmholtz_argument_errors(args, code):
    lib = L.lib()
    o = L.default_opts()
    assert lib.helmholtz_solve(*args, C.byref(o)) == code


def test_bad_enums_and_sizes():
    lib = L.lib()
    for field, val in (("precision", 5), ("quad", 2), ("transpose", 3), ("variant", 9), ("refine_max", 1000),
                       ("chunk", -1), ("chunk", 65)):
        o = L.default_opts()
        setattr(o, field, val)
        assert lib.helmholtz_solve(16, 4, ALIGNED, ALIGNED, ALIGNED, C.byref(o)) == L.SHEN_EINVAL, field
        assert lib.biharmonic_solve(16, 4, ALIGNED, ALIGNED, ALIGNED, ALIGNED, C.byref(o)) == L.SHEN_EINVAL, field
    o = L.default_opts()
    o.work, o.work_bytes = ALIGNED + 8, 1 << 20  # misaligned workspace
    assert lib.helmholtz_solve(16, 4, ALIGNED, ALIGNED, ALIGNED, C.byref(o)) == L.SHEN_EINVAL
    o.work, o.work_bytes = ALIGNED, -1           # negative size
    assert lib.biharmonic_solve(16, 4, ALIGNED, ALIGNED, ALIGNED, ALIGNED, C.byref(o)) == L.SHEN_EINVAL
    o = L.default_opts()
    assert lib.biharmonic_solve(4, 4, ALIGNED, ALIGNED, ALIGNED, ALIGNED, C.byref(o)) == L.SHEN_EINVAL
    o.info = ALIGNED + 2
    assert lib.helmholtz_solve(16, 4, ALIGNED, ALIGNED, ALIGNED, C.byref(o)) == L.SHEN_EINVAL
    o = L.default_opts()
    o.precision = L.SHEN_FP32_REFINE
    o.transpose = 1
    assert lib.helmholtz_solve(16, 4, ALIGNED, ALIGNED, ALIGNED, C.byref(o)) == L.SHEN_ENOTSUP
    # matvec output may not alias its input; adjoint lambda may not alias u
    o = L.default_opts()
    assert lib.helmholtz_matvec(16, 4, ALIGNED, ALIGNED, ALIGNED, C.byref(o)) == L.SHEN_EINVAL
    assert lib.biharmonic_matvec(16, 4, ALIGNED, ALIGNED, ALIGNED, ALIGNED, C.byref(o)) == L.SHEN_EINVAL
    assert lib.helmholtz_adjoint(16, 4, ALIGNED, ALIGNED, ALIGNED + 4096, ALIGNED, ALIGNED, C.byref(o)) == L.SHEN_EINVAL


def test_iters_nsys_and_chunk_validation():
    """Host-side refusals: a misaligned iters array, nsys beyond SHEN_MAX_NSYS, and chunk lengths
    that no wave configuration of (family, N) is built with (instead of a silent substitute)."""
    lib = L.lib()
    A = ALIGNED
    o = L.default_opts()
    o.iters = A + 2
    assert lib.helmholtz_solve(16, 4, A, A, A + 4096, C.byref(o)) == L.SHEN_EINVAL
    o = L.default_opts()
    big = 2147483647
    assert lib.helmholtz_solve(16, big, A, A, A + 4096, C.byref(o)) == L.SHEN_EINVAL
    assert lib.biharmonic_matvec(16, big, A, A, A, A + 4096, C.byref(o)) == L.SHEN_EINVAL
    assert lib.dirichlet_mass_solve(16, big, A, A, C.byref(o)) == L.SHEN_EINVAL
    for fam, N, chunk in ((L.SHEN_HELMHOLTZ, 512, 4), (L.SHEN_HELMHOLTZ, 1024, 8), (L.SHEN_HELMHOLTZ, 9, 4),
                          (L.SHEN_BIHARMONIC, 512, 4), (L.SHEN_BIHARMONIC, 65, 8), (L.SHEN_BIHARMONIC, 128, 12)):
        o = L.default_opts()
        o.chunk = chunk
        assert lib.shen_factor_bytes(fam, N, C.byref(o)) == L.SHEN_EINVAL, (fam, N, chunk)
        if fam == L.SHEN_HELMHOLTZ:
            assert lib.helmholtz_solve(N, 4, A, A, A + (1 << 16), C.byref(o)) == L.SHEN_EINVAL
            assert lib.helmholtz_factor(N, 4, A, A, C.byref(o)) == L.SHEN_EINVAL
        else:
            assert lib.biharmonic_solve(N, 4, A, A, A, A + (1 << 16), C.byref(o)) == L.SHEN_EINVAL
            assert lib.biharmonic_adjoint(N, 4, A, A, None, A, A + (1 << 16), None, None, C.byref(o)) == L.SHEN_EINVAL
    for fam, N, chunk in ((L.SHEN_HELMHOLTZ, 64, 4), (L.SHEN_HELMHOLTZ, 512, 8), (L.SHEN_BIHARMONIC, 512, 8),
                          (L.SHEN_BIHARMONIC, 1024, 16)):
        o = L.default_opts()
        o.chunk = chunk
        assert lib.shen_factor_bytes(fam, N, C.byref(o)) > 0, (fam, N, chunk)


def test_binding_checks_host_only():
    """The Python binding refuses an out tensor of the wrong shape or device, and a factor
    state made for another configuration, before any call into the library."""
    import torch
    from paper_1701_03787_amd import api
    f = torch.zeros((3, 16), dtype=torch.complex128)
    with pytest.raises(ValueError):
        api._out(torch.zeros((2, 16), dtype=torch.complex128), f)  # short
    with pytest.raises(ValueError):
        api._out(torch.zeros((3, 16), dtype=torch.complex128, device="meta"), f)  # another device
    fac = api.ShenFactor(torch.zeros((3, 32), dtype=torch.float64), "biharmonic", 16, "gc", 0)
    for args in (("helmholtz", 16, "gc", 0), ("biharmonic", 17, "gc", 0), ("biharmonic", 16, "gl", None),
                 ("biharmonic", 16, None, 8)):
        fam, N, quad, chunk = args
        with pytest.raises(ValueError):
            api._check_fac(fac, fam, N, (3,), f.device, quad, chunk)
    with pytest.raises(ValueError):
        api._check_fac(fac.data, "biharmonic", 16, (3,), f.device)  # a bare tensor


def test_valid_call_without_device_reports_device_error():
    """With valid arguments and no GPU the library says so instead of crashing."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    lib = L.lib()
    o = L.default_opts()
    rc = lib.helmholtz_solve(16, 4, ALIGNED, ALIGNED, ALIGNED + (1 << 16), C.byref(o))
    assert rc == L.SHEN_EDEVICE


def test_null_opts_uses_defaults():
    lib = L.lib()
    assert lib.helmholtz_solve(2, 4, ALIGNED, ALIGNED, ALIGNED, None) == L.SHEN_EINVAL


def test_factor_bytes_host_only():
    """Per-system size of the factor-once state: 2G restart states of 16 bytes (Helmholtz) or
    80 bytes (biharmonic), G lanes per parity chain of the wave configuration for N."""
    lib = L.lib()
    o = L.default_opts()
    assert lib.shen_factor_bytes(L.SHEN_HELMHOLTZ, 512, C.byref(o)) == 2 * 16 * 16
    assert lib.shen_factor_bytes(L.SHEN_BIHARMONIC, 512, C.byref(o)) == 2 * 16 * 80
    o.chunk = 8
    assert lib.shen_factor_bytes(L.SHEN_BIHARMONIC, 512, C.byref(o)) == 2 * 32 * 80
    o = L.default_opts()
    assert lib.shen_factor_bytes(7, 512, C.byref(o)) == L.SHEN_EINVAL
    assert lib.shen_factor_bytes(L.SHEN_BIHARMONIC, 4, C.byref(o)) == L.SHEN_EINVAL
    assert lib.shen_factor_bytes(L.SHEN_HELMHOLTZ, 1 << 16, C.byref(o)) == L.SHEN_ENOTSUP  # beyond the wave kernels


def test_factored_argument_errors():
    lib = L.lib()
    A = ALIGNED
    o = L.default_opts()
    assert lib.helmholtz_factor(16, 4, A, None, C.byref(o)) == L.SHEN_EINVAL            # NULL fac
    assert lib.helmholtz_factor(16, 4, A, A + 8, C.byref(o)) == L.SHEN_EINVAL           # misaligned fac
    assert lib.biharmonic_factor(16, 4, A, None, A, C.byref(o)) == L.SHEN_EINVAL        # NULL b
    assert lib.helmholtz_factor(16, 0, None, None, C.byref(o)) == L.SHEN_OK             # empty batch
    # fac overlapping u
    assert lib.helmholtz_solve_factored(16, 4, A, A + 4096, A, A + 4096, C.byref(o)) == L.SHEN_EINVAL
    # partial overlap of f and u
    assert lib.biharmonic_solve_factored(16, 4, A, A, A + (1 << 16), A, A + 16, C.byref(o)) == L.SHEN_EINVAL
    for field, val in (("precision", L.SHEN_FP32_REFINE), ("transpose", 1), ("variant", 1)):
        o = L.default_opts()
        setattr(o, field, val)
        assert lib.helmholtz_factor(16, 4, A, A, C.byref(o)) == L.SHEN_ENOTSUP, field
        assert lib.biharmonic_solve_factored(16, 4, A, A, A + (1 << 16), A, A, C.byref(o)) == L.SHEN_ENOTSUP, field


def test_adjoint_factored_argument_errors():
    lib = L.lib()
    A = ALIGNED
    o = L.default_opts()
    # NULL fac; fac overlapping lambda; gradient without u
    assert lib.helmholtz_adjoint_factored(16, 4, A, None, A, A, A + 4096, None, C.byref(o)) == L.SHEN_EINVAL
    assert lib.helmholtz_adjoint_factored(16, 4, A, A + 4096, None, A, A + 4096, None, C.byref(o)) == L.SHEN_EINVAL
    assert lib.biharmonic_adjoint_factored(16, 4, A, A, A + (1 << 16), None, A, A, A + 8, None, C.byref(o)) == L.SHEN_EINVAL
    o.variant = 1
    assert lib.biharmonic_adjoint_factored(16, 4, A, A, A + (1 << 16), None, A, A, None, None, C.byref(o)) == L.SHEN_ENOTSUP


@pytest.mark.parametrize("fam", ["dirichlet_mass_solve", "biharmonic_mass_solve"])
def test_mass_solve_argument_errors(fam):
    lib = L.lib()
    fn = getattr(lib, fam)
    o = L.default_opts()
    nmin = 3 if fam.startswith("dirichlet") else 5
    assert fn(nmin - 1, 4, ALIGNED, ALIGNED + 4096, C.byref(o)) == L.SHEN_EINVAL        # N too small
    assert fn(16, -1, ALIGNED, ALIGNED + 4096, C.byref(o)) == L.SHEN_EINVAL             # nsys < 0
    assert fn(16, 4, None, ALIGNED, C.byref(o)) == L.SHEN_EINVAL                        # NULL f
    assert fn(16, 4, ALIGNED + 8, ALIGNED + 4096, C.byref(o)) == L.SHEN_EINVAL          # misaligned f
    assert fn(16, 4, ALIGNED, ALIGNED + 16, C.byref(o)) == L.SHEN_EINVAL                # partial overlap
    assert fn(1025, 4, ALIGNED, ALIGNED + (1 << 20), C.byref(o)) == L.SHEN_ENOTSUP      # beyond N = 1024
    assert fn(16, 0, None, None, C.byref(o)) == L.SHEN_OK                               # empty batch
    o32 = L.default_opts()
    o32.precision = 1
    assert fn(16, 4, ALIGNED, ALIGNED + 4096, C.byref(o32)) == L.SHEN_ENOTSUP           # FP64 only
    oc = L.default_opts()
    oc.variant = 1
    assert fn(16, 4, ALIGNED, ALIGNED + 4096, C.byref(oc)) == L.SHEN_ENOTSUP            # no chain kernel
    # in place is valid: with no device the call reaches the device query
    assert fn(16, 4, ALIGNED, ALIGNED, C.byref(o)) == L.SHEN_EDEVICE


def test_derivative_solve_argument_errors():
    lib = L.lib()
    o = L.default_opts()
    fn = lib.dirichlet_derivative_solve
    assert fn(4, 4, ALIGNED, ALIGNED + 4096, C.byref(o)) == L.SHEN_EINVAL              # N < 5
    assert fn(16, 4, ALIGNED, ALIGNED + 16, C.byref(o)) == L.SHEN_EINVAL               # partial overlap
    assert fn(1025, 4, ALIGNED, ALIGNED + (1 << 20), C.byref(o)) == L.SHEN_ENOTSUP     # beyond N = 1024
    assert fn(16, 0, None, None, C.byref(o)) == L.SHEN_OK
    assert fn(16, 4, ALIGNED, ALIGNED, C.byref(o)) == L.SHEN_EDEVICE                  # in place reaches the device


def test_rhs_argument_errors():
    """Crank-Nicolson right-hand sides: nu, dt > 0, no transpose, no aliasing of uhat."""
    lib = L.lib()
    A, B, S = ALIGNED, ALIGNED + (1 << 16), ALIGNED + (2 << 16)
    for fn in (lib.helmholtz_rhs, lib.biharmonic_rhs):
        o = L.default_opts()
        assert fn(16, 4, A, 0.0, 5e-4, B, None, S, C.byref(o)) == L.SHEN_EINVAL       # nu = 0
        assert fn(16, 4, A, 5e-5, -1.0, B, None, S, C.byref(o)) == L.SHEN_EINVAL      # dt < 0
        assert fn(16, 4, A, float("nan"), 5e-4, B, None, S, C.byref(o)) == L.SHEN_EINVAL
        assert fn(16, 4, A, 1e-300, 1e-300, B, None, S, C.byref(o)) == L.SHEN_EINVAL  # 2/(nu dt) overflows
        assert fn(16, 4, A, 5e-5, 5e-4, B, None, B, C.byref(o)) == L.SHEN_EINVAL      # rhs == uhat
        assert fn(16, 4, A, 5e-5, 5e-4, B, S + 16, S, C.byref(o)) == L.SHEN_EINVAL    # sh overlaps rhs partially
        assert fn(16, 4, A + 4, 5e-5, 5e-4, B, None, S, C.byref(o)) == L.SHEN_EINVAL  # misaligned K2
        assert fn(2, 4, A, 5e-5, 5e-4, B, None, S, C.byref(o)) == L.SHEN_EINVAL
        assert fn(16, 0, None, 5e-5, 5e-4, None, None, None, C.byref(o)) == L.SHEN_OK
        o.transpose = 1
        assert fn(16, 4, A, 5e-5, 5e-4, B, None, S, C.byref(o)) == L.SHEN_EINVAL


def test_missing_library_fails_loudly(monkeypatch):
    from paper_1701_03787_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libshenhip.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _lib.lib()


def test_product_path_never_reaches_the_oracle():
    # the package (binding, kernels, launchers) imports and includes nothing of the oracle
    import ast
    pkg = os.path.join(ROOT, "paper_1701_03787_amd")
    for dirpath, _, files in os.walk(pkg):
        for name in files:
            path = os.path.join(dirpath, name)
            if name.endswith(".py"):
                tree = ast.parse(open(path).read(), path)
                for node in ast.walk(tree):
                    if isinstance(node, ast.Import):
                        mods = [a.name for a in node.names]
                    elif isinstance(node, ast.ImportFrom):
                        mods = [node.module or ""]
                    else:
                        continue
                    assert not any(m.split(".")[0] == "oracle" for m in mods), (path, mods)
            elif name.endswith((".hip", ".hpp", ".h", ".cpp")):
                src = open(path).read()
                assert "oracle/" not in src and "shen_oracle" not in src, path


def test_oracle_is_independent_of_the_package():
    # the oracle imports nothing of the GPU package, not even the shared input generators
    import ast
    odir = os.path.join(ROOT, "oracle")
    for name in os.listdir(odir):
        if not name.endswith(".py"):
            continue
        path = os.path.join(odir, name)
        for node in ast.walk(ast.parse(open(path).read(), path)):
            if isinstance(node, ast.Import):
                mods = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                mods = [node.module or ""] if node.level == 0 else []
            else:
                continue
            assert not any(m.split(".")[0] in ("paper_1701_03787_amd", "torch", "ctypes") for m in mods), (path, mods)
