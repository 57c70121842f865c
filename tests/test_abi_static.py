"""Host-only checks of batched_solve_static, the batched launch for callers that cannot
allocate (no GPU needed): it is exported, its static buffer covers every work size the
ABI hands out, and it rejects bad arguments before touching a device."""
import ctypes as C

from paper_1701_03787_amd import _lib as L

ALIGNED = 1 << 20  # never dereferenced: validation fails first


def test_static_entry_point_exported_and_sized():
    lib = L.lib()
    cap = lib.shen_batched_static_bytes()
    assert cap == 4096
    for nd in (1, 2, 48, 512):
        assert 0 < lib.shen_batched_work_bytes(nd) <= cap
    for nd in (513, 1000, 1 << 20):
        assert lib.shen_batched_work_bytes(nd) > cap
    assert b"static buffer" in lib.shen_status_string(L.SHEN_ESCRATCH)


def test_static_argument_errors():
    lib = L.lib()
    o = L.default_opts()
    host = (L.ShenProblem * 2)()
    assert lib.batched_solve_static(None, 1, C.byref(o)) == L.SHEN_EINVAL   # NULL descriptors
    assert lib.batched_solve_static(host, 0, C.byref(o)) == L.SHEN_EINVAL   # no descriptors
    assert lib.batched_solve_static(host, 1, C.byref(o)) == L.SHEN_EINVAL   # not planned (sys_per_tile 0)
    big = (L.ShenProblem * 700)()
    assert lib.batched_solve_static(big, 700, C.byref(o)) == L.SHEN_ESCRATCH  # beyond the static buffer
    o.quad = 7
    assert lib.batched_solve_static(host, 1, C.byref(o)) == L.SHEN_EINVAL   # bad enum
