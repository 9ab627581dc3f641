"""CPU checks of the C ABI: the library loads, exports every entry point that
include/tprec.h declares with the binding's signatures, and rejects bad
arguments on the host before touching a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tprec.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:tp_status|const char\*|int32_t)\s+(tp_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_0910_0992_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libtprec.so missing: build with __graft_entry__.build()")
    return _lib.load()


def test_header_declares_the_expected_entry_points():
    names = _declared()
    for must in ["tp_ctx_create", "tp_gauge_create", "tp_clover_create", "tp_op_create", "tp_apply_M",
                 "tp_apply_Tinv", "tp_apply_prec", "tp_prepare_source", "tp_reconstruct", "tp_solve",
                 "tp_solve_multi", "tp_force"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_0910_0992_amd import _lib
    bound = {n for n, _, _ in _lib.SIGNATURES}
    assert set(_declared()) == bound


def test_status_strings(lib):
    assert lib.tp_status_string(0) == b"ok"
    assert lib.tp_status_string(-2) == b"unsupported lattice dimensions"


@pytest.mark.parametrize("dims", [(3, 4, 4, 8), (4, 5, 4, 8), (4, 4, 0, 8), (4, 4, 4, 1)])
def test_bad_dimensions_rejected_on_host(lib, dims):
    out = C.c_void_p()
    st = lib.tp_ctx_create((C.c_int32 * 4)(*dims), -1, 0, C.byref(out))
    assert st == -2 and not out.value
    assert lib.tp_last_error()


def test_bad_boundary_phase_rejected(lib):
    out = C.c_void_p()
    st = lib.tp_ctx_create((C.c_int32 * 4)(4, 4, 4, 8), 0, 0, C.byref(out))
    assert st == -1


def test_null_handles_rejected(lib):
    assert lib.tp_apply_M(None, 0, None, None, 0) == -1
    assert lib.tp_solve(None, None, None, None, None) == -1
    assert lib.tp_solve_multi(None, None, 2, None, None, None) == -1
    assert lib.tp_force(None, None, None, None, 1) == -1
    assert lib.tp_prof_select(None, 0xFFFFFFFF) == -1
    # destroy of a null handle is a no-op
    assert lib.tp_op_destroy(None) == 0


def test_kernel_profile_names(lib):
    n = lib.tp_prof_count()
    names = [lib.tp_prof_name(k).decode() for k in range(n)]
    assert "ilu_mid" in names and "scan_cr" in names and "hop_ds" in names and len(set(names)) == n
