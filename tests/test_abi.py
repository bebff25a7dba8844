"""The C-ABI library loads and exports every symbol include/sfdp.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfdp.h")
LIB = os.path.join(ROOT, "paper_1312_5653_amd", "libsfdp.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sfdp_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1312_5653_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_header_declares_the_api():
    names = declared_functions()
    for required in ("sfdp_ctx_create", "sfdp_problem_create", "sfdp_set_beta",
                     "sfdp_solve_range_space", "sfdp_apply_schur_inv", "sfdp_feti_solve",
                     "sfdp_apply_operator", "sfdp_kkt_residual", "sfdp_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_export():
    from paper_1312_5653_amd import sfdp
    assert set(declared_functions()) == set(sfdp.EXPORTS)


def test_errors_without_gpu_are_reported_not_raised(lib):
    """Without a usable device, context creation fails with a status code."""
    lib.sfdp_ctx_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p,
                                    ctypes.POINTER(ctypes.c_void_p)]
    lib.sfdp_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    st = lib.sfdp_ctx_create(-1, 0, None, ctypes.byref(h))
    assert st != 0
    assert lib.sfdp_last_error()


def test_destroying_a_null_context_is_a_no_op(lib):
    lib.sfdp_ctx_destroy.argtypes = [ctypes.c_void_p]
    lib.sfdp_ctx_destroy.restype = ctypes.c_int
    assert lib.sfdp_ctx_destroy(None) == 0
