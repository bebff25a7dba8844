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


def test_process_settings_reject_values_outside_their_range(lib):
    """The process-wide switches take their documented values only (host code, no GPU)."""
    for name, good, bad in (("sfdp_set_gmres_launch", (0, 1, 2), (-1, 3)), ("sfdp_set_graphs", (0, 1), (2,)),
                            ("sfdp_set_tuning", (1,), (-1, 6))):
        fn = getattr(lib, name)
        fn.argtypes = [ctypes.c_int]
        fn.restype = ctypes.c_int
        for v in bad:
            assert fn(v) != 0, (name, v)
        for v in good:
            assert fn(v) == 0, (name, v)
    assert lib.sfdp_set_gmres_launch(1) == 0 and lib.sfdp_set_graphs(0) == 0


def test_destroying_a_null_context_is_a_no_op(lib):
    lib.sfdp_ctx_destroy.argtypes = [ctypes.c_void_p]
    lib.sfdp_ctx_destroy.restype = ctypes.c_int
    assert lib.sfdp_ctx_destroy(None) == 0


def test_binding_structures_match_the_header(tmp_path):
    """Size and field offsets of every structure of include/sfdp.h, as the C
    compiler lays it out, equal those of the binding's ctypes structures (a field
    added on one side only would shift everything after it)."""
    import shutil
    import subprocess

    from paper_1312_5653_amd import sfdp
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pairs = {"sfdp_opts": sfdp.Opts, "sfdp_info": sfdp.Info, "sfdp_request": sfdp.Request,
             "sfdp_server_info": sfdp.ServerInfo, "sfdp_timing": sfdp.Timing, "sfdp_sizes": sfdp.Sizes}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "sfdp.h"', "int main(void) {"]
    for cname, py in pairs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            name, field, val = line.split()
            got[(name, field)] = int(val)
    for cname, py in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
