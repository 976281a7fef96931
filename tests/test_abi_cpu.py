"""Host-only checks of the C ABI: the library builds, loads, exports every function that
include/nnls.h declares, and its host-side entry points behave without a GPU."""
import ctypes as C
import os
import re

import pytest

import paper_cs_0408029_amd as N
from paper_cs_0408029_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nnls.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(nnls_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(N.LIB_PATH):
        from paper_cs_0408029_amd.build import build
        build()
    return N.load()


def test_header_declares_expected_calls():
    names = declared_functions()
    for must in ["nnls_solve_csc", "nnls_solve_dense", "nnls_create", "nnls_destroy",
                 "nnls_cholesky", "nnls_gram_csc", "nnls_dual_csc", "nnls_pivot_step"]:
        assert must in names


def test_every_declared_symbol_is_exported_and_bound(lib):
    names = declared_functions()
    assert names, "no declarations parsed"
    for name in names:
        assert hasattr(lib, name), f"{name} not exported"
        assert name in _lib.PROTOTYPES, f"{name} has no Python binding"
    assert set(_lib.PROTOTYPES) == set(names)


def test_default_options_are_the_papers(lib):
    o = N.default_options()
    assert o.tau == 1e-12 and o.p_max == 3          # Sec. 2 algorithm box
    assert o.max_iter == 0 and o.precision == N.NNLS_FP64


def test_status_strings(lib):
    assert N.status_string(N.NNLS_OK) == "NNLS_OK"
    assert N.status_string(N.NNLS_ERR_NOT_PD) == "NNLS_ERR_NOT_PD"
    assert N.status_string(-99) == "NNLS_ERR_UNKNOWN"


def test_struct_sizes_match_header(lib, tmp_path):
    """The ctypes mirrors have the sizes a C compiler gives the header's structs."""
    import shutil
    import subprocess
    names = ["nnls_options", "nnls_info", "nnls_trace_row", "nnls_server_config", "nnls_serving_stats"]
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "sizes.c"
    inc = os.path.join(ROOT, "include")
    src.write_text('#include <stdio.h>\n#include "nnls.h"\nint main(void) {\n' +
                   "".join(f'  printf("%zu\\n", sizeof({t}));\n' for t in names) + "  return 0;\n}\n")
    exe = tmp_path / "sizes"
    subprocess.run([cc, "-I", inc, str(src), "-o", str(exe)], check=True)
    sizes = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True,
                                            text=True).stdout.split()]
    assert sizes == [C.sizeof(getattr(N, t)) for t in names]


def test_null_arguments_rejected_without_device(lib):
    assert lib.nnls_create(None, 0, None) == N.NNLS_ERR_INVALID_ARG
    assert lib.nnls_destroy(None) == N.NNLS_ERR_INVALID_ARG
    info = N.nnls_info()
    st = lib.nnls_solve_csc(None, 10, 5, 0, None, None, None, None, None, None, None, C.byref(info))
    assert st == N.NNLS_ERR_INVALID_ARG and info.status == N.NNLS_ERR_INVALID_ARG


def test_create_reports_missing_device(lib):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert lib.nnls_create(C.byref(h), 0, None) == N.NNLS_ERR_DEVICE


def test_server_structs_and_null_arguments(lib):
    assert C.sizeof(N.nnls_server_config) == 32
    assert C.sizeof(N.nnls_serving_stats) == 4 * 8 + 2 * 4 + 8 * 8
    assert lib.nnls_server_create(None, 0, None, None) == N.NNLS_ERR_INVALID_ARG
    assert lib.nnls_server_destroy(None) == N.NNLS_ERR_INVALID_ARG
    assert lib.nnls_server_stats(None, None) == N.NNLS_ERR_INVALID_ARG
    assert lib.nnls_server_reset_stats(None) == N.NNLS_ERR_INVALID_ARG
    t = C.c_uint64()
    assert lib.nnls_server_submit_csc(None, 4, 2, 0, None, None, None, None, C.byref(t)) == N.NNLS_ERR_INVALID_ARG
    done = C.c_int32()
    assert lib.nnls_server_poll(None, 1, C.byref(done), None, None, None) == N.NNLS_ERR_INVALID_ARG
    assert lib.nnls_server_wait(None, 1, 0.0, None, None, None) == N.NNLS_ERR_INVALID_ARG
    assert N.status_string(N.NNLS_ERR_TIMEOUT) == "NNLS_ERR_TIMEOUT"


def test_server_rejects_bad_config_and_missing_device(lib):
    torch = pytest.importorskip("torch")
    s = C.c_void_p()
    bad = N.nnls_server_config(workers=-1)
    assert lib.nnls_server_create(C.byref(s), 0, C.byref(bad), None) == N.NNLS_ERR_INVALID_ARG
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert lib.nnls_server_create(C.byref(s), 0, None, None) == N.NNLS_ERR_DEVICE
