"""The C-ABI library loads and exports every function that include/mih.h
declares (no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mih.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["mih_build", "mih_knn", "linscan_knn", "mih_free", "mih_status_str"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_1307_2982_amd as mih
    if not os.path.exists(mih.lib_path()):
        pytest.fail("libmih.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(mih.lib_path())
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) <= set(mih.EXPORTED)
    lib.mih_status_str.restype = ctypes.c_char_p
    lib.mih_status_str.argtypes = [ctypes.c_int]
    assert lib.mih_status_str(0) == b"ok"
    assert lib.mih_status_str(2) == b"out of device memory"


def test_argument_errors_need_no_device():
    # argument checks happen before any device work
    import paper_1307_2982_amd as mih
    lib = mih.load()
    h = ctypes.c_void_p()
    assert lib.mih_build(None, 10, 64, 2, None, None, ctypes.byref(h)) == 1       # codes NULL
    assert lib.mih_build(None, 0, 96, 2, None, None, ctypes.byref(h)) == 1        # bad bits
    assert lib.mih_build(None, 0, 64, 0, None, None, ctypes.byref(h)) == 1        # m = 0
    assert lib.mih_build(None, 0, 64, 1, None, None, ctypes.byref(h)) == 4        # s = 64 > 32
    assert lib.mih_build(None, 0, 64, 2, None, None, None) == 1                   # out NULL
    assert lib.linscan_knn(None, 0, 64, None, 1, 5, None, None, None, None) == 1  # queries NULL
    assert lib.mih_knn(None, None, 0, 1, None, None, None, None) == 1             # index NULL
    assert lib.mih_rnn(None, None, 0, 3, None, None, ctypes.byref(h)) == 1        # index NULL
    assert lib.linscan_rnn(None, 0, 96, None, 0, 3, None, None, ctypes.byref(h)) == 1   # bad bits
    assert lib.linscan_rnn(None, 0, 64, None, 2, 3, None, None, ctypes.byref(h)) == 1   # queries NULL
    assert lib.linscan_rnn(None, 0, 64, None, 0, 3, None, None, None) == 1        # out NULL
    assert lib.linscan_knn_noalloc(None, 0, 64, None, 1, 5, None, None, None, None) == 1   # queries NULL
    assert lib.linscan_knn_noalloc(None, 0, 96, None, 0, 5, None, None, None, None) == 1   # bad bits
    assert lib.mih_rnn_result_view(None, None) == 1
    lib.mih_rnn_result_free(None)                                                 # ignored


def test_header_is_plain_c():
    # the boundary compiles as C99 (no C++ or HIP types leak into it)
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-x", "c", HEADER],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
