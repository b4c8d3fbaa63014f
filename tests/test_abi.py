"""The C ABI library loads on a machine without a GPU and exports every
function declared in include/bf.h; the Python binding declares the same names.
No compute call is made here."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bf.h")
LIB = os.path.join(ROOT, "paper_2602_19697_amd", "libbf.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(bf_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2602_19697_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_five_entry_points():
    names = declared_functions()
    for n in ("bf_build_band", "bf_assemble", "bf_pcg_solve", "bf_diag_estimate", "bf_nbv_score"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, f"declared in bf.h but not exported: {missing}"
    for n in declared_functions():
        assert hasattr(lib, n)


def test_binding_covers_header():
    from paper_2602_19697_amd import _lib
    missing = [n for n in declared_functions() if n not in _lib.SIGNATURES]
    assert not missing, f"no Python declaration for {missing}"


def test_version_and_null_handling(lib):
    lib.bf_version.restype = ctypes.c_char_p
    assert lib.bf_version().startswith(b"bayesfusion")
    # NULL contexts are rejected without touching a device
    lib.bf_destroy.argtypes = [ctypes.c_void_p]
    assert lib.bf_destroy(None) == 0
    lib.bf_last_error.restype = ctypes.c_char_p
    lib.bf_last_error.argtypes = [ctypes.c_void_p]
    assert lib.bf_last_error(None) == b"null context"
    for fn in ("bf_pcg_solve", "bf_diag_estimate", "bf_build_band", "bf_assemble", "bf_nbv_score"):
        f = getattr(lib, fn)
        f.restype = ctypes.c_int
        assert f(*([None] * 11)) == 1  # BF_ERR_INVALID_ARG


def test_struct_layouts_match_header():
    """ctypes structures mirror the C structs: sizes follow the header's field lists."""
    from paper_2602_19697_amd import _lib as L
    assert ctypes.sizeof(L.bf_grid) == 8 + 8 + 24 + 8 + 8
    assert ctypes.sizeof(L.bf_camera) == 8 + 32
    assert ctypes.sizeof(L.bf_solve_opts) == 8 + 16
    assert ctypes.sizeof(L.bf_solve_report) == 16 + 8 + 8 + 8
    assert ctypes.sizeof(L.bf_probe_opts) == 8 + 8 + 8 + 8

