"""The C-ABI library loads and exports every entry point that include/sssp.h declares;
host-side argument checks that need no device (no compute calls here)."""
import ctypes
import os
import re

import pytest

from paper_1911_06895_amd import sssp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sssp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sssp_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for fn in ("sssp_create", "sssp_solve", "sssp_destroy", "sssp_last_stats", "sssp_status_string"):
        assert fn in names
    assert set(names) == set(sssp.EXPORTS), "binding and header disagree"


def test_library_exports_every_declared_symbol():
    lib = sssp.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), f"libsssp.so does not export {name}"


def test_status_strings():
    lib = sssp.load_library()
    for code in range(8):
        assert lib.sssp_status_string(code)
    assert sssp.sssp_status_string(5) == "distance overflow"


def test_host_argument_checks_without_device():
    lib = sssp.load_library()
    h = ctypes.c_void_p()
    # null graph / null out pointer are rejected before any device call
    assert lib.sssp_create(None, 1.0, None, ctypes.byref(h)) == sssp.SSSP_ERR_INVALID_ARGUMENT
    assert h.value is None
    g = sssp.SsspGraph(n=0, m=0, row_ptr=None, col_idx=None, weights=None, wtype=0)
    assert lib.sssp_create(ctypes.byref(g), 1.0, None, ctypes.byref(h)) == sssp.SSSP_ERR_INVALID_ARGUMENT
    g = sssp.SsspGraph(n=4, m=2, row_ptr=8, col_idx=None, weights=None, wtype=0)
    assert lib.sssp_create(ctypes.byref(g), 1.0, None, ctypes.byref(h)) == sssp.SSSP_ERR_INVALID_ARGUMENT
    g = sssp.SsspGraph(n=4, m=0, row_ptr=8, col_idx=None, weights=None, wtype=7)
    assert lib.sssp_create(ctypes.byref(g), 1.0, None, ctypes.byref(h)) == sssp.SSSP_ERR_INVALID_ARGUMENT
    g = sssp.SsspGraph(n=4, m=0, row_ptr=8, col_idx=None, weights=None, wtype=0)
    for bad_delta in (0.0, -1.0, 1.5, float("nan"), float("inf"), 2.0**33):
        assert lib.sssp_create(ctypes.byref(g), bad_delta, None, ctypes.byref(h)) == sssp.SSSP_ERR_INVALID_ARGUMENT
    g = sssp.SsspGraph(n=1 << 31, m=0, row_ptr=8, col_idx=None, weights=None, wtype=0)
    assert lib.sssp_create(ctypes.byref(g), 1.0, None, ctypes.byref(h)) == sssp.SSSP_ERR_UNSUPPORTED
    src = (ctypes.c_int32 * 1)(0)
    assert lib.sssp_solve(None, src, 1, 8, None) == sssp.SSSP_ERR_INVALID_ARGUMENT
    assert lib.sssp_solve_async(None, src, 1, 8, None) == sssp.SSSP_ERR_INVALID_ARGUMENT
    assert lib.sssp_solve_status(None, None) == sssp.SSSP_ERR_INVALID_ARGUMENT
    assert lib.sssp_solve_multi(None, src, 1, 8, None) == sssp.SSSP_ERR_INVALID_ARGUMENT
    assert lib.sssp_solve_multi_async(None, src, 1, 8, None) == sssp.SSSP_ERR_INVALID_ARGUMENT
    res = sssp.SsspAutotuneResult()
    assert lib.sssp_autotune(None, src, 1, 0, None, 0, 8, None, ctypes.byref(h), ctypes.byref(res)) == \
        sssp.SSSP_ERR_INVALID_ARGUMENT
    g = sssp.SsspGraph(n=4, m=0, row_ptr=8, col_idx=None, weights=None, wtype=0)
    bad = (ctypes.c_int32 * 1)(4)  # source outside [0, n): rejected on the host
    assert lib.sssp_autotune(ctypes.byref(g), bad, 1, 0, None, 0, 8, None, ctypes.byref(h), None) == \
        sssp.SSSP_ERR_INVALID_ARGUMENT
    assert lib.sssp_autotune(ctypes.byref(g), src, 1, 2, None, 0, 8, None, ctypes.byref(h), None) == \
        sssp.SSSP_ERR_INVALID_ARGUMENT
    assert lib.sssp_set_tuning(None, ctypes.byref(sssp.SsspTuning())) == sssp.SSSP_ERR_INVALID_ARGUMENT
    st = sssp.SsspStats()
    assert lib.sssp_last_stats(None, ctypes.byref(st)) == sssp.SSSP_ERR_INVALID_ARGUMENT
    lib.sssp_destroy(None)


def test_tuning_struct_matches_header():
    """The ctypes mirror of sssp_tuning has the header's fields in the header's order."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\} sssp_tuning;", text).group(1)
    fields = re.findall(r"int32_t\s+(\w+);", body)
    assert fields == [name for name, _ in sssp.SsspTuning._fields_]


def test_product_path_has_no_oracle_dependency():
    """The library and its binding never reach into the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_1911_06895_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "oracle.c" not in text and "liboracle" not in text, f
