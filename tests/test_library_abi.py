"""The C-ABI library loads on the CPU host and exports every symbol that
include/rw.h declares (no compute calls: those need a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rw.h")).read()
    return sorted(set(re.findall(r"^\s*(?:rw_status|const char\*)\s+(rw_\w+)\s*\(", src, re.M)))


def test_header_declares_the_expected_entry_points():
    from paper_2605_15418_amd.rw import EXPORTED
    assert set(_declared()) == set(EXPORTED)


def test_library_exports_every_declared_symbol():
    from paper_2605_15418_amd import rw as R
    assert os.path.exists(R.LIB_PATH), "librw.so not built (run __graft_entry__.build())"
    lib = ctypes.CDLL(R.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings_without_gpu():
    from paper_2605_15418_amd import rw as R
    lib = R.load_library()
    for code, name in R.STATUS.items():
        assert lib.rw_status_string(code)


def test_plan_create_rejects_bad_input_without_gpu():
    """Argument validation happens before any device allocation."""
    from paper_2605_15418_amd import rw as R
    lib = R.load_library()
    h = ctypes.c_void_p()
    st = lib.rw_plan_create(None, 0, None, None, 0, None, ctypes.byref(h))
    assert R.STATUS[st] == "RW_ERR_INVALID_ARG"
    assert b"null" in lib.rw_last_error()
