"""CPU checks of the C ABI library: it loads, exports every symbol the header
declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccproj.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cc_[a-z0-9_]+)\s*\(", src)))


def test_header_declarations_found():
    names = declared_functions()
    assert "cc_sweep" in names and "cc_residuals" in names and "cc_solve_cc_lp" in names


def test_library_exports_every_declared_symbol():
    from paper_1901_10084_amd import ccproj as C
    lib = ctypes.CDLL(C.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_num_metric_duals():
    from paper_1901_10084_amd import ccproj as C
    assert C.num_metric_duals(60) == 102660          # configuration with n = 60
    assert C.num_metric_duals(500) == 62125500
    assert C.num_metric_duals(4000) == 31976004000
    assert C.num_metric_duals(2) == 0


@pytest.mark.parametrize("n,b,prec", [(2, 8, 0), (100, 0, 0), (100, 33, 0), (100, 8, 7)])
def test_create_rejects_bad_arguments(n, b, prec):
    from paper_1901_10084_amd import ccproj as C
    h = ctypes.c_void_p()
    rc = C._L.cc_create(ctypes.byref(h), n, b, prec, None)
    assert rc == C.CC_EINVAL
    assert C.last_error()
    assert not h.value


def test_null_pointers_rejected():
    from paper_1901_10084_amd import ccproj as C
    assert C._L.cc_sweep(None, None, None, None, None, None, None, 1, 0) == C.CC_EINVAL
    assert C._L.cc_destroy(None) == C.CC_OK
    assert C._L.cc_widen(None, None, -1, None) == C.CC_EINVAL


def test_gate_entry_points_reject_bad_arguments():
    """The sampled gate's entry points check their arguments before any GPU
    call: a null context, a negative or oversized count."""
    import ctypes
    from paper_1901_10084_amd import ccproj as C
    assert C._L.cc_set_gate_sample(None, 16) == C.CC_EINVAL
    assert C._L.cc_last_gate_sample(None, None, None, None, None) == C.CC_EINVAL
    assert C._L.cc_warm_gate_terms(None, None, None, None, None, 1.0, None, None, 1, None,
                                   None) == C.CC_EINVAL
    assert C.last_error()
