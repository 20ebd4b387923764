"""The C-ABI library loads on the CPU and exports every function include/*.h declares
(no compute call: there is no GPU here).  Also the host-side status paths that need no device."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SO = os.path.join(ROOT, "paper_2203_01877_amd", "libtqp.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(tqp_[A-Za-z0-9_]+)\s*\(", text, re.M):
            names.add(m.group(1))
    return sorted(names)


def _lib():
    if not os.path.exists(SO):
        pytest.skip("libtqp.so not built")
    return ctypes.CDLL(SO)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("tqp_filter", "tqp_sort", "tqp_join", "tqp_groupby_agg", "tqp_topk",
                     "tqp_fragment_flags", "tqp_fragment_cust", "tqp_ctx_create"):
        assert required in names


def test_every_declared_symbol_is_exported():
    lib = _lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_null_arguments_are_rejected_without_a_device():
    lib = _lib()
    lib.tqp_sort.restype = ctypes.c_int
    sz = ctypes.c_size_t(0)
    # null context -> TQP_ERR_INVALID, reported synchronously, no device touched
    st = lib.tqp_sort(None, None, None, ctypes.c_int64(10), None, 0, None, None, None, ctypes.byref(sz), None)
    assert st == 1
    lib.tqp_last_error.restype = ctypes.c_char_p
    assert b"tqp_sort" in lib.tqp_last_error()


def test_binding_struct_layouts_match_header():
    import paper_2203_01877_amd._lib as L
    # field order and sizes of the descriptor structs (x86-64 C layout)
    assert ctypes.sizeof(L.Column) == 16 and ctypes.sizeof(L.Pred) == 16
    assert ctypes.sizeof(L.FlagsFragment) == 6 * 8 + 8 + 8 + 2 * 8 + 8 + 4 * 4
    assert ctypes.sizeof(L.FlagsOut) == 6 * 8
    assert ctypes.sizeof(L.CustFragment) == 4 * 8 + 8 + 2 * 8 + 8 + 4 * 4 + 8
    assert ctypes.sizeof(L.CustOut) == 3 * 8 + 8 + 6 * 8
