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
    for required in ("tqp_filter", "tqp_sort", "tqp_join", "tqp_join_kind", "tqp_hash_join", "tqp_join_band",
                     "tqp_pack_keys", "tqp_groupby_agg", "tqp_hash_groupby", "tqp_gather", "tqp_eval",
                     "tqp_topk",
                     "tqp_fragment_flags", "tqp_fragment_cust", "tqp_ctx_create"):
        assert required in names


def test_every_declared_symbol_is_exported():
    lib = _lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_unknown_join_kind_is_rejected_without_a_device():
    lib = _lib()
    lib.tqp_join_kind.restype = ctypes.c_int
    sz = ctypes.c_size_t(0)
    st = lib.tqp_join_kind(None, 9, None, None, ctypes.c_int64(0), None, None, None, ctypes.c_int64(0), None, None,
                           None, ctypes.c_int64(0), None, None, ctypes.byref(sz), None)
    assert st == 1
    lib.tqp_last_error.restype = ctypes.c_char_p
    assert b"kind 9" in lib.tqp_last_error()


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
    assert ctypes.sizeof(L.CustFragment) == 4 * 8 + 8 + 2 * 8 + 8 + 4 * 4 + 8 + 2 * 4
    assert ctypes.sizeof(L.CustOut) == 3 * 8 + 8 + 6 * 8


def test_struct_layouts_match_the_c_header(tmp_path):
    """Sizes and field offsets of every struct in include/tqp.h, as the host compiler lays them out,
    equal those of the ctypes declarations of the binding."""
    import shutil
    import subprocess
    import paper_2203_01877_amd._lib as L
    if not shutil.which("g++"):
        pytest.skip("no g++")
    structs = {"tqp_column": L.Column, "tqp_pred": L.Pred, "tqp_flags_fragment": L.FlagsFragment,
               "tqp_flags_out": L.FlagsOut, "tqp_cust_fragment": L.CustFragment, "tqp_cust_out": L.CustOut,
               "tqp_prof_entry": L.ProfEntry, "tqp_server_config": L.ServerConfig, "tqp_request": L.Request,
               "tqp_result": L.Result, "tqp_xinstr": L.XInstr, "tqp_group_col": L.GroupCol, "tqp_agg": L.Agg,
               "tqp_fragment": L.Fragment, "tqp_fragment_out": L.FragmentOut, "tqp_chain_table": L.ChainTable}
    lines = ['#include "tqp.h"', "#include <cstddef>", "#include <cstdio>", "int main() {"]
    for cname, py in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines.append("return 0; }")
    src = tmp_path / "layout.cpp"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                           "-I", "/opt/rocm/include", str(src), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got["%s.%s" % (cname, fname)]) == getattr(py, fname).offset, (cname, fname)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without libtqp.so the binding raises instead of computing anything another way."""
    from paper_2203_01877_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "SO", str(tmp_path / "libtqp.so"))
    with pytest.raises(ImportError, match="no CPU fallback"):
        _lib.load()
