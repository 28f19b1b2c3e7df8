"""The C ABI library loads and exports every function include/jp.h declares.

No GPU is needed: only symbol presence and the argument checks that happen
before any device work.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", "jp.h"), os.path.join(ROOT, "include", "jp_testing.h")]
LIB = os.path.join(ROOT, "paper_2002_12459_amd", "libjoinproject.so")


def declared_functions():
    text = "\n".join(open(p).read() for p in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(jp_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libjoinproject.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("jp_create", "jp_destroy", "jp_set_stream", "jp_two_path", "jp_star", "jp_result_size",
              "jp_result_copy", "jp_result_columns", "jp_result_stats", "jp_result_free", "jp_last_error",
              "jp_bool_matmul", "jp_default_options"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_null_handle_and_result_are_rejected(lib):
    lib.jp_two_path.restype = ctypes.c_int
    lib.jp_result_size.restype = ctypes.c_int
    lib.jp_last_error.restype = ctypes.c_char_p
    out = ctypes.c_void_p()
    assert lib.jp_two_path(None, None, None, ctypes.c_int64(0), None, None, ctypes.c_int64(0), None,
                           ctypes.byref(out)) == 1
    assert lib.jp_result_size(None, None, None) == 1
    lib.jp_result_free(None)  # no-op
    lib.jp_destroy(None)      # no-op
    assert lib.jp_last_error(None) == b"null handle"


def test_default_options(lib):
    import paper_2002_12459_amd as jp
    o = jp.Options()
    lib.jp_default_options(ctypes.byref(o))
    assert o.strategy == jp.STRATEGY["auto"] and o.bmm == 0 and o.y_rule == 0 and o.dedup == 0


def test_struct_layouts_match_header():
    import paper_2002_12459_amd as jp
    # jp_options: 2 x int64 + 4 x int32 + 2 x uint64
    assert ctypes.sizeof(jp.Options) == 48
    # jp_stats: 7 int64, 4 int32, 8 int64, 10 double, 1 int64, 2 double, 2 int64
    assert ctypes.sizeof(jp.Stats) == 7 * 8 + 4 * 4 + 8 * 8 + 10 * 8 + 8 + 2 * 8 + 2 * 8


def test_lookback_wait_hook_rejects_a_null_handle(lib):
    lib.jp_test_set_lookback_wait.restype = ctypes.c_int
    lib.jp_test_set_lookback_wait.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    assert lib.jp_test_set_lookback_wait(None, 0) == 1
