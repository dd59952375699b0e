"""The C-ABI library loads and exports every function the headers under include/ declare (no GPU
needed)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))
LIB = os.path.join(ROOT, "paper_2111_12478_amd", "librd.so")


def declared_functions():
    """Every function the headers declare as a prototype (header-only device code, defined in the
    header with a body, is not a library symbol)."""
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        text = text.replace('extern "C" {', "")
        # keep what lies outside braces (struct and function bodies); the extern "C" block's
        # closing brace is unmatched
        top, depth = [], 0
        for ch in text:
            if ch == "{":
                depth += 1
            elif ch == "}":
                depth = max(0, depth - 1)
            elif depth == 0:
                top.append(ch)
        names |= set(re.findall(r"\b(rd_[a-z_]+)\s*\([^;()]*\)\s*;", "".join(top), flags=re.S))
    return sorted(names)


def test_header_declares_the_interface():
    names = declared_functions()
    for n in ("rd_init", "rd_trace_upload", "rd_check", "rd_races", "rd_trace_free", "rd_workspace_bytes"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="librd.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="librd.so not built")
def test_strerror_without_gpu():
    lib = ctypes.CDLL(LIB)
    lib.rd_strerror.restype = ctypes.c_char_p
    lib.rd_strerror.argtypes = [ctypes.c_int32]
    assert lib.rd_strerror(0) == b"ok"
    assert lib.rd_strerror(-3) == b"invalid trace"
