"""The C-ABI library loads and exports every entry point declared in include/*.h (no GPU needed)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SO = os.path.join(ROOT, "paper_2501_08261_amd", "liblisatd.so")


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+(lt_[a-z0-9_]+)\s*\(", src, re.M):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(SO):
        from paper_2501_08261_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(SO)


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("lt_phenomt_modes", "lt_lisa_tdi_response", "lt_tdi_loglike", "lt_ctx_create"):
        assert n in names


def test_every_declared_symbol_is_exported(so):
    missing = [n for n in sorted(_declared()) if not hasattr(so, n)]
    assert not missing, missing


def test_binding_covers_the_header(so):
    from paper_2501_08261_amd import lib
    assert set(_declared()) <= set(lib.EXPORTED)


def test_null_context_is_an_error(so):
    so.lt_ctx_destroy.argtypes = [ctypes.c_void_p]
    so.lt_ctx_destroy.restype = ctypes.c_int
    assert so.lt_ctx_destroy(None) == -1
    so.lt_last_error.restype = ctypes.c_char_p
    assert b"null" in so.lt_last_error()
