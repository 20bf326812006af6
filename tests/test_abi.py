"""Host-side checks of the C-ABI library: it loads, exports every declared
symbol, and rejects invalid arguments before touching a device."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

import paper_1512_02831_amd as bkd

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "bkd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bkd_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = bkd.lib()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
    assert set(bkd.exported_names()) <= set(names)


def test_version_and_defaults_follow_the_paper_rule():
    assert "gfx950" in bkd.version()
    for h, B, M in ((9, 1 << 15, 10 << 15), (14, 1024, 10240), (10, 16384, 163840)):
        o = bkd.default_options(h)
        assert (o.buffer_size, o.fetch_size, o.chunk_mode) == (B, M, bkd.CHUNK_LEAF)


@pytest.mark.parametrize("n,d,h", [(0, 3, 0), (10, 0, 0), (10, 33, 0), (10, 3, -1), (10, 3, 4), (10, 3, 25)])
def test_build_rejects_invalid_shapes(n, d, h):
    L = bkd.lib()
    P = np.zeros((max(n, 1), max(d, 1)), dtype=np.float32)
    out = ctypes.c_void_p()
    rc = L.bkd_build(P.ctypes.data_as(ctypes.c_void_p), n, d, h, None, ctypes.byref(out))
    assert rc == bkd.EINVAL and out.value is None
    assert L.bkd_last_error()


def test_build_rejects_null_and_nonfinite():
    L = bkd.lib()
    out = ctypes.c_void_p()
    assert L.bkd_build(None, 10, 2, 1, None, ctypes.byref(out)) == bkd.EINVAL
    assert L.bkd_build(None, 10, 2, 1, None, None) == bkd.EINVAL
    P = np.zeros((16, 2), dtype=np.float32)
    P[3, 1] = np.nan
    assert L.bkd_build(P.ctypes.data_as(ctypes.c_void_p), 16, 2, 1, None, ctypes.byref(out)) == bkd.EINVAL
    assert b"finite" in L.bkd_last_error()


def test_query_rejects_null_tree():
    L = bkd.lib()
    Q = np.zeros((1, 2), dtype=np.float32)
    assert L.bkd_query(None, Q.ctypes.data_as(ctypes.c_void_p), 1, 1, None, None) == bkd.EINVAL
    assert L.bkd_free(None) == bkd.OK


@pytest.mark.parametrize("field,value", [("age_max", -1), ("straggle_max", -1), ("max_requests", -2),
                                         ("slots_per_session", -5), ("device", -1)])
def test_server_create_rejects_invalid_options(field, value):
    # checked before any device is touched
    L = bkd.lib()
    o = bkd.ServerOpts()
    setattr(o, field, value)
    out = ctypes.c_void_p()
    assert L.bkd_server_create(ctypes.byref(o), ctypes.byref(out)) == bkd.EINVAL
    assert b"invalid server options" in L.bkd_last_error()
    assert out.value is None
