"""C ABI checks that need no GPU: the library loads, exports every function
include/gcdf.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

import paper_2601_18548_amd as g
from paper_2601_18548_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gcdf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gcdf_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    assert declared_functions() == sorted(g.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = g.library()
    for name in declared_functions():
        assert hasattr(lib, name), name


def _cfg(width=256, depth=4, precision=2):
    c = g._Config()
    c.width, c.depth, c.precision, c.device = width, depth, precision, 0
    return c


def test_create_rejects_bad_config_and_blob():
    lib = g.library()
    blob = wl.weights(256, 0).to_blob()
    h = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(blob, len(blob))
    assert lib.gcdf_create(ctypes.byref(_cfg(width=300)), buf, len(blob), ctypes.byref(h)) == g.EINVAL
    assert b"width" in lib.gcdf_last_error(None)
    assert lib.gcdf_create(ctypes.byref(_cfg(depth=3)), buf, len(blob), ctypes.byref(h)) == g.EINVAL
    assert lib.gcdf_create(ctypes.byref(_cfg(precision=7)), buf, len(blob), ctypes.byref(h)) == g.EINVAL
    assert lib.gcdf_create(ctypes.byref(_cfg()), buf, len(blob) - 4, ctypes.byref(h)) == g.EINVAL
    assert b"bytes" in lib.gcdf_last_error(None)
    bad = ctypes.create_string_buffer(b"XCDF" + blob[4:], len(blob))
    assert lib.gcdf_create(ctypes.byref(_cfg()), bad, len(blob), ctypes.byref(h)) == g.EINVAL
    wrong_width = wl.weights(512, 0).to_blob()
    buf2 = ctypes.create_string_buffer(wrong_width, len(wrong_width))
    assert lib.gcdf_create(ctypes.byref(_cfg(width=256)), buf2, len(wrong_width), ctypes.byref(h)) == g.EINVAL


def test_create_rejects_weights_outside_fp16_for_the_fp16_reverse_mode():
    """BF16X2_F16 holds the BF16-rounded hidden weights as FP16: a weight that
    rounds past FP16's largest finite value (|w| >= 65408: BF16 65536) or is not
    finite is rejected before any device work."""
    lib = g.library()
    w = wl.weights(256, 0)
    h = ctypes.c_void_p()
    for bad_value in (65408.0, -1e5, float("inf"), float("nan")):
        w2 = wl.Weights(w.width, w.depth, [m.copy() for m in w.mats], [b.copy() for b in w.biases], w.in_dim)
        w2.mats[2][17, 5] = bad_value
        blob = w2.to_blob()
        buf = ctypes.create_string_buffer(blob, len(blob))
        assert lib.gcdf_create(ctypes.byref(_cfg(precision=g.BF16X2_F16)), buf, len(blob), ctypes.byref(h)) == g.EINVAL
        assert b"W3" in lib.gcdf_last_error(None) and b"FP16" in lib.gcdf_last_error(None)


def test_calls_on_null_context_fail_cleanly():
    lib = g.library()
    assert lib.gcdf_eval(None, None, 1, None, 1, None, None) == g.EINVAL
    assert lib.gcdf_query(None, None, 1, None, 1, None, None, None, None, None, None) == g.EINVAL
    assert lib.gcdf_poll(None, 1) == g.EINVAL
    t = ctypes.c_uint64()
    assert lib.gcdf_submit(None, None, ctypes.byref(t)) == g.EINVAL
    lib.gcdf_destroy(None)
