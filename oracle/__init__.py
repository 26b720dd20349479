"""FP64 CPU oracle for the batched neural GCDF query (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path (the HIP library
and its Python binding) never does, and this package never imports it.

``gcdf_oracle.c`` holds the plain double-precision definition of every step
of the query (base-frame transform, distance MLP, reverse-mode input gradient,
chain rule to the full configuration, per-knot minimum, and the MSE weight
gradient used by the training form), for point obstacles (network input
[p', a], 9 wide) and for sphere obstacles (x, y, z, r) with the 10-wide input
[p', r, a] of the primitive-aware extension (Sec. VII); the blob's in_dim
selects which.  ``toy.py`` holds a brute-force GCDF for
a small planar robot, used to test the GCDF structure of Theorem 1.
"""
from __future__ import annotations

import ctypes
import os
import struct
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gcdf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile gcdf_oracle.c with gcc + OpenMP into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    lib.gcdf_ref_in_dim.argtypes = [P, ctypes.c_size_t]
    lib.gcdf_ref_in_dim.restype = ctypes.c_int
    lib.gcdf_ref_threads.argtypes = [ctypes.c_int]
    lib.gcdf_ref_threads.restype = ctypes.c_int
    lib.gcdf_ref_transform.argtypes = [P, P, I64, P]
    lib.gcdf_ref_transform.restype = None
    lib.gcdf_ref_chain.argtypes = [P, P, P, I64, P]
    lib.gcdf_ref_chain.restype = None
    lib.gcdf_ref_mlp.argtypes = [P, ctypes.c_size_t, P, I64, P, P, ctypes.c_int]
    lib.gcdf_ref_mlp.restype = ctypes.c_int
    lib.gcdf_ref_eval_grad.argtypes = [P, ctypes.c_size_t, P, I64, P, I64, P, P, ctypes.c_int]
    lib.gcdf_ref_eval_grad.restype = ctypes.c_int
    lib.gcdf_ref_eval_grad_f64.argtypes = [P, ctypes.c_size_t, P, I64, P, I64, P, P, ctypes.c_int]
    lib.gcdf_ref_eval_grad_f64.restype = ctypes.c_int
    lib.gcdf_ref_eval_pairs.argtypes = [P, ctypes.c_size_t, P, P, P, P, I64, P, P, ctypes.c_int]
    lib.gcdf_ref_eval_pairs.restype = ctypes.c_int
    lib.gcdf_ref_table1_grad.argtypes = [P, ctypes.c_size_t, P, P, P, P, P, P, I64, P, P]
    lib.gcdf_ref_table1_grad.restype = ctypes.c_double
    lib.gcdf_ref_knot_min.argtypes = [P, I64, I64, P, P]
    lib.gcdf_ref_knot_min.restype = None
    lib.gcdf_ref_mse_grad.argtypes = [P, ctypes.c_size_t, P, P, P, I64, P]
    lib.gcdf_ref_mse_grad.restype = ctypes.c_double
    _lib = lib
    return lib


def _f64(a, cols):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim != 2 or a.shape[1] != cols:
        raise ValueError("expected an (n, %d) array" % cols)
    return a


def _f32(a, cols):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.ndim != 2 or a.shape[1] != cols:
        raise ValueError("expected an (n, %d) array" % cols)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def threads(nthreads: int = 0) -> int:
    return _load().gcdf_ref_threads(nthreads)


def transform(knots, points) -> np.ndarray:
    """Base-frame point p' for each row pair (knot i, point i) -> (n, 3) float64."""
    k, p = _f64(knots, 9), _f64(points, 3)
    assert len(k) == len(p)
    out = np.empty((len(k), 3), np.float64)
    _load().gcdf_ref_transform(_ptr(k), _ptr(p), len(k), _ptr(out))
    return out


def chain(knots, points, e) -> np.ndarray:
    """Configuration gradient J (n, 9) from base-frame input gradients e (n, 9)."""
    k, p = _f64(knots, 9), _f64(points, 3)
    e = np.ascontiguousarray(e, dtype=np.float64)
    assert e.shape == (len(k), 9) and len(k) == len(p)
    out = np.empty((len(k), 9), np.float64)
    _load().gcdf_ref_chain(_ptr(k), _ptr(p), _ptr(e), len(k), _ptr(out))
    return out


def in_dim(blob: bytes) -> int:
    """Network input width of a weight blob: 9 (points) or 10 (spheres)."""
    b = ctypes.create_string_buffer(blob, len(blob))
    n = _load().gcdf_ref_in_dim(b, len(blob))
    if n < 0:
        raise ValueError("oracle rejected the weight blob")
    return n


def obstacle_dim(blob: bytes) -> int:
    """Floats per obstacle for a blob: 3 (x, y, z) or 4 (x, y, z, r)."""
    return in_dim(blob) - 6


def mlp(blob: bytes, v, with_grad: bool = True, nthreads: int = 0):
    """Network value d (n,) and input gradient e (n, in_dim) at network inputs v (n, in_dim)."""
    ni = in_dim(blob)
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert v.ndim == 2 and v.shape[1] == ni
    n = len(v)
    d = np.empty(n, np.float64)
    e = np.empty((n, ni), np.float64) if with_grad else None
    b = ctypes.create_string_buffer(blob, len(blob))
    rc = _load().gcdf_ref_mlp(b, len(blob), _ptr(v), n, _ptr(d), _ptr(e) if with_grad else None, nthreads)
    if rc:
        raise ValueError("oracle rejected the weight blob")
    return d, e


def eval_grad(blob: bytes, knots, points, with_grad: bool = True, nthreads: int = 0):
    """All pairs, knot-major: d (K, Np) and J (K, Np, 9) in float64.

    points: (Np, 3), or (Np, 4) spheres for a 10-input blob.  float32 inputs
    go through the float32 entry point (exact widening); float64 inputs
    through the double-precision one.
    """
    dbl = np.asarray(knots).dtype == np.float64 or np.asarray(points).dtype == np.float64
    conv = _f64 if dbl else _f32
    k, p = conv(knots, 9), conv(points, obstacle_dim(blob))
    K, Np = len(k), len(p)
    d = np.empty((K, Np), np.float64)
    J = np.empty((K, Np, 9), np.float64) if with_grad else None
    b = ctypes.create_string_buffer(blob, len(blob))
    fn = _load().gcdf_ref_eval_grad_f64 if dbl else _load().gcdf_ref_eval_grad
    rc = fn(b, len(blob), _ptr(k), K, _ptr(p), Np, _ptr(d), _ptr(J) if with_grad else None, nthreads)
    if rc:
        raise ValueError("oracle rejected the weight blob")
    return d, J


def eval_pairs(blob: bytes, knots, points, kidx, pidx, with_grad: bool = True, nthreads: int = 0):
    """Selected pairs (knots[kidx[i]], points[pidx[i]]): d (n,), J (n, 9)."""
    k, p = _f32(knots, 9), _f32(points, obstacle_dim(blob))
    ki = np.ascontiguousarray(kidx, dtype=np.int64)
    pi = np.ascontiguousarray(pidx, dtype=np.int64)
    assert ki.shape == pi.shape and ki.ndim == 1
    if len(ki) and (ki.min() < 0 or ki.max() >= len(k) or pi.min() < 0 or pi.max() >= len(p)):
        raise IndexError("pair index out of range")
    n = len(ki)
    d = np.empty(n, np.float64)
    J = np.empty((n, 9), np.float64) if with_grad else None
    b = ctypes.create_string_buffer(blob, len(blob))
    rc = _load().gcdf_ref_eval_pairs(b, len(blob), _ptr(k), _ptr(p), _ptr(ki), _ptr(pi), n,
                                     _ptr(d), _ptr(J) if with_grad else None, nthreads)
    if rc:
        raise ValueError("oracle rejected the weight blob")
    return d, J


def project(q, f, J, m_diag):
    """Single-step projection onto the zero set and the weighted eikonal norm
    (Theorem 1): q_z = q - f M^{-1} grad_q f and |grad_q f|_{M^{-1}}, with
    M = diag(m_diag) positive.  q (..., 9), f (...), J (..., 9) broadcast
    together; float64 results (q_z (..., 9), eik (...))."""
    q = np.asarray(q, np.float64)
    f = np.asarray(f, np.float64)
    J = np.asarray(J, np.float64)
    minv = 1.0 / np.asarray(m_diag, np.float64)
    qz = q - f[..., None] * (minv * J)
    eik = np.sqrt(np.sum(minv * J * J, axis=-1))
    return qz, eik


def knot_min(d):
    """Per-row minimum of d (K, Np) and the lowest column index attaining it."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    K, Np = d.shape
    dmin = np.empty(K, np.float64)
    am = np.empty(K, np.int32)
    _load().gcdf_ref_knot_min(_ptr(d), K, Np, _ptr(dmin), _ptr(am))
    return dmin, am


def mse_grad(blob: bytes, knots, points, y):
    """MSE loss over samples (knot i, point i) vs targets y, and d loss / d parameters.

    Returns (loss, grads) where grads is a list [dW1, db1, ..., dw_out, db_out]
    shaped like the weight arrays, float64.
    """
    k, p = _f64(knots, 9), _f64(points, 3)
    y = np.ascontiguousarray(y, dtype=np.float64)
    n = len(k)
    assert len(p) == n and y.shape == (n,)
    width, depth = struct.unpack("<2I", blob[12:20])
    dims = [9] + [width] * depth + [1]
    shapes = []
    for li in range(depth + 1):
        shapes += [(dims[li + 1], dims[li]), (dims[li + 1],)]
    total = sum(int(np.prod(s)) for s in shapes)
    g = np.empty(total, np.float64)
    b = ctypes.create_string_buffer(blob, len(blob))
    loss = _load().gcdf_ref_mse_grad(b, len(blob), _ptr(k), _ptr(p), _ptr(y), n, _ptr(g))
    if np.isnan(loss):
        raise ValueError("oracle rejected the weight blob")
    out, off = [], 0
    for s in shapes:
        c = int(np.prod(s))
        out.append(g[off:off + c].reshape(s))
        off += c
    return loss, out


LAMBDA_PAPER = (5.0, 0.1, 0.01, 0.01)  # loss weights of Sec. V-A


def table1_grad(blob: bytes, knots, points, fstar, Jstar, m_diag, lam=LAMBDA_PAPER):
    """Table I training loss over samples (knot i, point i) and its weight gradient.

    Returns (total, [L_dist, L_grad, L_eikonal, L_tension], grads) with grads
    shaped like the weight arrays, float64.
    """
    k, p = _f64(knots, 9), _f64(points, 3)
    n = len(k)
    fs = np.ascontiguousarray(fstar, dtype=np.float64)
    Js = _f64(Jstar, 9)
    m = np.ascontiguousarray(m_diag, dtype=np.float64)
    lm = np.ascontiguousarray(lam, dtype=np.float64)
    assert len(p) == n and fs.shape == (n,) and Js.shape == (n, 9) and m.shape == (9,) and lm.shape == (4,)
    width, depth = struct.unpack("<2I", blob[12:20])
    dims = [9] + [width] * depth + [1]
    shapes = []
    for li in range(depth + 1):
        shapes += [(dims[li + 1], dims[li]), (dims[li + 1],)]
    total_n = sum(int(np.prod(s)) for s in shapes)
    g = np.empty(total_n, np.float64)
    losses = np.empty(4, np.float64)
    b = ctypes.create_string_buffer(blob, len(blob))
    total = _load().gcdf_ref_table1_grad(b, len(blob), _ptr(k), _ptr(p), _ptr(fs), _ptr(Js), _ptr(m), _ptr(lm), n,
                                         _ptr(losses), _ptr(g))
    if np.isnan(total):
        raise ValueError("oracle rejected the weight blob")
    out, off = [], 0
    for s in shapes:
        c = int(np.prod(s))
        out.append(g[off:off + c].reshape(s))
        off += c
    return total, losses, out
