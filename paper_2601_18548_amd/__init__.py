"""MI355X-native batched neural GCDF queries (libgcdf) -- Python binding.

The binding only marshals arguments: every step of the query runs in the HIP
kernels of ``libgcdf.so`` (built in-tree by ``build.py``).  PyTorch provides the
device memory (tensors) and the stream.  If the library is missing this module
raises instead of computing anything itself.

Names follow the C ABI in ``include/gcdf.h``:
``Context.eval``, ``Context.eval_grad``, ``Context.knot_min``,
``Context.submit`` / ``Context.poll``.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgcdf.so")

FP32, BF16, BF16X2 = 0, 1, 2
PRECISIONS = {"fp32": FP32, "bf16": BF16, "bf16x2": BF16X2}
OK, PENDING, EINVAL, ENOMEM, EDEVICE, EBUSY = 0, 1, 2, 3, 4, 5
STATUS_NAMES = {0: "OK", 1: "PENDING", 2: "EINVAL", 3: "ENOMEM", 4: "EDEVICE", 5: "EBUSY"}


class GcdfError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


class _Config(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("depth", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("device", ctypes.c_int32), ("max_knots", ctypes.c_int64), ("serve_mem_budget", ctypes.c_size_t),
                ("serve_slots", ctypes.c_int32), ("reserved", ctypes.c_int32 * 7)]


class _Request(ctypes.Structure):
    _fields_ = [("knots", ctypes.c_void_p), ("K", ctypes.c_int64), ("points", ctypes.c_void_p),
                ("Np", ctypes.c_int64), ("d", ctypes.c_void_p), ("J", ctypes.c_void_p),
                ("dmin", ctypes.c_void_p), ("argmin", ctypes.c_void_p)]


_lib = None


def library() -> ctypes.CDLL:
    """Load libgcdf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libgcdf.so is not built (run paper_2601_18548_amd/build.py); "
                          "there is no fallback implementation")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64 = ctypes.c_void_p, ctypes.c_int64
    lib.gcdf_create.argtypes = [ctypes.POINTER(_Config), P, ctypes.c_size_t, ctypes.POINTER(P)]
    lib.gcdf_create.restype = ctypes.c_int
    lib.gcdf_destroy.argtypes = [P]
    lib.gcdf_destroy.restype = None
    lib.gcdf_last_error.argtypes = [P]
    lib.gcdf_last_error.restype = ctypes.c_char_p
    lib.gcdf_eval.argtypes = [P, P, I64, P, I64, P, P]
    lib.gcdf_eval.restype = ctypes.c_int
    lib.gcdf_eval_grad.argtypes = [P, P, I64, P, I64, P, P, P]
    lib.gcdf_eval_grad.restype = ctypes.c_int
    lib.gcdf_knot_min.argtypes = [P, P, I64, P, I64, P, P, P, P]
    lib.gcdf_knot_min.restype = ctypes.c_int
    lib.gcdf_query.argtypes = [P, P, I64, P, I64, P, P, P, P, P, P]
    lib.gcdf_query.restype = ctypes.c_int
    lib.gcdf_param_count.argtypes = [ctypes.c_int32]
    lib.gcdf_param_count.restype = ctypes.c_int64
    lib.gcdf_trainer_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, I64, ctypes.POINTER(P)]
    lib.gcdf_trainer_create.restype = ctypes.c_int
    lib.gcdf_trainer_destroy.argtypes = [P]
    lib.gcdf_trainer_destroy.restype = None
    lib.gcdf_train_forward.argtypes = [P, P, P, P, I64, P, P]
    lib.gcdf_train_forward.restype = ctypes.c_int
    lib.gcdf_train_backward.argtypes = [P, P, P, P, I64, P, P, P]
    lib.gcdf_train_backward.restype = ctypes.c_int
    lib.gcdf_submit.argtypes = [P, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_uint64)]
    lib.gcdf_submit.restype = ctypes.c_int
    lib.gcdf_poll.argtypes = [P, ctypes.c_uint64]
    lib.gcdf_poll.restype = ctypes.c_int
    _lib = lib
    return lib


EXPORTED = ["gcdf_create", "gcdf_destroy", "gcdf_last_error", "gcdf_eval", "gcdf_eval_grad",
            "gcdf_knot_min", "gcdf_query", "gcdf_submit", "gcdf_poll", "gcdf_param_count",
            "gcdf_trainer_create", "gcdf_trainer_destroy", "gcdf_train_forward", "gcdf_train_backward"]


def _check(st: int, ctx=None):
    if st != OK and st != PENDING:
        msg = library().gcdf_last_error(ctx).decode(errors="replace")
        raise GcdfError(st, msg)
    return st


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _need(t, shape, name):
    import torch

    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError("%s must be a contiguous float32 CUDA tensor of shape %s" % (name, tuple(shape)))


class Context:
    """A libgcdf context: one network on one device."""

    def __init__(self, weight_blob: bytes, width: int, precision="bf16x2", device: int = 0, depth: int = 4,
                 max_knots: int = 0, serve_mem_budget: int = 0, serve_slots: int = 0):
        lib = library()
        cfg = _Config()
        cfg.width, cfg.depth = width, depth
        cfg.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        cfg.device, cfg.max_knots = device, max_knots
        cfg.serve_mem_budget, cfg.serve_slots = serve_mem_budget, serve_slots
        h = ctypes.c_void_p()
        buf = ctypes.create_string_buffer(weight_blob, len(weight_blob))
        _check(lib.gcdf_create(ctypes.byref(cfg), buf, len(weight_blob), ctypes.byref(h)))
        self._h = h
        self.width, self.precision, self.device = width, cfg.precision, device

    def close(self):
        if getattr(self, "_h", None):
            library().gcdf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- queries ------------------------------------------------------------
    def eval(self, knots, points, d=None, stream=None):
        import torch

        K, Np = knots.shape[0], points.shape[0]
        _need(knots, (K, 9), "knots")
        _need(points, (Np, 3), "points")
        if d is None:
            d = torch.empty((K, Np), dtype=torch.float32, device=knots.device)
        _need(d, (K, Np), "d")
        _check(library().gcdf_eval(self._h, _ptr(knots), K, _ptr(points), Np, _ptr(d), _stream(stream)), self._h)
        return d

    def eval_grad(self, knots, points, d=None, J=None, stream=None):
        import torch

        K, Np = knots.shape[0], points.shape[0]
        _need(knots, (K, 9), "knots")
        _need(points, (Np, 3), "points")
        if d is None:
            d = torch.empty((K, Np), dtype=torch.float32, device=knots.device)
        if J is None:
            J = torch.empty((K, Np, 9), dtype=torch.float32, device=knots.device)
        _need(d, (K, Np), "d")
        _need(J, (K, Np, 9), "J")
        _check(library().gcdf_eval_grad(self._h, _ptr(knots), K, _ptr(points), Np, _ptr(d), _ptr(J),
                                        _stream(stream)), self._h)
        return d, J

    def knot_min(self, knots, points, with_jacobian: bool = False, stream=None):
        import torch

        K, Np = knots.shape[0], points.shape[0]
        _need(knots, (K, 9), "knots")
        _need(points, (Np, 3), "points")
        dmin = torch.empty(K, dtype=torch.float32, device=knots.device)
        am = torch.empty(K, dtype=torch.int32, device=knots.device)
        Jm = torch.empty((K, 9), dtype=torch.float32, device=knots.device) if with_jacobian else None
        _check(library().gcdf_knot_min(self._h, _ptr(knots), K, _ptr(points), Np, _ptr(dmin), _ptr(am), _ptr(Jm),
                                       _stream(stream)), self._h)
        return (dmin, am, Jm) if with_jacobian else (dmin, am)

    def query(self, knots, points, d=None, J=None, dmin=None, argmin=None, Jmin=None, stream=None):
        """All requested outputs from one fused pass (preallocated tensors or None)."""
        K, Np = knots.shape[0], points.shape[0]
        _need(knots, (K, 9), "knots")
        _need(points, (Np, 3), "points")
        if d is not None:
            _need(d, (K, Np), "d")
        if J is not None:
            _need(J, (K, Np, 9), "J")
        _check(library().gcdf_query(self._h, _ptr(knots), K, _ptr(points), Np, _ptr(d), _ptr(J), _ptr(dmin),
                                    _ptr(argmin), _ptr(Jmin), _stream(stream)), self._h)
        return d, J, dmin, argmin, Jmin

    # -- serving ------------------------------------------------------------
    def submit(self, knots, points, d=None, J=None, dmin=None, argmin=None) -> int:
        req = _Request()
        req.knots, req.K = knots.data_ptr(), knots.shape[0]
        req.points, req.Np = points.data_ptr(), points.shape[0]
        req.d = d.data_ptr() if d is not None else None
        req.J = J.data_ptr() if J is not None else None
        req.dmin = dmin.data_ptr() if dmin is not None else None
        req.argmin = argmin.data_ptr() if argmin is not None else None
        t = ctypes.c_uint64()
        _check(library().gcdf_submit(self._h, ctypes.byref(req), ctypes.byref(t)), self._h)
        return t.value

    def poll(self, ticket: int) -> bool:
        return _check(library().gcdf_poll(self._h, ticket), self._h) == OK
