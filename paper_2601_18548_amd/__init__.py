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

FP32, BF16, BF16X2, BF16X2_F16 = 0, 1, 2, 3
PRECISIONS = {"fp32": FP32, "bf16": BF16, "bf16x2": BF16X2, "bf16x2_f16": BF16X2_F16}
OK, PENDING, EINVAL, ENOMEM, EDEVICE, EBUSY, ERANGE = 0, 1, 2, 3, 4, 5, 6
STATUS_NAMES = {0: "OK", 1: "PENDING", 2: "EINVAL", 3: "ENOMEM", 4: "EDEVICE", 5: "EBUSY", 6: "ERANGE"}


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
                ("dmin", ctypes.c_void_p), ("argmin", ctypes.c_void_p), ("Jmin", ctypes.c_void_p)]


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
    lib.gcdf_query_noalloc.argtypes = [P, P, I64, P, I64, P, P, P, P, P, P]
    lib.gcdf_query_noalloc.restype = ctypes.c_int
    lib.gcdf_param_count.argtypes = [ctypes.c_int32]
    lib.gcdf_param_count.restype = ctypes.c_int64
    lib.gcdf_trainer_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, I64, ctypes.POINTER(P)]
    lib.gcdf_trainer_create.restype = ctypes.c_int
    lib.gcdf_trainer_destroy.argtypes = [P]
    lib.gcdf_trainer_destroy.restype = None
    lib.gcdf_train_forward.argtypes = [P, P, P, P, I64, P, P]
    lib.gcdf_train_forward.restype = ctypes.c_int
    lib.gcdf_train_backward.argtypes = [P, P, P, P, I64, P, P, ctypes.c_int32, P]
    lib.gcdf_train_backward.restype = ctypes.c_int
    lib.gcdf_train_mse.argtypes = [P, P, P, P, I64, P, P, P, P, ctypes.c_int32, P]
    lib.gcdf_train_mse.restype = ctypes.c_int
    lib.gcdf_train_table1.argtypes = [P, P, P, P, I64, P, P, P, P, P, P, P]
    lib.gcdf_train_table1.restype = ctypes.c_int
    lib.gcdf_train_adam_step.argtypes = [P, P, P, P, P, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_float, I64, P]
    lib.gcdf_train_adam_step.restype = ctypes.c_int
    lib.gcdf_adam_step.argtypes = [P, P, P, P, I64, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                   I64, P]
    lib.gcdf_adam_step.restype = ctypes.c_int
    F = ctypes.c_float
    lib.gcdf_partition_count.argtypes = [P, P, I64, I64, P, I64, F, P, P]
    lib.gcdf_partition_count.restype = ctypes.c_int
    lib.gcdf_partition_fill.argtypes = [P, P, I64, I64, P, I64, F, P, P, I64, P]
    lib.gcdf_partition_fill.restype = ctypes.c_int
    lib.gcdf_eval_grad_csr.argtypes = [P, P, I64, P, I64, P, P, I64, P, P, P]
    lib.gcdf_eval_grad_csr.restype = ctypes.c_int
    lib.gcdf_jacobian_pattern.argtypes = [P, P, I64, I64, ctypes.c_int32, I64, P, P, P]
    lib.gcdf_jacobian_pattern.restype = ctypes.c_int
    lib.gcdf_project.argtypes = [P, P, I64, I64, P, P, P, P, P, P]
    lib.gcdf_project.restype = ctypes.c_int
    lib.gcdf_project_csr.argtypes = [P, P, I64, P, I64, P, P, P, P, P, P]
    lib.gcdf_project_csr.restype = ctypes.c_int
    lib.gcdf_submit.argtypes = [P, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_uint64)]
    lib.gcdf_submit.restype = ctypes.c_int
    lib.gcdf_poll.argtypes = [P, ctypes.c_uint64]
    lib.gcdf_poll.restype = ctypes.c_int
    _lib = lib
    return lib


EXPORTED = ["gcdf_create", "gcdf_destroy", "gcdf_last_error", "gcdf_eval", "gcdf_eval_grad",
            "gcdf_knot_min", "gcdf_query", "gcdf_query_noalloc", "gcdf_submit", "gcdf_poll", "gcdf_param_count",
            "gcdf_trainer_create", "gcdf_trainer_destroy", "gcdf_train_forward", "gcdf_train_backward",
            "gcdf_partition_count", "gcdf_partition_fill", "gcdf_eval_grad_csr", "gcdf_jacobian_pattern",
            "gcdf_project", "gcdf_project_csr", "gcdf_adam_step", "gcdf_train_table1", "gcdf_train_mse",
            "gcdf_train_adam_step"]


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


def _need(t, shape, name, dtype=None, device=None):
    """Raise unless t is a contiguous CUDA tensor of this shape and dtype (float32
    by default), on `device` if given."""
    import torch

    dtype = torch.float32 if dtype is None else dtype
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError("%s must be a contiguous %s CUDA tensor of shape %s" % (name, dtype, tuple(shape)))
    if device is not None and t.device != device:
        raise ValueError("%s is on %s, expected %s" % (name, t.device, device))


def _need_min(K, dmin, argmin, Jmin, device):
    """Shapes of the per-knot minimum outputs (None = not requested)."""
    import torch

    if dmin is not None:
        _need(dmin, (K,), "dmin", device=device)
    if argmin is not None:
        _need(argmin, (K,), "argmin", torch.int32, device=device)
    if Jmin is not None:
        _need(Jmin, (K, 9), "Jmin", device=device)


class Context:
    """A libgcdf context: one network on one device.

    precision: "fp32", "bf16" (fast, misses the 1e-3 bar), "bf16x2" (split BF16
    products, FP32-class error) or "bf16x2_f16" (split BF16 forward products, FP16
    reverse-sweep products: d as bf16x2, Jacobian relative error a few 1e-3)."""

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
        # network input width from the blob header: 9 (points, (Np, 3)) or 10
        # (spheres (x, y, z, r), (Np, 4)); the library has validated it
        self.in_dim = int.from_bytes(weight_blob[8:12], "little")
        self.obstacle_dim = self.in_dim - 6
        self._live = {}  # serving ticket -> the request's tensors, until complete

    def close(self):
        if getattr(self, "_h", None):
            library().gcdf_destroy(self._h)  # waits for every serving request
            self._h = None
            self._live = {}

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
        _need(points, (Np, self.obstacle_dim), "points")
        if d is None:
            d = torch.empty((K, Np), dtype=torch.float32, device=knots.device)
        _need(d, (K, Np), "d")
        _check(library().gcdf_eval(self._h, _ptr(knots), K, _ptr(points), Np, _ptr(d), _stream(stream)), self._h)
        return d

    def eval_grad(self, knots, points, d=None, J=None, stream=None):
        import torch

        K, Np = knots.shape[0], points.shape[0]
        _need(knots, (K, 9), "knots")
        _need(points, (Np, self.obstacle_dim), "points")
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
        _need(points, (Np, self.obstacle_dim), "points")
        dmin = torch.empty(K, dtype=torch.float32, device=knots.device)
        am = torch.empty(K, dtype=torch.int32, device=knots.device)
        Jm = torch.empty((K, 9), dtype=torch.float32, device=knots.device) if with_jacobian else None
        _check(library().gcdf_knot_min(self._h, _ptr(knots), K, _ptr(points), Np, _ptr(dmin), _ptr(am), _ptr(Jm),
                                       _stream(stream)), self._h)
        return (dmin, am, Jm) if with_jacobian else (dmin, am)

    def query(self, knots, points, d=None, J=None, dmin=None, argmin=None, Jmin=None, stream=None,
              noalloc: bool = False):
        """All requested outputs from one fused pass (preallocated tensors or None).
        noalloc: through gcdf_query_noalloc (the library's fixed per-GPU key array,
        at most 65,536 knots with the minimum; calls on one GPU must not overlap)."""
        K, Np = knots.shape[0], points.shape[0]
        _need(knots, (K, 9), "knots")
        _need(points, (Np, self.obstacle_dim), "points")
        dev = knots.device
        _need(points, (Np, self.obstacle_dim), "points", device=dev)
        if d is not None:
            _need(d, (K, Np), "d", device=dev)
        if J is not None:
            _need(J, (K, Np, 9), "J", device=dev)
        _need_min(K, dmin, argmin, Jmin, dev)
        fn = library().gcdf_query_noalloc if noalloc else library().gcdf_query
        _check(fn(self._h, _ptr(knots), K, _ptr(points), Np, _ptr(d), _ptr(J), _ptr(dmin), _ptr(argmin), _ptr(Jmin),
                  _stream(stream)), self._h)
        return d, J, dmin, argmin, Jmin

    # -- obstacle partitions and the sparse constraint Jacobian --------------
    def partition(self, ref, points, radius: float, ref_stride: int | None = None, stream=None):
        """CSR partitions (offsets int64[N+1], idx int32[total]) of the points
        around each reference base position (rows of ``ref``; its first two
        columns are (x, y)).  Synchronises once to size idx."""
        import torch

        if ref.dtype != torch.float32 or not ref.is_cuda or not ref.is_contiguous() or ref.dim() != 2:
            raise ValueError("ref must be a contiguous 2-D float32 CUDA tensor")
        N, Np = ref.shape[0], points.shape[0]
        _need(points, (Np, self.obstacle_dim), "points")
        stride = ref.shape[1] if ref_stride is None else ref_stride
        off = torch.empty(N + 1, dtype=torch.int64, device=ref.device)
        lib = library()
        _check(lib.gcdf_partition_count(self._h, _ptr(ref), N, stride, _ptr(points), Np, float(radius), _ptr(off),
                                        _stream(stream)), self._h)
        total = int(off[-1].item())
        idx = torch.empty(max(total, 1), dtype=torch.int32, device=ref.device)
        _check(lib.gcdf_partition_fill(self._h, _ptr(ref), N, stride, _ptr(points), Np, float(radius), _ptr(off),
                                       _ptr(idx), total, _stream(stream)), self._h)
        return off, idx[:total]

    def eval_grad_csr(self, knots, points, offsets, idx, with_grad: bool = True, c=None, J=None, stream=None):
        """Stacked constraints c (float32[total]) and gradient rows J (float32[total][9])."""
        import torch

        N, Np, total = knots.shape[0], points.shape[0], idx.shape[0]
        _need(knots, (N, 9), "knots")
        _need(points, (Np, self.obstacle_dim), "points")
        if offsets.dtype != torch.int64 or idx.dtype != torch.int32 or offsets.shape[0] != N + 1:
            raise ValueError("offsets must be int64[N+1] and idx int32[total]")
        if c is None:
            c = torch.empty(total, dtype=torch.float32, device=knots.device)
        if with_grad and J is None:
            J = torch.empty((total, 9), dtype=torch.float32, device=knots.device)
        _check(library().gcdf_eval_grad_csr(self._h, _ptr(knots), N, _ptr(points), Np, _ptr(offsets), _ptr(idx),
                                            total, _ptr(c), _ptr(J) if with_grad else None, _stream(stream)), self._h)
        return (c, J) if with_grad else c

    def jacobian_pattern(self, offsets, total: int, state_dim: int = 18, col0: int = 0, stream=None):
        """CSR pattern (row_ptr int64[total+1], cols int32[9 total]) whose values are J rows."""
        import torch

        N = offsets.shape[0] - 1
        row_ptr = torch.empty(total + 1, dtype=torch.int64, device=offsets.device)
        cols = torch.empty(max(9 * total, 1), dtype=torch.int32, device=offsets.device)
        _check(library().gcdf_jacobian_pattern(self._h, _ptr(offsets), N, total, state_dim, col0, _ptr(row_ptr),
                                               _ptr(cols), _stream(stream)), self._h)
        return row_ptr, cols[:9 * total]

    def project(self, knots, d, J, m_diag, offsets=None, with_qz: bool = True, with_eik: bool = True, stream=None):
        """Theorem 1 projection: (qz, eik) for dense rows (d (K, Np), J (K, Np, 9))
        or, with ``offsets``, the stacked CSR rows (c (total,), J (total, 9))."""
        import torch

        m = (ctypes.c_float * 9)(*[float(v) for v in m_diag])
        N = knots.shape[0]
        _need(knots, (N, 9), "knots")
        shape = tuple(d.shape)
        _need(d, shape, "d")
        _need(J, shape + (9,), "J")
        qz = torch.empty(shape + (9,), dtype=torch.float32, device=d.device) if with_qz else None
        eik = torch.empty(shape, dtype=torch.float32, device=d.device) if with_eik else None
        lib = library()
        if offsets is None:
            if len(shape) != 2 or shape[0] != N:
                raise ValueError("dense d must be (K, Np)")
            st = lib.gcdf_project(self._h, _ptr(knots), N, shape[1], _ptr(d), _ptr(J), m, _ptr(qz), _ptr(eik),
                                  _stream(stream))
        else:
            if len(shape) != 1 or offsets.dtype != torch.int64 or offsets.shape[0] != N + 1:
                raise ValueError("CSR c must be (total,) with offsets int64[N+1]")
            st = lib.gcdf_project_csr(self._h, _ptr(knots), N, _ptr(offsets), shape[0], _ptr(d), _ptr(J), m,
                                      _ptr(qz), _ptr(eik), _stream(stream))
        _check(st, self._h)
        return qz, eik

    # -- serving ------------------------------------------------------------
    def submit(self, knots, points, d=None, J=None, dmin=None, argmin=None, Jmin=None) -> int:
        """Queue a serving request.  The serving loop runs on the library's own
        stream, so the current torch stream (which may still be producing the
        inputs or initialising the outputs) is synchronised first.  The request's
        tensors are kept alive here until poll() reports it complete."""
        import torch

        K, Np = knots.shape[0], points.shape[0]
        dev = knots.device
        _need(knots, (K, 9), "knots")
        _need(points, (Np, self.obstacle_dim), "points", device=dev)
        if d is not None:
            _need(d, (K, Np), "d", device=dev)
        if J is not None:
            _need(J, (K, Np, 9), "J", device=dev)
        _need_min(K, dmin, argmin, Jmin, dev)
        torch.cuda.current_stream(dev).synchronize()
        req = _Request()
        req.knots, req.K = knots.data_ptr(), K
        req.points, req.Np = points.data_ptr(), Np
        req.d = d.data_ptr() if d is not None else None
        req.J = J.data_ptr() if J is not None else None
        req.dmin = dmin.data_ptr() if dmin is not None else None
        req.argmin = argmin.data_ptr() if argmin is not None else None
        req.Jmin = Jmin.data_ptr() if Jmin is not None else None
        t = ctypes.c_uint64()
        _check(library().gcdf_submit(self._h, ctypes.byref(req), ctypes.byref(t)), self._h)
        # the device writes through these pointers until the request completes
        self._live[t.value] = (knots, points, d, J, dmin, argmin, Jmin)
        return t.value

    def poll(self, ticket: int) -> bool:
        try:
            done = _check(library().gcdf_poll(self._h, ticket), self._h) == OK
        except GcdfError:
            self._live.pop(ticket, None)
            raise
        if done:
            self._live.pop(ticket, None)
        return done
