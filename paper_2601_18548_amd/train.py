"""Training form: the distance network's weight gradients behind torch.autograd.

``GcdfNet.apply(params, knots, points, trainer)`` returns the distances of the
samples (knot i, point i); its backward calls ``gcdf_train_backward``, whose
HIP kernels run the network's reverse mode seeded with dL/dd and reduce the
weight gradients over the batch.  ``params`` is one flat FP32 tensor in the
weight-blob order (W1, b1, ..., w_out, b_out); the optimiser keeps it as the
FP32 master copy, and the kernels pack it (to BF16 for the BF16 precision) at
every call.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import BF16, FP32, PRECISIONS, GcdfError, _check, _stream, library


def param_count(width: int) -> int:
    return int(library().gcdf_param_count(width))


def flat_params(weights, device="cuda"):
    """Flat FP32 parameter tensor (blob order) from a workloads.Weights."""
    import torch

    return torch.from_numpy(np.concatenate([a.ravel() for a in weights.flat_params()]).astype(np.float32)).to(device)


class Trainer:
    def __init__(self, width: int = 256, precision="bf16", max_batch: int = 65536, device: int = 0):
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        h = ctypes.c_void_p()
        _check(library().gcdf_trainer_create(width, prec, device, max_batch, ctypes.byref(h)))
        self._h, self.width, self.precision, self.max_batch = h, width, prec, max_batch

    def close(self):
        if getattr(self, "_h", None):
            library().gcdf_trainer_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, params, knots, points, d=None, stream=None):
        import torch

        B = knots.shape[0]
        if d is None:
            d = torch.empty(B, dtype=torch.float32, device=knots.device)
        self._packed = None
        _check(library().gcdf_train_forward(self._h, params.data_ptr(), knots.data_ptr(), points.data_ptr(), B,
                                            d.data_ptr(), _stream(stream)))
        self._packed = (params, params._version)  # the weights this call packed
        return d

    def packed_is_current(self, params) -> bool:
        """True if the library's packed weights were made from `params` as it is now:
        the same storage (a detached alias shares it and its version counter) at the
        same version."""
        pk = getattr(self, "_packed", None)
        return (pk is not None and pk[0].data_ptr() == params.data_ptr() and pk[1] == params._version
                and pk[0]._version == pk[1])

    def backward(self, params, knots, points, grad_d, grad=None, reuse_packed: bool = False, stream=None):
        """reuse_packed: params is unchanged since the last forward/backward call
        (the weights packed then are reused)."""
        import torch

        B = knots.shape[0]
        if grad is None:
            grad = torch.empty_like(params)
        reuse = bool(reuse_packed) and self.packed_is_current(params)
        self._packed = None
        _check(library().gcdf_train_backward(self._h, params.data_ptr(), knots.data_ptr(), points.data_ptr(), B,
                                             grad_d.data_ptr(), grad.data_ptr(), 1 if reuse else 0,
                                             _stream(stream)))
        self._packed = (params, params._version)
        return grad


    def mse(self, params, knots, points, target, grad=None, d=None, reuse_packed: bool = False, stream=None):
        """Mean squared error of the network distances against target and its weight
        gradient in one pass (gcdf_train_mse): (loss float32[1], grad).
        reuse_packed: params is unchanged since this trainer last packed it (a forward,
        backward or mse call, or an Adam step with this trainer)."""
        import torch

        _check_samples(params, knots, points, self)
        B = knots.shape[0]
        if target is None:
            raise ValueError("target is required")
        for t, name in ((target, "target"), (d, "d")):
            if t is not None:
                _checked(t, name)
                if tuple(t.shape) != (B,) or t.device != params.device:
                    raise ValueError("%s must be (B,) on the parameters' device" % name)
        if grad is None:
            grad = torch.empty_like(params)
        elif tuple(grad.shape) != tuple(params.shape):
            raise ValueError("grad must be shaped like params")
        else:
            _checked(grad, "grad")
        loss = torch.empty(1, dtype=torch.float32, device=params.device)
        reuse = bool(reuse_packed) and self.packed_is_current(params)
        self._packed = None
        _check(library().gcdf_train_mse(self._h, params.data_ptr(), knots.data_ptr(), points.data_ptr(), B,
                                        target.data_ptr(), loss.data_ptr(), grad.data_ptr(),
                                        d.data_ptr() if d is not None else None, 1 if reuse else 0,
                                        _stream(stream)))
        self._packed = (params, params._version)
        return loss, grad

    LAMBDA_PAPER = (5.0, 0.1, 0.01, 0.01)  # loss weights of Sec. V-A

    def table1(self, params, knots, points, fstar, Jstar, m_diag, lam=LAMBDA_PAPER, grad=None, stream=None):
        """Table I loss (4 terms + total, device float32[5]) and its weight gradient."""
        import torch

        B = knots.shape[0]
        if grad is None:
            grad = torch.empty_like(params)
        losses = torch.empty(5, dtype=torch.float32, device=params.device)
        m = (ctypes.c_float * 9)(*[float(v) for v in m_diag])
        lm = (ctypes.c_float * 4)(*[float(v) for v in lam])
        self._packed = None
        _check(library().gcdf_train_table1(self._h, params.data_ptr(), knots.data_ptr(), points.data_ptr(), B,
                                           fstar.data_ptr(), Jstar.data_ptr(), m, lm, losses.data_ptr(),
                                           grad.data_ptr(), _stream(stream)))
        self._packed = (params, params._version)
        return losses, grad


def _checked(t, dtype_name):
    import torch

    if not (t.is_cuda and t.is_contiguous() and t.dtype == torch.float32):
        raise ValueError("%s must be a contiguous float32 CUDA tensor" % dtype_name)
    return t


def _check_samples(params, knots, points, trainer):
    _checked(params, "params")
    _checked(knots, "knots")
    _checked(points, "points")
    if knots.device != params.device or points.device != params.device:
        raise ValueError("params, knots and points must be on one device")
    B = knots.shape[0]
    if knots.dim() != 2 or knots.shape[1] != 9 or tuple(points.shape) != (B, 3):
        raise ValueError("knots must be (B, 9) and points (B, 3)")
    if params.numel() != param_count(trainer.width):
        raise ValueError("params must hold %d floats" % param_count(trainer.width))
    if B > trainer.max_batch:
        raise ValueError("batch %d exceeds the trainer's max_batch %d" % (B, trainer.max_batch))


def _make_function():
    import torch

    class GcdfNet(torch.autograd.Function):
        """d = network(params)(samples); backward -> d loss / d params only."""

        @staticmethod
        def forward(ctx, params, knots, points, trainer):
            _check_samples(params, knots, points, trainer)
            d = trainer.forward(params, knots, points)
            ctx.save_for_backward(params, knots, points)
            ctx.trainer = trainer
            ctx.params = params
            return d

        @staticmethod
        def backward(ctx, grad_d):
            params, knots, points = ctx.saved_tensors
            # reuse the weights packed by the forward if nothing has packed since and
            # the parameters were not modified in place
            g = ctx.trainer.backward(ctx.params, knots, points, grad_d.contiguous().float(), reuse_packed=True)
            ctx.params = None
            return g, None, None, None

    class GcdfMSE(torch.autograd.Function):
        """loss = mean (network(params)(samples) - target)^2; the forward computes the
        weight gradient with it (one training-mode pass), the backward scales it."""

        @staticmethod
        def forward(ctx, params, knots, points, target, trainer):
            # (Trainer.mse checks its arguments, and packs the weights unless this trainer's
            # last packing, e.g. by its Adam step, is of these unchanged parameters)
            loss, g = trainer.mse(params.detach(), knots, points, target, reuse_packed=True)
            ctx.grad = g
            return loss.reshape(())

        @staticmethod
        def backward(ctx, grad_loss):
            g = ctx.grad
            ctx.grad = None
            # the step's own unit seed (a cached 1.0 that nothing writes) needs no scaling
            if grad_loss.data_ptr() != _unit(grad_loss.device).data_ptr():
                g.mul_(grad_loss)
            return g, None, None, None, None

    return GcdfNet, GcdfMSE


_fn = None


def _functions():
    global _fn
    if _fn is None:
        _fn = _make_function()
    return _fn


def gcdf_net(params, knots, points, trainer):
    """Differentiable network distances of the samples (knot i, point i)."""
    return _functions()[0].apply(params, knots, points, trainer)


def gcdf_mse(params, knots, points, target, trainer):
    """Differentiable mean squared error of the network distances of the samples
    (knot i, point i) against target, loss and weight gradient from one fused pass."""
    return _functions()[1].apply(params, knots, points, target, trainer)


class Adam:
    """Adam over one flat FP32 parameter tensor with the library's update kernel
    (gcdf_adam_step: torch.optim.Adam's arithmetic, one launch over the whole
    vector).  Minimal optimiser interface: zero_grad(), step()."""

    def __init__(self, params, lr: float = 5e-3, betas=(0.9, 0.999), eps: float = 1e-8, trainer=None):
        import torch

        if not (params.is_cuda and params.dtype == torch.float32 and params.is_contiguous()):
            raise ValueError("params must be a contiguous float32 CUDA tensor")
        if trainer is not None and params.numel() != param_count(trainer.width):
            raise ValueError("params must hold the trainer's %d floats" % param_count(trainer.width))
        # with a trainer, each step also packs the updated weights into it
        # (gcdf_train_adam_step), so its next loss call skips the packing
        self.trainer = trainer
        self.params, self.lr, self.betas, self.eps = params, float(lr), (float(betas[0]), float(betas[1])), float(eps)
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.t = 0

    def zero_grad(self, set_to_none: bool = False):
        if self.params.grad is not None:
            if set_to_none:
                self.params.grad = None
            else:
                self.params.grad.zero_()

    def step(self, stream=None):
        g = self.params.grad
        if g is None:
            return
        self.t += 1
        p = self.params.detach()
        g = g.contiguous()
        tr = self.trainer
        if tr is not None:
            tr._packed = None
            _check(library().gcdf_train_adam_step(tr._h, p.data_ptr(), g.data_ptr(), self.m.data_ptr(),
                                                  self.v.data_ptr(), self.lr, self.betas[0], self.betas[1],
                                                  self.eps, self.t, _stream(stream)))
        else:
            _check(library().gcdf_adam_step(p.data_ptr(), g.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                                            p.numel(), self.lr, self.betas[0], self.betas[1], self.eps, self.t,
                                            _stream(stream)))
        # the kernel wrote the parameters in place: let torch (and Trainer's packed-weight
        # check) see a new version
        import torch

        torch.autograd.graph.increment_version(self.params)
        if tr is not None:
            tr._packed = (self.params, self.params._version)


def adam(params, lr: float = 5e-3, betas=(0.9, 0.999), trainer=None):
    return Adam(params, lr=lr, betas=betas, trainer=trainer)


_UNIT = {}


def _unit(device):
    """A cached device scalar 1.0 per device (never written), the upstream gradient
    mse_step hands to backward instead of the one loss.backward() would fill."""
    import torch

    t = _UNIT.get(device)
    if t is None:
        t = _UNIT[device] = torch.ones((), dtype=torch.float32, device=device)
    return t


def mse_step(params, opt, trainer, knots, points, targets):
    """One training step: the fused MSE loss through the HIP network, backward,
    optimiser step."""
    opt.zero_grad(set_to_none=True)
    loss = gcdf_mse(params, knots, points, targets, trainer)
    loss.backward(_unit(loss.device))
    opt.step()
    return loss
