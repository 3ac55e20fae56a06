"""Training of the predictor on the GPU (argument marshalling over libboa).

* :class:`SelectiveScan` -- ``torch.autograd.Function`` whose forward and
  backward are the library's selective-scan kernels (chunked forward keeping
  the state every ``chunk_t`` steps, hand-written reverse recurrence with
  chunk recomputation);
* :func:`loss_and_grad` -- mean next-byte cross-entropy of device sequences
  and its gradient in the flat weight layout;
* :func:`train_step` / :func:`train` -- AdamW steps (the optimiser moments
  live with the model in the library).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib


def _stream_ptr():
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


def opts(lr=1e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.01, grad_clip=1.0, warmup=100, steps=0,
         batch=32, seq_len=8192, chunk_t=256, seed=1, dtype="f32") -> _lib.boa_train_opts:
    o = _lib.boa_train_opts()
    o.lr, o.beta1, o.beta2, o.eps = lr, betas[0], betas[1], eps
    o.weight_decay, o.grad_clip = weight_decay, grad_clip if grad_clip > 0 else -1.0
    o.warmup, o.steps, o.batch, o.seq_len, o.chunk_t, o.seed = warmup, steps, batch, seq_len, chunk_t, seed
    o.dtype = _lib.DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    return o


def loss_and_grad(model, tokens, chunk_t: int = 256, dtype="f32"):
    """tokens: device uint8 [B, T].  Returns (mean loss in nats, grad float32 device tensor)."""
    import torch
    assert tokens.is_cuda and tokens.dtype == torch.uint8 and tokens.dim() == 2
    tokens = tokens.contiguous()
    B, T = tokens.shape
    grad = torch.empty(model.n_params, dtype=torch.float32, device=tokens.device)
    loss = torch.empty(1, dtype=torch.float64, device=tokens.device)
    dt = _lib.DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    _lib.check(_lib.load().boa_loss_grad_dev(model.handle, tokens.data_ptr(), B, T, chunk_t, dt, loss.data_ptr(),
                                             grad.data_ptr(), _stream_ptr()))
    return float(loss.item()), grad


def optimizer_step(model, grad, o=None) -> None:
    """One AdamW step of the model's master weights from a device float32 gradient (flat layout)."""
    import torch
    assert grad.is_cuda and grad.dtype == torch.float32 and grad.numel() == model.n_params
    oo = o if o is not None else opts()
    _lib.check(_lib.load().boa_optimizer_step_dev(model.handle, grad.contiguous().data_ptr(), C.byref(oo),
                                                  _stream_ptr()))


def save_state(model, path: str) -> None:
    """Training checkpoint: weights, AdamW moments and step count."""
    _lib.check(_lib.load().boa_train_state_save(model.handle, path.encode()))


def load_state(model, path: str) -> None:
    _lib.check(_lib.load().boa_train_state_load(model.handle, path.encode()))


def steps_done(model) -> int:
    v = C.c_uint64()
    _lib.check(_lib.load().boa_train_steps_done(model.handle, C.byref(v)))
    return int(v.value)


def train_step(model, tokens, o=None) -> float:
    import torch
    tokens = tokens.contiguous()
    B, T = tokens.shape
    loss = torch.empty(1, dtype=torch.float64, device=tokens.device)
    oo = o if o is not None else opts()
    _lib.check(_lib.load().boa_train_step_dev(model.handle, tokens.data_ptr(), B, T, C.byref(oo), loss.data_ptr(),
                                              _stream_ptr()))
    return float(loss.item())


def train(model, data, o) -> np.ndarray:
    """Host-level train(model, bytes): o.steps AdamW steps; returns per-step losses (nats)."""
    buf = np.ascontiguousarray(np.frombuffer(bytes(data), dtype=np.uint8) if not isinstance(data, np.ndarray)
                               else data, dtype=np.uint8)
    losses = np.zeros(max(int(o.steps), 1), dtype=np.float32)
    _lib.check(_lib.load().boa_train(model.handle, buf.ctypes.data, buf.size, C.byref(o), losses.ctypes.data,
                                     losses.size))
    return losses[:int(o.steps)]


def _make_scan_fn():
    import torch

    class SelectiveScan(torch.autograd.Function):
        """y = selective_scan(x, dt, A_log, B, C, D) on the library's kernels.

        x, dt: [Bt, T, Di]; A_log: [Di, 16]; B, C: [Bt, T, 16]; D: [Di]; float32 CUDA."""

        @staticmethod
        def forward(ctx, x, dt, A_log, Bm, Cm, Dv, chunk_t=256):
            x, dt, A_log, Dv = (t.contiguous().float() for t in (x, dt, A_log, Dv))
            bc = torch.cat([Bm, Cm], dim=-1).contiguous().float()
            Bt, T, Di = x.shape
            nch = (T + chunk_t - 1) // chunk_t
            y = torch.empty_like(x)
            hsave = torch.empty((Bt, nch, 16, Di), dtype=torch.float32, device=x.device)
            _lib.check(_lib.load().boa_scan_fwd_dev(x.data_ptr(), dt.data_ptr(), A_log.data_ptr(), bc.data_ptr(),
                                                    Dv.data_ptr(), Bt, T, Di, chunk_t, y.data_ptr(),
                                                    hsave.data_ptr(), _stream_ptr()))
            ctx.save_for_backward(x, dt, A_log, bc, Dv, hsave)
            ctx.chunk_t = chunk_t
            return y

        @staticmethod
        def backward(ctx, dy):
            x, dt, A_log, bc, Dv, hsave = ctx.saved_tensors
            Bt, T, Di = x.shape
            dy = dy.contiguous().float()
            dx, ddt = torch.empty_like(x), torch.empty_like(dt)
            dbc = torch.empty_like(bc)
            dA = torch.zeros_like(A_log)
            dD = torch.zeros_like(Dv)
            _lib.check(_lib.load().boa_scan_bwd_dev(x.data_ptr(), dt.data_ptr(), A_log.data_ptr(), bc.data_ptr(),
                                                    Dv.data_ptr(), dy.data_ptr(), Bt, T, Di, ctx.chunk_t,
                                                    hsave.data_ptr(), dx.data_ptr(), ddt.data_ptr(), dbc.data_ptr(),
                                                    dA.data_ptr(), dD.data_ptr(), _stream_ptr()))
            return dx, ddt, dA, dbc[..., :16], dbc[..., 16:], dD, None

    return SelectiveScan


_SCAN = None


def selective_scan(x, dt, A_log, Bm, Cm, Dv, chunk_t: int = 256):
    global _SCAN
    if _SCAN is None:
        _SCAN = _make_scan_fn()
    return _SCAN.apply(x, dt, A_log, Bm, Cm, Dv, chunk_t)
