"""FP64 reference of the byte-level Mamba predictor (test infrastructure only).

The paper's predictor (Models section, Algorithm 1 "Forward Pass"; Range
coding section, the ``step`` function) is an embedding of the previous byte,
``n_l`` Mamba blocks carrying a per-stream cache, and a linear head giving 256
logits:  (S_{t+1}, l_{t+1}) = Phi_theta(S_t, s_t).

Readings taken where the paper defers to the cited Mamba implementation:

* Block = pre-norm residual ``r <- r + Mixer(LayerNorm(r))``; a final
  LayerNorm before the head; LayerNorm eps 1e-5 with biased variance.
* With ``ffn_mult > 0`` each block is followed by Algorithm 1's feed-forward
  sub-layer taken as printed, ``r <- LayerNorm(FFN(r))`` with no residual
  around it: FFN(r) = W2 GELU(W1 r + b1) + b2, hidden width ffn_mult *
  d_model, GELU the exact Gaussian form u Phi(u) (the paper names neither the
  activation nor the width), its own affine LayerNorm.
* Mixer = Mamba-1: in_proj -> [x; z]; causal depthwise conv1d (kernel K, with
  bias) over x, then SiLU; x_proj -> [delta; B; C] (no bias); dt_proj with bias
  then softplus gives Delta (Appendix A, selection mechanism); the selective
  scan h <- exp(Delta A) h + Delta B x, y = C h + D x (Appendix A, discrete
  recurrence, with A-bar = exp(Delta A) and the first-order input term
  B-bar x = Delta B x); gate y * SiLU(z); out_proj.
* A = -exp(A_log).  softplus(v) = log1p(exp(v)) for v <= 20, else v.

Everything is float64; weights are the float32 flat vector from ``synth``
widened exactly.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

from synth.weights import ModelConfig, unflatten

LN_EPS = 1e-5


# ----------------------------------------------------------------------------
# elementwise pieces
# ----------------------------------------------------------------------------
def layer_norm(x, w, b, eps=LN_EPS):
    """LayerNorm over the last axis, biased variance (Models: layer normalisation)."""
    mu = x.mean(axis=-1, keepdims=True)
    var = ((x - mu) ** 2).mean(axis=-1, keepdims=True)
    return (x - mu) / np.sqrt(var + eps) * w + b


def sigmoid(v):
    return 1.0 / (1.0 + np.exp(-v))


def silu(v):
    return v * sigmoid(v)


def gelu(u):
    """GELU(u) = u Phi(u), Phi the standard normal CDF = (1 + erf(u / sqrt 2)) / 2."""
    return u * 0.5 * (1.0 + erf(u / np.sqrt(2.0)))


def softplus(v):
    """softplus keeps Delta positive (Appendix A, selection mechanism)."""
    v = np.asarray(v, dtype=np.float64)
    return np.where(v <= 20.0, np.log1p(np.exp(np.minimum(v, 20.0))), v)


def softmax(logits):
    """p(a) = exp l(a) / sum_x exp l(x) (Range coding: Probabilities), max-shifted."""
    m = logits.max(axis=-1, keepdims=True)
    e = np.exp(logits - m)
    return e / e.sum(axis=-1, keepdims=True)


# ----------------------------------------------------------------------------
# weights and state
# ----------------------------------------------------------------------------
class Weights:
    """float64 copies of the named tensors of a flat weight vector (float32 as
    stored, or float64 for finite-difference checks)."""

    def __init__(self, cfg: ModelConfig, flat: np.ndarray):
        assert flat.dtype in (np.float32, np.float64)
        self.cfg = cfg
        self.t = {k: v.astype(np.float64) for k, v in unflatten(cfg, flat).items()}

    def layer(self, l):
        p = f"layers.{l}."
        return {k[len(p):]: v for k, v in self.t.items() if k.startswith(p)}


class StreamState:
    """Per-stream cache S_t: for each layer the conv shift register (last K-1
    inputs of the conv) and the SSM state h (Range coding: stream cache)."""

    def __init__(self, cfg: ModelConfig, n_lanes: int):
        Di, N, K = cfg.d_inner, cfg.d_state, cfg.d_conv
        self.conv = [np.zeros((n_lanes, Di, K - 1)) for _ in range(cfg.n_layers)]
        self.h = [np.zeros((n_lanes, Di, N)) for _ in range(cfg.n_layers)]


# ----------------------------------------------------------------------------
# the step function Phi_theta
# ----------------------------------------------------------------------------
def proj_mm(a, w, proj="f64"):
    """a @ w.T for the projections (in_proj, out_proj, head): exact in float64,
    or in the FP8 (E4M3) mode of oracle.fp8 when proj == "fp8"."""
    if proj == "fp8":
        from oracle import fp8
        return fp8.matmul_t(a, w)
    return a @ w.T


def mixer_step(lw, cfg: ModelConfig, a, conv_buf, h, proj="f64"):
    """One Mamba mixer step for a batch of lanes.

    a: [B, D] normalised input; conv_buf: [B, Di, K-1] (updated in place);
    h: [B, Di, N] (updated in place).  Returns the mixer output [B, D].
    """
    Di, N, R = cfg.d_inner, cfg.d_state, cfg.dt_rank
    xz = proj_mm(a, lw["in_proj_w"], proj)          # [B, 2Di]
    x, z = xz[:, :Di], xz[:, Di:]
    win = np.concatenate([conv_buf, x[:, :, None]], axis=2)       # [B, Di, K]
    xc = (win * lw["conv_w"][None]).sum(axis=2) + lw["conv_b"]
    conv_buf[:] = win[:, :, 1:]
    xs = silu(xc)
    dbc = xs @ lw["x_proj_w"].T                     # [B, R + 2N]
    delta, Bv, Cv = dbc[:, :R], dbc[:, R:R + N], dbc[:, R + N:]
    dt = softplus(delta @ lw["dt_proj_w"].T + lw["dt_proj_b"])    # [B, Di]
    A = -np.exp(lw["A_log"])                         # [Di, N]
    dA = np.exp(dt[:, :, None] * A[None])            # A-bar = exp(Delta A)
    h[:] = dA * h + (dt * xs)[:, :, None] * Bv[:, None, :]
    y = (h * Cv[:, None, :]).sum(axis=2) + lw["D"] * xs
    g = y * silu(z)
    return proj_mm(g, lw["out_proj_w"], proj)


def ffn_step(lw, r, proj="f64"):
    """Algorithm 1's sub-layer after a Mamba block: LayerNorm(FFN(r))."""
    u = proj_mm(r, lw["ffn_w1"], proj) + lw["ffn_b1"]
    f = proj_mm(gelu(u), lw["ffn_w2"], proj) + lw["ffn_b2"]
    return layer_norm(f, lw["ffn_norm_w"], lw["ffn_norm_b"])


def step(W: Weights, S: StreamState, y_prev, proj="f64"):
    """(S_{t+1}, l_{t+1}) = Phi_theta(S_t, s_t) for a batch of lanes.

    y_prev: int array [B] of the bytes just seen.  S is updated in place.
    Returns logits [B, 256] for the next byte.  proj selects the projection
    arithmetic (proj_mm).
    """
    cfg = W.cfg
    r = W.t["embed"][np.asarray(y_prev, dtype=np.int64)]           # ByteEmbed
    for l in range(cfg.n_layers):
        lw = W.layer(l)
        a = layer_norm(r, lw["norm_w"], lw["norm_b"])
        r = r + mixer_step(lw, cfg, a, S.conv[l], S.h[l], proj)
        if cfg.ffn_mult:
            r = ffn_step(lw, r, proj)
    rf = layer_norm(r, W.t["norm_f_w"], W.t["norm_f_b"])
    return proj_mm(rf, W.t["head_w"], proj) + W.t["head_b"]        # Head


def stream_logits(W: Weights, seqs, proj="f64"):
    """Logits predicting byte t+1 from bytes <= t, for equal-length lanes.

    seqs: uint8 [B, T].  Returns [B, T-1, 256]: row t predicts seqs[:, t+1].
    Runs the step recurrence from the zero state, one byte at a time.
    """
    seqs = np.asarray(seqs)
    B, T = seqs.shape
    S = StreamState(W.cfg, B)
    out = np.empty((B, max(T - 1, 0), 256))
    for t in range(T - 1):
        out[:, t] = step(W, S, seqs[:, t], proj)
    return out


# ----------------------------------------------------------------------------
# the selective scan on its own (used by pins and by the gradient oracle)
# ----------------------------------------------------------------------------
def selective_scan(x, dt, A, Bm, Cm, Dv, h0=None, return_h=False):
    """Sequential recurrence over time (Appendix A, discrete recurrence).

    x, dt: [T, Di]; A: [Di, N]; Bm, Cm: [T, N]; Dv: [Di].
    h_t = exp(dt_t A) h_{t-1} + dt_t B_t x_t ;  y_t = C_t . h_t + D x_t.
    """
    T, Di = x.shape
    N = A.shape[1]
    h = np.zeros((Di, N)) if h0 is None else h0.copy()
    ys = np.empty((T, Di))
    hs = np.empty((T, Di, N))
    for t in range(T):
        h = np.exp(dt[t][:, None] * A) * h + (dt[t] * x[t])[:, None] * Bm[t][None, :]
        ys[t] = h @ Cm[t] + Dv * x[t]
        hs[t] = h
    return (ys, hs) if return_h else ys
