"""FP64 cross-entropy loss, hand-written reverse mode and AdamW (test infrastructure only).

The predictor is trained by minimising the cross-entropy of the next byte
(Theoretical Framework, per-step loss and its sum over the sequence); the loss
here is the mean over coded positions in nats (a constant rescaling of the
base-256 loss).  Training runs the whole sequence at once: in-time
dependence sits only in the causal conv and the selective scan (Appendix A:
the input-dependent recurrence is evaluated with a scan during training).

Gradients are derived by hand for every stage: LayerNorm, the linear maps,
the depthwise causal conv, SiLU, softplus, the selective scan (reverse
recurrence over time) and softmax-cross-entropy.  ``scan_backward`` can
recompute the scan state chunk by chunk from states saved at chunk
boundaries, so the memory kept between the passes is O(T / T_c).
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

from synth.weights import ModelConfig, param_layout
from .model import Weights, layer_norm, sigmoid, silu, softplus, gelu, LN_EPS


# ----------------------------------------------------------------------------
# pieces
# ----------------------------------------------------------------------------
def ln_fwd(x, w, b):
    mu = x.mean(axis=-1, keepdims=True)
    var = ((x - mu) ** 2).mean(axis=-1, keepdims=True)
    rstd = 1.0 / np.sqrt(var + LN_EPS)
    xhat = (x - mu) * rstd
    return xhat * w + b, (xhat, rstd)


def ln_bwd(dy, cache, w):
    xhat, rstd = cache
    dxhat = dy * w
    dw = (dy * xhat).reshape(-1, w.size).sum(0)
    db = dy.reshape(-1, w.size).sum(0)
    dx = rstd * (dxhat - dxhat.mean(-1, keepdims=True)
                 - xhat * (dxhat * xhat).mean(-1, keepdims=True))
    return dx, dw, db


def dgelu(u):
    """d/du u Phi(u) = Phi(u) + u phi(u), phi the standard normal density."""
    return 0.5 * (1.0 + erf(u / np.sqrt(2.0))) + u * np.exp(-0.5 * u * u) / np.sqrt(2.0 * np.pi)


def dsilu(v):
    s = sigmoid(v)
    return s * (1.0 + v * (1.0 - s))


def conv_fwd(x, w, b):
    """Causal depthwise conv over time. x: [B, T, Di]; w: [Di, K]."""
    Bn, T, Di = x.shape
    K = w.shape[1]
    xp = np.concatenate([np.zeros((Bn, K - 1, Di)), x], axis=1)
    out = np.broadcast_to(b, (Bn, T, Di)).copy()
    for k in range(K):
        out += xp[:, k:k + T, :] * w[:, k]
    return out


def conv_bwd(dout, x, w):
    Bn, T, Di = x.shape
    K = w.shape[1]
    xp = np.concatenate([np.zeros((Bn, K - 1, Di)), x], axis=1)
    dw = np.empty_like(w)
    dxp = np.zeros_like(xp)
    for k in range(K):
        dw[:, k] = (dout * xp[:, k:k + T, :]).sum(axis=(0, 1))
        dxp[:, k:k + T, :] += dout * w[:, k]
    db = dout.sum(axis=(0, 1))
    return dxp[:, K - 1:, :], dw, db


def scan_forward(x, dt, A, Bm, Cm, Dv, save_every=None):
    """Batched selective scan. x, dt: [B, T, Di]; Bm, Cm: [B, T, N]; A: [Di, N].

    Returns y [B, T, Di] and the states saved before steps 0, Tc, 2Tc, ...
    (all states before each step when save_every is None).
    """
    Bn, T, Di = x.shape
    N = A.shape[1]
    h = np.zeros((Bn, Di, N))
    y = np.empty((Bn, T, Di))
    Tc = 1 if save_every is None else save_every
    saved = []
    for t in range(T):
        if t % Tc == 0:
            saved.append(h.copy())
        dA = np.exp(dt[:, t, :, None] * A[None])
        h = dA * h + (dt[:, t] * x[:, t])[:, :, None] * Bm[:, t, None, :]
        y[:, t] = (h * Cm[:, t, None, :]).sum(-1) + Dv * x[:, t]
    return y, saved


def scan_backward(dy, x, dt, A, Bm, Cm, Dv, saved, Tc=1):
    """Reverse-time gradients of the selective scan.

    With a_t = exp(dt_t A), h_t = a_t h_{t-1} + dt_t x_t B_t, y_t = C_t.h_t + D x_t:
      gh_t = C_t gy_t + a_{t+1} gh_{t+1}
      g(dt_t) = sum_n gh_t (A a_t h_{t-1} + x_t B_t),  gA = sum_t gh_t a_t dt_t h_{t-1}
      gx_t = sum_n gh_t dt_t B_t + D gy_t,  gB_t = sum_d gh_t dt_t x_t,
      gC_t = sum_d gy_t h_t,  gD = sum_t gy_t x_t.
    States h_{t-1} are recomputed forward within each chunk of Tc steps from
    the saved chunk-start state.
    """
    Bn, T, Di = x.shape
    N = A.shape[1]
    dx = np.empty_like(x)
    ddt = np.empty_like(dt)
    dB = np.empty_like(Bm)
    dC = np.empty_like(Cm)
    dA = np.zeros_like(A)
    dD = (dy * x).sum(axis=(0, 1))
    gh = np.zeros((Bn, Di, N))
    n_chunks = (T + Tc - 1) // Tc
    for c in reversed(range(n_chunks)):
        t0, t1 = c * Tc, min(T, (c + 1) * Tc)
        # recompute h_{t-1} for t in [t0, t1)
        hprev = []
        h = saved[c].copy()
        for t in range(t0, t1):
            hprev.append(h)
            a = np.exp(dt[:, t, :, None] * A[None])
            h = a * h + (dt[:, t] * x[:, t])[:, :, None] * Bm[:, t, None, :]
        for t in reversed(range(t0, t1)):
            hp = hprev[t - t0]
            a = np.exp(dt[:, t, :, None] * A[None])
            h_t = a * hp + (dt[:, t] * x[:, t])[:, :, None] * Bm[:, t, None, :]
            gh = gh + Cm[:, t, None, :] * dy[:, t, :, None]
            dC[:, t] = (dy[:, t, :, None] * h_t).sum(axis=1)
            ga = gh * hp                                   # d/da_t
            gb = gh                                        # d/d(dt x B)
            ddt[:, t] = (ga * a * A[None]).sum(-1) + (gb * x[:, t, :, None] * Bm[:, t, None, :]).sum(-1)
            dA += (ga * a * dt[:, t, :, None]).sum(0)
            dx[:, t] = (gb * dt[:, t, :, None] * Bm[:, t, None, :]).sum(-1) + Dv * dy[:, t]
            dB[:, t] = (gb * (dt[:, t] * x[:, t])[:, :, None]).sum(axis=1)
            gh = gh * a                                    # carry to step t-1
    return dx, ddt, dA, dB, dC, dD


# ----------------------------------------------------------------------------
# whole model
# ----------------------------------------------------------------------------
def loss_and_grad(cfg: ModelConfig, flat: np.ndarray, seqs, Tc=None, need_grad=True):
    """Mean next-byte cross-entropy (nats) of lanes ``seqs`` [B, T] and its gradient.

    Returns (loss, grad_flat float64 in the layout of ``param_layout``).
    ``flat`` may be float32 or float64 (float64 is used for finite differences).
    """
    W = Weights(cfg, np.asarray(flat))
    seqs = np.asarray(seqs, dtype=np.int64)
    Bn, T = seqs.shape
    yin, tgt = seqs[:, :-1], seqs[:, 1:]
    Tn = T - 1
    D, Di, N, R = cfg.d_model, cfg.d_inner, cfg.d_state, cfg.dt_rank
    Tc = Tn if Tc is None else Tc

    r = W.t["embed"][yin]                                 # [B, Tn, D]
    caches = []
    for l in range(cfg.n_layers):
        lw = W.layer(l)
        a, lnc = ln_fwd(r, lw["norm_w"], lw["norm_b"])
        xz = a @ lw["in_proj_w"].T
        x, z = xz[..., :Di], xz[..., Di:]
        xc = conv_fwd(x, lw["conv_w"], lw["conv_b"])
        xs = silu(xc)
        dbc = xs @ lw["x_proj_w"].T
        delta, Bm, Cm = dbc[..., :R], dbc[..., R:R + N], dbc[..., R + N:]
        dtr = delta @ lw["dt_proj_w"].T + lw["dt_proj_b"]
        dt = softplus(dtr)
        A = -np.exp(lw["A_log"])
        y, saved = scan_forward(xs, dt, A, Bm, Cm, lw["D"], save_every=Tc)
        g = y * silu(z)
        out = g @ lw["out_proj_w"].T
        cache = dict(r_in=r, a=a, lnc=lnc, x=x, z=z, xc=xc, xs=xs, delta=delta,
                     Bm=Bm, Cm=Cm, dtr=dtr, dt=dt, A=A, y=y, g=g, saved=saved)
        r = r + out
        if cfg.ffn_mult:            # r <- LayerNorm(FFN(r)), no residual
            u = r @ lw["ffn_w1"].T + lw["ffn_b1"]
            gu = gelu(u)
            f = gu @ lw["ffn_w2"].T + lw["ffn_b2"]
            cache.update(r_ffn=r, u=u, gu=gu)
            r, cache["lnc_ffn"] = ln_fwd(f, lw["ffn_norm_w"], lw["ffn_norm_b"])
        caches.append(cache)
    rf, lnfc = ln_fwd(r, W.t["norm_f_w"], W.t["norm_f_b"])
    logits = rf @ W.t["head_w"].T + W.t["head_b"]
    m = logits.max(-1, keepdims=True)
    lse = m[..., 0] + np.log(np.exp(logits - m).sum(-1))
    picked = np.take_along_axis(logits, tgt[..., None], -1)[..., 0]
    ntok = Bn * Tn
    loss = float((lse - picked).sum() / ntok)
    if not need_grad:
        return loss, None

    grads = {}
    p = np.exp(logits - lse[..., None])
    dlog = p
    np.put_along_axis(dlog, tgt[..., None], np.take_along_axis(dlog, tgt[..., None], -1) - 1.0, -1)
    dlog /= ntok
    grads["head_w"] = dlog.reshape(-1, 256).T @ rf.reshape(-1, D)
    grads["head_b"] = dlog.reshape(-1, 256).sum(0)
    drf = dlog @ W.t["head_w"]
    dr, grads["norm_f_w"], grads["norm_f_b"] = ln_bwd(drf, lnfc, W.t["norm_f_w"])
    for l in reversed(range(cfg.n_layers)):
        lw, c = W.layer(l), caches[l]
        p_ = f"layers.{l}."
        if cfg.ffn_mult:
            H = cfg.d_ffn
            df, grads[p_ + "ffn_norm_w"], grads[p_ + "ffn_norm_b"] = ln_bwd(dr, c["lnc_ffn"], lw["ffn_norm_w"])
            grads[p_ + "ffn_w2"] = df.reshape(-1, D).T @ c["gu"].reshape(-1, H)
            grads[p_ + "ffn_b2"] = df.reshape(-1, D).sum(0)
            du = (df @ lw["ffn_w2"]) * dgelu(c["u"])
            grads[p_ + "ffn_w1"] = du.reshape(-1, H).T @ c["r_ffn"].reshape(-1, D)
            grads[p_ + "ffn_b1"] = du.reshape(-1, H).sum(0)
            dr = du @ lw["ffn_w1"]
        dout = dr
        grads[p_ + "out_proj_w"] = dout.reshape(-1, D).T @ c["g"].reshape(-1, Di)
        dg = dout @ lw["out_proj_w"]
        dy = dg * silu(c["z"])
        dz = dg * c["y"] * dsilu(c["z"])
        dxs, ddt, dA, dBm, dCm, dD = scan_backward(dy, c["xs"], c["dt"], c["A"], c["Bm"], c["Cm"],
                                                   lw["D"], c["saved"], Tc)
        grads[p_ + "D"] = dD
        grads[p_ + "A_log"] = dA * c["A"]
        ddtr = ddt * np.where(c["dtr"] <= 20.0, sigmoid(np.minimum(c["dtr"], 20.0)), 1.0)
        grads[p_ + "dt_proj_w"] = ddtr.reshape(-1, Di).T @ c["delta"].reshape(-1, R)
        grads[p_ + "dt_proj_b"] = ddtr.reshape(-1, Di).sum(0)
        ddelta = ddtr @ lw["dt_proj_w"]
        ddbc = np.concatenate([ddelta, dBm, dCm], axis=-1)
        grads[p_ + "x_proj_w"] = ddbc.reshape(-1, R + 2 * N).T @ c["xs"].reshape(-1, Di)
        dxs = dxs + ddbc @ lw["x_proj_w"]
        dxc = dxs * dsilu(c["xc"])
        dx, grads[p_ + "conv_w"], grads[p_ + "conv_b"] = conv_bwd(dxc, c["x"], lw["conv_w"])
        dxz = np.concatenate([dx, dz], axis=-1)
        grads[p_ + "in_proj_w"] = dxz.reshape(-1, 2 * Di).T @ c["a"].reshape(-1, D)
        da = dxz @ lw["in_proj_w"]
        dr_in, grads[p_ + "norm_w"], grads[p_ + "norm_b"] = ln_bwd(da, c["lnc"], lw["norm_w"])
        dr = dr + dr_in
    dE = np.zeros((256, D))
    np.add.at(dE, yin.reshape(-1), dr.reshape(-1, D))
    grads["embed"] = dE
    gflat = np.concatenate([grads[name].reshape(-1) for name, _ in param_layout(cfg)])
    return loss, gflat


# ----------------------------------------------------------------------------
# AdamW (decoupled weight decay) and global-norm clipping
# ----------------------------------------------------------------------------
class AdamW:
    def __init__(self, n, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, wd=0.01):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps, self.wd = lr, betas[0], betas[1], eps, wd

    def step(self, theta, g, lr=None):
        lr = self.lr if lr is None else lr
        self.t += 1
        theta = theta * (1.0 - lr * self.wd)
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mhat = self.m / (1 - self.b1 ** self.t)
        vhat = self.v / (1 - self.b2 ** self.t)
        return theta - lr * mhat / (np.sqrt(vhat) + self.eps)


def clip_global_norm(g, max_norm=1.0):
    n = float(np.sqrt((g * g).sum()))
    return g * min(1.0, max_norm / (n + 1e-6)), n
