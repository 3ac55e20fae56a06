"""Model configuration, canonical parameter layout and seeded initial weights.

The predictor is the byte-level Mamba network of the paper's Models section
(embedding, stacked Mamba blocks with a per-stream cache, linear head).  The
flat weight vector is float32, little-endian, tensors concatenated in the
order of :func:`param_layout`, each tensor row-major with Linear weights
stored as [out_features, in_features].  Both the oracle and the GPU library
read this flat vector; the layout is an interface, not arithmetic.

Initialisation (a seeded input recipe; the paper does not state one):
Linear / conv weights U(+-1/sqrt(fan_in)); embedding N(0, 1);
A_log[d, n] = ln(n + 1); D = 1; dt bias = inverse-softplus of
exp(U[ln 1e-3, ln 1e-1]) floored at 1e-4; dt_proj weight U(+-dt_rank**-0.5);
LayerNorm gamma = 1, beta = 0; head bias 0.  With ffn_mult > 0 each layer also
carries the feed-forward sub-layer of the paper's Algorithm 1 (hidden width
ffn_mult * d_model): its Linear weights and biases U(+-1/sqrt(fan_in)), its
LayerNorm gamma = 1, beta = 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict

import numpy as np


@dataclass(frozen=True)
class ModelConfig:
    d_model: int = 64
    n_layers: int = 2
    d_state: int = 16
    d_conv: int = 4
    expand: int = 2
    ffn_mult: int = 0          # 0: no feed-forward sub-layer; k: hidden width k * d_model

    @property
    def d_ffn(self) -> int:
        return self.ffn_mult * self.d_model

    @property
    def d_inner(self) -> int:
        return self.expand * self.d_model

    @property
    def dt_rank(self) -> int:
        return math.ceil(self.d_model / 16)

    def to_dict(self) -> dict:
        return asdict(self)


def param_layout(cfg: ModelConfig) -> list[tuple[str, tuple[int, ...]]]:
    D, Di, N, K, R = cfg.d_model, cfg.d_inner, cfg.d_state, cfg.d_conv, cfg.dt_rank
    out = [("embed", (256, D))]
    for l in range(cfg.n_layers):
        p = f"layers.{l}."
        out += [
            (p + "norm_w", (D,)), (p + "norm_b", (D,)),
            (p + "in_proj_w", (2 * Di, D)),
            (p + "conv_w", (Di, K)), (p + "conv_b", (Di,)),
            (p + "x_proj_w", (R + 2 * N, Di)),
            (p + "dt_proj_w", (Di, R)), (p + "dt_proj_b", (Di,)),
            (p + "A_log", (Di, N)), (p + "D", (Di,)),
            (p + "out_proj_w", (D, Di)),
        ]
        if cfg.ffn_mult:
            H = cfg.d_ffn
            out += [(p + "ffn_w1", (H, D)), (p + "ffn_b1", (H,)), (p + "ffn_w2", (D, H)), (p + "ffn_b2", (D,)),
                    (p + "ffn_norm_w", (D,)), (p + "ffn_norm_b", (D,))]
    out += [("norm_f_w", (D,)), ("norm_f_b", (D,)), ("head_w", (256, D)), ("head_b", (256,))]
    return out


def param_count(cfg: ModelConfig) -> int:
    return sum(int(np.prod(s)) for _, s in param_layout(cfg))


def init_weights(cfg: ModelConfig, seed: int) -> np.ndarray:
    """Flat float32 weight vector for ``cfg`` drawn from PCG64(seed)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in param_layout(cfg):
        leaf = name.split(".")[-1]
        if leaf == "embed":
            v = rng.standard_normal(shape)
        elif leaf in ("norm_w", "norm_f_w", "ffn_norm_w"):
            v = np.ones(shape)
        elif leaf in ("norm_b", "norm_f_b", "head_b", "ffn_norm_b"):
            v = np.zeros(shape)
        elif leaf in ("ffn_b1", "ffn_b2"):
            b = 1.0 / math.sqrt(cfg.d_model if leaf == "ffn_b1" else cfg.d_ffn)
            v = rng.uniform(-b, b, shape)
        elif leaf == "A_log":
            v = np.log(np.broadcast_to(np.arange(1, shape[1] + 1, dtype=np.float64), shape))
        elif leaf == "D":
            v = np.ones(shape)
        elif leaf == "dt_proj_b":
            dt = np.exp(rng.uniform(math.log(1e-3), math.log(1e-1), shape))
            dt = np.maximum(dt, 1e-4)
            v = dt + np.log(-np.expm1(-dt))       # inverse of softplus
        elif leaf == "dt_proj_w":
            b = cfg.dt_rank ** -0.5
            v = rng.uniform(-b, b, shape)
        elif leaf == "conv_w":
            b = 1.0 / math.sqrt(shape[1])          # depthwise: fan_in = kernel width
            v = rng.uniform(-b, b, shape)
        elif leaf == "conv_b":
            b = 1.0 / math.sqrt(cfg.d_conv)
            v = rng.uniform(-b, b, shape)
        else:                                      # Linear [out, in]
            b = 1.0 / math.sqrt(shape[1])
            v = rng.uniform(-b, b, shape)
        parts.append(np.asarray(v, dtype=np.float64).astype(np.float32).ravel())
    return np.concatenate(parts)


def unflatten(cfg: ModelConfig, flat: np.ndarray) -> dict[str, np.ndarray]:
    """Views of ``flat`` by parameter name (no copies, no arithmetic)."""
    out, off = {}, 0
    for name, shape in param_layout(cfg):
        n = int(np.prod(shape))
        out[name] = flat[off:off + n].reshape(shape)
        off += n
    assert off == flat.size, (off, flat.size)
    return out
