"""Integer-only predictor for decoding on any device (test infrastructure only).

The paper (Results & Discussion, portability and limitations) observes that
floating-point matrix products and the float LayerNorm / softmax differ
between devices, so a stream encoded on one machine may not decode on
another.  Its proposed remedy is to quantise the Mamba state-space and affine
maps to INT8 or fixed point with explicit rounding and saturation rules, and
to give LayerNorm and softmax deterministic integer forms.  This module is
that pipeline written out plainly: every quantity after the weight conversion
is an integer, every rounding and clamp is stated, so any implementation that
follows these rules produces the same integer frequency tables bit for bit.

This is test infrastructure: only ``tests/``, the smoke check and the
benchmark's CPU leg may use it (today only tests do).  It shares no code with
the library.

Definitions (all integer; ``>>`` is the arithmetic shift, i.e. floor):
  rs(x, s)    x for s = 0; floor((x + 2^(s-1)) / 2^s) for s > 0 (round half
              up); x * 2^-s for s < 0
  fdiv(a, b)  floor(a / b), b > 0
  rdiv(a, b)  fdiv(2a + b, 2b): a / b rounded half up
  sat23(x)    clamp to [-(2^23 - 1), 2^23 - 1]
Formats: activations Q12 (int, 12 fractional bits) saturated by sat23 after
every operation that makes one; Delta Q20; the scan state h Q16, clamped to
[-(2^31 - 1), 2^31 - 1]; exponentials Q30; LayerNorm variance Q24.

Weight conversion (float64; every step exact or a single rounding):
  projection W [out, in] (in_proj, x_proj, dt_proj, out_proj, head): per row j
    with m_j = max_i |W_ji|, p_j is the largest integer with m_j 2^p_j <= 127,
    clamped to [0, 40] (0 for an all-zero row); w8_ji = clamp(rint(W_ji 2^p_j),
    -127, 127), rint rounding half to even.
  embedding, LayerNorm gains and biases, conv bias, dt bias, D, head bias:
    Q12, rint and sat23.  conv weights: Q14, rint, clamp +-2^20.
  A = -exp(A_log) is made from A_log in integers: a = rint(A_log 2^24) (Q24)
    clamped to [-16, 9] (outside it A is 0, or saturated, in Q12); y =
    rs(a LOG2E, 24), n = y >> 30, g = y - n 2^30; A = -min(rs(P(g), 18 - n),
    2^24) in Q12 (the exponential below, with a positive argument allowed).
Integer exponential (exp2 by a table of 2^(k/16) and a degree-4 Taylor
polynomial of 2^u on [0, 1/16), Horner in Q30):
  P(g), 0 <= g < 2^30:  k = g >> 26, u = g - k 2^26;
    q = C4; q = C3 + rs(q u, 30); q = C2 + rs(q u, 30); q = C1 + rs(q u, 30);
    q = 2^30 + rs(q u, 30);  P = rs(T[k] q, 30)   (~ 2^30 2^(g / 2^30))
  exp of x <= 0 given in Q24:  x = max(x, -64 2^24); y = rs(x LOG2E, 24)
    (Q30); n = y >> 30; g = y - n 2^30; result rs(P(g), -n) in Q30 (0 when
    -n >= 62).
sigmoid(u) (u Q12; e = exp(-|u|) in Q30):  fdiv(2^60, 2^30 + e) for u >= 0,
  fdiv(e 2^30, 2^30 + e) for u < 0 (Q30).   silu(u) = sat23(rs(u sigmoid(u), 30)).
log1p(w) for 0 <= w <= 2^30 (Q30): k = w >> 26 (0..16), c = 2^30 + k 2^26,
  r = fdiv((2^30 + w - c) 2^30, c); h = H5; h = 2^28 - rs(h r, 30);
  h = H3 - rs(h r, 30); h = 2^29 - rs(h r, 30); h = 2^30 - rs(h r, 30);
  log1p = LNC[k] + rs(h r, 30)     (ln(1 + k/16) + the series of ln(1 + r))
softplus(v) (v Q12 -> Delta Q20): w = exp(-|v|) (Q30);
  Delta = clamp(max(v, 0) 2^8 + rs(log1p(w), 10), 0, 2^30).
LayerNorm (r Q12, D values, gain g and bias b Q12):  mu = fdiv(sum r, D);
  d = r - mu; var = fdiv(sum d^2, D) (Q24); s = isqrt(var + 168) (Q12;
  168 = rint(1e-5 2^24)); n_i = sat23(rs(rdiv(d_i 2^12, s) g_i, 12) + b_i).
Dynamic INT8 input of a projection (a Q12 vector): m = max |a_i|;
  e = max(0, bitlen(m) - 7); a8_i = clamp(rs(a_i, e), -127, 127).
Projection: acc_j = sum_i a8_i w8_ji (exact: |acc| < 2^24), out_j =
  sat23(rs(acc_j, p_j - e) + bias_j) in Q12.
One step of a lane (the Mamba step of the FP64 reference, same order):
  r = E[y];  per layer:  a = LN(r); [x; z] = in_proj(a);
  u = sat23(rs(sum_k cw_k win_k, 14) + cb) over the window (x_{t-3}..x_t);
  xs = silu(u);  [delta; B; C] = x_proj(xs);  v = dt_proj(delta) + dt_bias;
  Delta = softplus(v);  dx = rs(Delta xs, 20) (Q12);
  per state n: dA = exp(rs(Delta A_n, 8)) (Q30, the argument Q24);
    h_n = clamp(rs(dA h_n, 30) + rs(dx B_n, 8));
  y = sat23(rs(sum_n C_n h_n, 16) + rs(D xs, 12));
  gate = sat23(rs(y silu(z), 12));  r = sat23(r + out_proj(gate)).
  Then LN_f, head (with its bias): logits l (Q12).
Integer softmax and table (Range coding: probabilities and integer CDF):
  e_a = exp((l_a - max l) 2^12) (Q30; e = 2^30 at the maximum);
  S = sum e_a;  f_a = max(1, fdiv(e_a 2^16, S)); the remainder M - sum f goes
  to the largest f (lowest index on ties), as in the float pipeline.

Supported: d_state 16, d_conv 4, no feed-forward sub-layer (ffn_mult 0).
"""
from __future__ import annotations

import numpy as np

from synth.weights import ModelConfig, unflatten

M = 1 << 16
SAT23 = (1 << 23) - 1
SAT31 = (1 << 31) - 1
EPS_Q24 = 168

# 2^(k/16) in Q30, k = 0..15
T16 = np.array([1073741824, 1121280436, 1170923762, 1222764986, 1276901417, 1333434672, 1392470869,
                1454120821, 1518500250, 1585730000, 1655936265, 1729250827, 1805811301, 1885761398,
                1969251188, 2056437387], dtype=np.int64)
# (ln 2)^k / k! in Q30, k = 1..4
C1, C2, C3, C4 = 744261118, 257941248, 59597083, 10327387
LOG2E = 1549082005                       # log2(e) in Q30
# ln(1 + k/16) in Q30, k = 0..16
LNC = np.array([0, 65095192, 126468572, 184522808, 239598564, 291986604, 341937090, 389666807, 435364845,
                479197128, 521310048, 561833416, 600882877, 638561895, 674963409, 710171213, 744261118],
               dtype=np.int64)
H5, H3 = 214748365, 357913941            # 1/5 and 1/3 in Q30


# ----------------------------------------------------------------------------
# integer primitives
# ----------------------------------------------------------------------------
def rs(x, s):
    """Rounding shift: round(x / 2^s), half up; a left shift for s < 0."""
    x = np.asarray(x, dtype=np.int64)
    s = np.broadcast_to(np.asarray(s, dtype=np.int64), x.shape)
    sp = np.maximum(s, 1)
    right = (x + (np.int64(1) << (sp - 1))) >> sp
    left = x << np.maximum(-s, 0)
    return np.where(s > 0, right, np.where(s < 0, left, x))


def fdiv(a, b):
    return np.floor_divide(np.asarray(a, dtype=np.int64), np.asarray(b, dtype=np.int64))


def rdiv(a, b):
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    return fdiv(2 * a + b, 2 * b)


def sat(x, lim):
    return np.clip(np.asarray(x, dtype=np.int64), -lim, lim)


def isqrt(v):
    """floor(sqrt(v)) for v >= 0, elementwise (Python's exact integer sqrt)."""
    import math
    v = np.asarray(v, dtype=np.int64)
    return np.vectorize(lambda a: math.isqrt(int(a)), otypes=[np.int64])(v) if v.size else v


def exp2_frac(g):
    """P(g) ~ 2^30 * 2^(g / 2^30) for 0 <= g < 2^30."""
    g = np.asarray(g, dtype=np.int64)
    k = g >> 26
    u = g - (k << 26)
    q = np.full_like(g, C4)
    q = C3 + rs(q * u, 30)
    q = C2 + rs(q * u, 30)
    q = C1 + rs(q * u, 30)
    q = (1 << 30) + rs(q * u, 30)
    return rs(T16[k] * q, 30)


def exp_neg_q24(x):
    """exp(x / 2^24) in Q30 for x <= 0."""
    x = np.maximum(np.asarray(x, dtype=np.int64), -(64 << 24))
    y = rs(x * LOG2E, 24)
    n = y >> 30
    g = y - (n << 30)
    p = exp2_frac(g)
    sh = -n
    return np.where(sh >= 62, 0, rs(p, np.minimum(sh, 62)))


def exp_q24_any(x):
    """exp(x / 2^24) as (mantissa Q30 in [2^30, 2^31), exponent n): value
    2^n * mantissa / 2^30.  Used only for A = -exp(A_log) at conversion."""
    x = np.asarray(x, dtype=np.int64)
    y = rs(x * LOG2E, 24)
    n = y >> 30
    g = y - (n << 30)
    return exp2_frac(g), n


def sigmoid_q30(u):
    u = np.asarray(u, dtype=np.int64)
    e = exp_neg_q24(-np.abs(u) << 12)
    pos = fdiv(np.int64(1) << 60, (1 << 30) + e)
    neg = fdiv(e << 30, (1 << 30) + e)
    return np.where(u >= 0, pos, neg)


def silu_q12(u):
    u = np.asarray(u, dtype=np.int64)
    return sat(rs(u * sigmoid_q30(u), 30), SAT23)


def log1p_q30(w):
    """ln(1 + w / 2^30) in Q30 for 0 <= w <= 2^30."""
    w = np.asarray(w, dtype=np.int64)
    k = w >> 26
    c = (1 << 30) + (k << 26)
    r = fdiv(((1 << 30) + w - c) << 30, c)
    h = np.full_like(w, H5)
    h = (1 << 28) - rs(h * r, 30)
    h = H3 - rs(h * r, 30)
    h = (1 << 29) - rs(h * r, 30)
    h = (1 << 30) - rs(h * r, 30)
    return LNC[k] + rs(h * r, 30)


def softplus_q20(v):
    v = np.asarray(v, dtype=np.int64)
    w = exp_neg_q24(-np.abs(v) << 12)
    return np.clip((np.maximum(v, 0) << 8) + rs(log1p_q30(w), 10), 0, 1 << 30)


def bitlen(m):
    m = np.asarray(m, dtype=np.int64)
    out = np.zeros_like(m)
    for b in range(63):
        out = np.where(m >= (np.int64(1) << b), b + 1, out)
    return out


def quant8(a):
    """Dynamic INT8 input of a projection: (a8 [..., n], e [...])."""
    a = np.asarray(a, dtype=np.int64)
    m = np.abs(a).max(axis=-1)
    e = np.maximum(bitlen(m) - 7, 0)
    return np.clip(rs(a, e[..., None]), -127, 127), e


def proj(a, P, bias=None):
    """Projection of Q12 rows a [B, in] by the converted matrix P."""
    a8, e = quant8(a)
    acc = a8 @ P["w8"].T                              # exact integer products and sums
    out = rs(acc, P["p"][None, :] - e[:, None])
    if bias is not None:
        out = out + bias
    return sat(out, SAT23)


def layer_norm(r, g, b):
    r = np.asarray(r, dtype=np.int64)
    D = r.shape[-1]
    mu = fdiv(r.sum(axis=-1, keepdims=True), D)
    d = r - mu
    var = fdiv((d * d).sum(axis=-1, keepdims=True), D)
    s = isqrt(var + EPS_Q24)
    return sat(rs(rdiv(d << 12, s) * g, 12) + b, SAT23)


def tables(logits):
    """Integer softmax and histogram: f [..., 256] with sum M, every f >= 1."""
    l = np.asarray(logits, dtype=np.int64)
    e = exp_neg_q24((l - l.max(axis=-1, keepdims=True)) << 12)
    S = e.sum(axis=-1, keepdims=True)
    f = np.maximum(fdiv(e << 16, S), 1)
    flat = f.reshape(-1, 256)
    for row in flat:
        a = int(np.argmax(row))                       # lowest index among ties
        row[a] += M - int(row.sum())
        assert row[a] >= 1
    return flat.reshape(f.shape)


# ----------------------------------------------------------------------------
# weight conversion
# ----------------------------------------------------------------------------
def conv_proj(W):
    """Per-row power-of-two INT8 quantisation of a projection matrix."""
    W = np.asarray(W, dtype=np.float64)
    m = np.abs(W).max(axis=1)
    fr, E = np.frexp(m)                               # m = fr 2^E, fr in [0.5, 1)
    p = np.where(fr <= 127.0 / 128.0, 7 - E, 6 - E)
    p = np.where(m == 0.0, 0, np.clip(p, 0, 40)).astype(np.int64)
    w8 = np.clip(np.rint(np.ldexp(W, p[:, None])), -127, 127).astype(np.int64)
    return {"w8": w8, "p": p}


def fixq(v, frac, lim):
    return np.clip(np.rint(np.ldexp(np.asarray(v, dtype=np.float64), frac)), -lim, lim).astype(np.int64)


def convert(cfg: ModelConfig, flat: np.ndarray) -> dict:
    """The integer model from the float32 flat weight vector."""
    assert cfg.ffn_mult == 0 and cfg.d_state == 16 and cfg.d_conv == 4
    t = {k: v.astype(np.float64) for k, v in unflatten(cfg, flat).items()}
    R, N = cfg.dt_rank, cfg.d_state
    IM = {"cfg": cfg, "embed": fixq(t["embed"], 12, SAT23), "layers": [],
          "nf_g": fixq(t["norm_f_w"], 12, SAT23), "nf_b": fixq(t["norm_f_b"], 12, SAT23),
          "head": conv_proj(t["head_w"]), "head_b": fixq(t["head_b"], 12, SAT23)}
    for l in range(cfg.n_layers):
        p = f"layers.{l}."
        a24 = np.clip(fixq(t[p + "A_log"], 24, 1 << 40), -(16 << 24), 9 << 24)
        mant, n = exp_q24_any(a24)
        A = -np.minimum(rs(mant, 18 - n), 1 << 24)    # -exp(A_log) in Q12
        IM["layers"].append({
            "ln_g": fixq(t[p + "norm_w"], 12, SAT23), "ln_b": fixq(t[p + "norm_b"], 12, SAT23),
            "in": conv_proj(t[p + "in_proj_w"]),
            "cw": fixq(t[p + "conv_w"], 14, 1 << 20), "cb": fixq(t[p + "conv_b"], 12, SAT23),
            "x": conv_proj(t[p + "x_proj_w"]),
            "dt": conv_proj(t[p + "dt_proj_w"]), "dtb": fixq(t[p + "dt_proj_b"], 12, SAT23),
            "A": A, "D": fixq(t[p + "D"], 12, SAT23),
            "out": conv_proj(t[p + "out_proj_w"]),
            "R": R, "N": N})
    return IM


# ----------------------------------------------------------------------------
# the step and the per-position tables
# ----------------------------------------------------------------------------
class IntState:
    """Per lane and layer: the conv window (last 3 x values, Q12) and h (Q16)."""

    def __init__(self, cfg: ModelConfig, B: int):
        Di, N = cfg.d_inner, cfg.d_state
        self.conv = [np.zeros((B, Di, 3), dtype=np.int64) for _ in range(cfg.n_layers)]
        self.h = [np.zeros((B, Di, N), dtype=np.int64) for _ in range(cfg.n_layers)]


def step(IM: dict, S: IntState, y_prev) -> np.ndarray:
    """Logits (Q12) of the next byte for every lane after bytes y_prev [B]."""
    cfg = IM["cfg"]
    Di = cfg.d_inner
    r = IM["embed"][np.asarray(y_prev, dtype=np.int64)]
    for l, L in enumerate(IM["layers"]):
        a = layer_norm(r, L["ln_g"], L["ln_b"])
        xz = proj(a, L["in"])
        x, z = xz[:, :Di], xz[:, Di:]
        win = np.concatenate([S.conv[l], x[:, :, None]], axis=2)          # x_{t-3} .. x_t
        u = sat(rs((win * L["cw"][None]).sum(axis=2), 14) + L["cb"], SAT23)
        S.conv[l][:] = win[:, :, 1:]
        xs = silu_q12(u)
        dbc = proj(xs, L["x"])
        R, N = L["R"], L["N"]
        delta, Bv, Cv = dbc[:, :R], dbc[:, R:R + N], dbc[:, R + N:]
        v = proj(delta, L["dt"], L["dtb"])
        dl = softplus_q20(v)                                                # [B, Di] Q20
        dx = rs(dl * xs, 20)                                                # Q12
        dA = exp_neg_q24(rs(dl[:, :, None] * L["A"][None], 8))              # [B, Di, N] Q30
        h = S.h[l]
        h[:] = sat(rs(dA * h, 30) + rs(dx[:, :, None] * Bv[:, None, :], 8), SAT31)
        y = sat(rs((Cv[:, None, :] * h).sum(axis=2), 16) + rs(L["D"] * xs, 12), SAT23)
        g = sat(rs(y * silu_q12(z), 12), SAT23)
        r = sat(r + proj(g, L["out"]), SAT23)
    rf = layer_norm(r, IM["nf_g"], IM["nf_b"])
    return proj(rf, IM["head"], IM["head_b"])


def stream_tables(IM: dict, seqs):
    """(logits Q12 [B, T-1, 256], tables [B, T-1, 256]) from the zero state:
    position t predicts seqs[:, t+1]."""
    seqs = np.asarray(seqs)
    B, T = seqs.shape
    S = IntState(IM["cfg"], B)
    lg = np.zeros((B, max(T - 1, 0), 256), dtype=np.int64)
    for t in range(T - 1):
        lg[:, t] = step(IM, S, seqs[:, t])
    return lg, tables(lg)


def decode_chunk(IM: dict, first_byte: int, payload: bytes, length: int) -> bytes:
    """Decode one chunk coded with this pipeline's tables, step by step."""
    from oracle import coder as oc
    if length == 0:
        return b""
    S = IntState(IM["cfg"], 1)
    out = [first_byte]
    dec = oc.Decoder(payload)
    for _ in range(length - 1):
        f = tables(step(IM, S, np.array([out[-1]])))[0]
        out.append(dec.decode(oc.cdf(f)))
    return bytes(out)
