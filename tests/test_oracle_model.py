"""Pins of the oracle's Mamba predictor (CPU only).

The recurrence is checked against its closed form and against an associative
scan (Appendix A: discrete recurrence; parallel scan for training), the LTI
special case against the textbook causal-convolution view of an SSM, the
elementwise pieces against PyTorch's library routines in float64, the step
form against the sequence (training) form, and degenerate weights against the
simpler models they reduce to.
"""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from synth import ModelConfig, init_weights, records_f32_mix
from synth.weights import unflatten
from oracle import model as om
from oracle import coder as oc
from oracle.grad import loss_and_grad, conv_fwd


def rnd_scan_inputs(rng, T=40, Di=6, N=5):
    x = rng.normal(size=(T, Di))
    dt = np.exp(rng.normal(-1.0, 0.7, size=(T, Di)))
    A = -np.exp(rng.normal(0.0, 0.5, size=(Di, N)))
    Bm = rng.normal(size=(T, N))
    Cm = rng.normal(size=(T, N))
    Dv = rng.normal(size=Di)
    return x, dt, A, Bm, Cm, Dv


# ------------------------------------------------------------------ P7 scan forms
def test_scan_matches_closed_form():
    """h_t = sum_{s<=t} exp(A sum_{r=s+1..t} dt_r) dt_s B_s x_s."""
    rng = np.random.default_rng(0)
    x, dt, A, Bm, Cm, Dv = rnd_scan_inputs(rng)
    ys, hs = om.selective_scan(x, dt, A, Bm, Cm, Dv, return_h=True)
    T = x.shape[0]
    cum = np.cumsum(dt, axis=0)
    for t in range(T):
        h = np.zeros_like(hs[0])
        for s in range(t + 1):
            decay = np.exp(A * (cum[t] - cum[s])[:, None])
            h += decay * (dt[s] * x[s])[:, None] * Bm[s][None, :]
        assert np.allclose(h, hs[t], rtol=1e-12, atol=1e-12)
        assert np.allclose(h @ Cm[t] + Dv * x[t], ys[t], rtol=1e-12, atol=1e-12)


def test_scan_matches_associative_tree():
    """(a1, b1) o (a2, b2) = (a1 a2, a2 b1 + b2) combined in a balanced tree."""
    rng = np.random.default_rng(1)
    x, dt, A, Bm, Cm, Dv = rnd_scan_inputs(rng, T=64)
    _, hs = om.selective_scan(x, dt, A, Bm, Cm, Dv, return_h=True)
    a = np.exp(dt[:, :, None] * A[None])
    b = (dt * x)[:, :, None] * Bm[:, None, :]
    # Hillis-Steele inclusive scan
    aa, bb = a.copy(), b.copy()
    step = 1
    while step < len(aa):
        na, nb = aa.copy(), bb.copy()
        na[step:] = aa[:-step] * aa[step:]
        nb[step:] = aa[step:] * bb[:-step] + bb[step:]
        aa, bb = na, nb
        step *= 2
    assert np.allclose(bb, hs, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------ P8 LTI view
@pytest.mark.parametrize("zoh", [False, True])
def test_lti_special_case_is_a_causal_convolution(zoh):
    """Constant dt, B, C: y = kappa * x with kappa_k = sum_n C_n abar_n^k bbar_n + D delta_k
    (S4 convolution view of the discretised SSM).  zoh=True uses the exact
    zero-order-hold input matrix (exp(dt A) - 1) / A * B instead of dt B."""
    rng = np.random.default_rng(2)
    T, Di, N = 50, 4, 6
    x = rng.normal(size=(T, Di))
    dt0 = np.exp(rng.normal(-1, 0.3, Di))
    A = -np.exp(rng.normal(0, 0.5, (Di, N)))
    B0, C0, Dv = rng.normal(size=N), rng.normal(size=N), rng.normal(size=Di)
    abar = np.exp(dt0[:, None] * A)
    bbar = (abar - 1.0) / A * B0[None] if zoh else dt0[:, None] * B0[None]
    # recurrence with the chosen input matrix
    h = np.zeros((Di, N))
    y_rec = np.empty((T, Di))
    for t in range(T):
        h = abar * h + bbar * x[t][:, None]
        y_rec[t] = h @ C0 + Dv * x[t]
    # convolution
    kappa = np.stack([(C0[None] * abar ** k * bbar).sum(-1) for k in range(T)])  # [T, Di]
    kappa[0] += Dv
    y_conv = np.stack([(kappa[:t + 1][::-1] * x[:t + 1]).sum(0) for t in range(T)])
    assert np.allclose(y_rec, y_conv, rtol=1e-11, atol=1e-11)
    if not zoh:   # the oracle's scan uses dt B (first-order input term)
        y_or = om.selective_scan(x, np.broadcast_to(dt0, (T, Di)), A,
                                 np.broadcast_to(B0, (T, N)), np.broadcast_to(C0, (T, N)), Dv)
        assert np.allclose(y_or, y_rec, rtol=1e-12, atol=1e-12)


def test_first_order_input_term_agrees_with_zoh_to_second_order():
    rng = np.random.default_rng(3)
    A = -np.exp(rng.normal(0, 0.5, 16))
    for dt in [1e-2, 1e-3]:
        zoh = (np.exp(dt * A) - 1.0) / A
        assert np.max(np.abs(zoh - dt) / dt) <= np.max(np.abs(dt * A))


# ------------------------------------------------------------------ library routines
def test_pieces_match_torch_float64():
    rng = np.random.default_rng(4)
    x = rng.normal(0, 3, (7, 33))
    w, b = rng.normal(size=33), rng.normal(size=33)
    tx = torch.from_numpy(x)
    assert np.allclose(om.layer_norm(x, w, b), F.layer_norm(tx, (33,), torch.from_numpy(w),
                       torch.from_numpy(b), eps=1e-5).numpy(), rtol=1e-12, atol=1e-12)
    v = rng.normal(0, 15, 1000)
    assert np.allclose(om.softplus(v), F.softplus(torch.from_numpy(v), threshold=20).numpy(),
                       rtol=1e-13, atol=1e-13)
    assert np.allclose(om.silu(v), F.silu(torch.from_numpy(v)).numpy(), rtol=1e-13, atol=1e-13)
    # exact GELU: the library's erf form; special values 0 -> 0, odd part u/2
    assert np.allclose(om.gelu(v), F.gelu(torch.from_numpy(v)).numpy(), rtol=1e-13, atol=1e-15)
    assert om.gelu(np.array(0.0)) == 0.0
    assert np.allclose(om.gelu(v) - om.gelu(-v), v, rtol=1e-13, atol=1e-15)
    # causal depthwise conv == conv1d with left padding K-1
    xs = rng.normal(size=(2, 20, 5))
    cw, cb = rng.normal(size=(5, 4)), rng.normal(size=5)
    ref = F.conv1d(torch.from_numpy(xs).transpose(1, 2), torch.from_numpy(cw)[:, None, :],
                   torch.from_numpy(cb), padding=3, groups=5)[..., :20].transpose(1, 2).numpy()
    assert np.allclose(conv_fwd(xs, cw, cb), ref, rtol=1e-12, atol=1e-12)


def torch_model_logits(cfg, flat, seqs):
    """Sequence forward of the same network with PyTorch float64 library ops."""
    t = {k: torch.from_numpy(v.astype(np.float64)) for k, v in unflatten(cfg, flat).items()}
    Di, R, N = cfg.d_inner, cfg.dt_rank, cfg.d_state
    y = torch.from_numpy(np.asarray(seqs, dtype=np.int64))
    r = F.embedding(y, t["embed"])
    for l in range(cfg.n_layers):
        p = f"layers.{l}."
        a = F.layer_norm(r, (cfg.d_model,), t[p + "norm_w"], t[p + "norm_b"], eps=1e-5)
        xz = F.linear(a, t[p + "in_proj_w"])
        x, z = xz[..., :Di], xz[..., Di:]
        T = x.shape[1]
        xc = F.conv1d(x.transpose(1, 2), t[p + "conv_w"][:, None, :], t[p + "conv_b"],
                      padding=cfg.d_conv - 1, groups=Di)[..., :T].transpose(1, 2)
        xs = F.silu(xc)
        dbc = F.linear(xs, t[p + "x_proj_w"])
        dt = F.softplus(F.linear(dbc[..., :R], t[p + "dt_proj_w"], t[p + "dt_proj_b"]))
        Bm, Cm = dbc[..., R:R + N], dbc[..., R + N:]
        A = -torch.exp(t[p + "A_log"])
        h = torch.zeros(x.shape[0], Di, N, dtype=torch.float64)
        ys = []
        for s in range(T):
            h = torch.exp(dt[:, s, :, None] * A) * h + (dt[:, s] * xs[:, s])[..., None] * Bm[:, s, None, :]
            ys.append(torch.einsum("bdn,bn->bd", h, Cm[:, s]) + t[p + "D"] * xs[:, s])
        yy = torch.stack(ys, 1)
        r = r + F.linear(yy * F.silu(z), t[p + "out_proj_w"])
        if cfg.ffn_mult:            # Algorithm 1: x <- LayerNorm(FFN(x)), exact GELU
            f = F.linear(F.gelu(F.linear(r, t[p + "ffn_w1"], t[p + "ffn_b1"])), t[p + "ffn_w2"], t[p + "ffn_b2"])
            r = F.layer_norm(f, (cfg.d_model,), t[p + "ffn_norm_w"], t[p + "ffn_norm_b"], eps=1e-5)
    rf = F.layer_norm(r, (cfg.d_model,), t["norm_f_w"], t["norm_f_b"], eps=1e-5)
    return F.linear(rf, t["head_w"], t["head_b"]).numpy()


# ------------------------------------------------------------------ step vs sequence
@pytest.mark.parametrize("ffn_mult", [0, 4])
def test_step_recurrence_equals_sequence_forms(ffn_mult):
    cfg = ModelConfig(d_model=32, n_layers=2, ffn_mult=ffn_mult)
    flat = init_weights(cfg, 7)
    seqs = np.stack([records_f32_mix(48, 100), records_f32_mix(48, 101)])
    W = om.Weights(cfg, flat)
    lg_step = om.stream_logits(W, seqs)                     # [B, T-1, 256]
    lg_torch = torch_model_logits(cfg, flat, seqs[:, :-1])
    assert np.allclose(lg_step, lg_torch, rtol=1e-11, atol=1e-11)
    # the training-form loss over the same positions
    p = om.softmax(lg_step)
    tgt = seqs[:, 1:].astype(np.int64)
    ce = -np.log(np.take_along_axis(p, tgt[..., None], -1)).mean()
    loss, _ = loss_and_grad(cfg, flat, seqs, need_grad=False)
    assert abs(loss - ce) <= 1e-12 * abs(ce)


# ------------------------------------------------------------------ P9 degenerate
def test_zero_out_proj_gives_bigram_model():
    """out_proj = 0: every block adds 0, so logits = head(LN_f(E[y])) + b."""
    cfg = ModelConfig(d_model=16, n_layers=2)
    flat = init_weights(cfg, 8)
    named = unflatten(cfg, flat)
    for l in range(cfg.n_layers):
        named[f"layers.{l}.out_proj_w"][:] = 0.0
    rng = np.random.default_rng(0)
    named["head_b"][:] = rng.normal(size=256).astype(np.float32)
    seq = np.array([records_f32_mix(30, 5)])
    lg = om.stream_logits(om.Weights(cfg, flat), seq)[0]
    E = torch.from_numpy(named["embed"].astype(np.float64))
    rf = F.layer_norm(E[torch.from_numpy(seq[0, :-1].astype(np.int64))], (16,),
                      torch.from_numpy(named["norm_f_w"].astype(np.float64)),
                      torch.from_numpy(named["norm_f_b"].astype(np.float64)), eps=1e-5)
    ref = F.linear(rf, torch.from_numpy(named["head_w"].astype(np.float64)),
                   torch.from_numpy(named["head_b"].astype(np.float64))).numpy()
    assert np.allclose(lg, ref, rtol=1e-12, atol=1e-12)


def test_vanishing_dt_keeps_state_zero():
    """softplus(very negative) ~ 0: Delta -> 0, h stays 0 and y = D x."""
    cfg = ModelConfig(d_model=16, n_layers=1)
    flat = init_weights(cfg, 9)
    named = unflatten(cfg, flat)
    named["layers.0.dt_proj_b"][:] = -80.0
    named["layers.0.dt_proj_w"][:] = 0.0
    W = om.Weights(cfg, flat)
    S = om.StreamState(cfg, 1)
    for y in records_f32_mix(20, 3):
        om.step(W, S, [y])
    assert np.max(np.abs(S.h[0])) < 1e-30


def test_large_decay_makes_model_memoryless_beyond_conv_window():
    """A_log large => exp(Delta A) = 0: the state forgets everything but the
    current input, so a byte influences logits for at most n_l (K-1) + 1 steps."""
    cfg = ModelConfig(d_model=16, n_layers=2)
    flat = init_weights(cfg, 10)
    named = unflatten(cfg, flat)
    for l in range(cfg.n_layers):
        named[f"layers.{l}.A_log"][:] = 30.0
        named[f"layers.{l}.dt_proj_b"][:] = 5.0
    W = om.Weights(cfg, flat)
    s1 = records_f32_mix(40, 11)
    s2 = s1.copy()
    s2[5] ^= 0x5A
    l1 = om.stream_logits(W, s1[None])[0]
    l2 = om.stream_logits(W, s2[None])[0]
    reach = cfg.n_layers * (cfg.d_conv - 1) + 1
    assert not np.allclose(l1[5], l2[5])
    assert np.array_equal(l1[5 + reach:], l2[5 + reach:])
    assert np.array_equal(l1[:5], l2[:5])


# ------------------------------------------------------------------ round trip
def test_model_driven_round_trip_cfg1_model():
    cfg = ModelConfig(d_model=64, n_layers=2)
    W = om.Weights(cfg, init_weights(cfg, 4243))
    chunk = records_f32_mix(300, 1338)

    def mk():
        S = om.StreamState(cfg, 1)
        return lambda y: om.softmax(om.step(W, S, [y])[0])

    first, payload, ib = oc.compress_chunk(mk(), chunk)
    assert first == chunk[0]
    assert len(payload) <= ib / 8 * (1 + 1e-3) + 2
    assert oc.decompress_chunk(mk(), first, payload, len(chunk)) == bytes(chunk)
