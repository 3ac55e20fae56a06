"""Pins of the integer-only pipeline's oracle (oracle/intpipe.py).

Each integer primitive is checked against the mathematics it approximates,
with a bound that follows from its construction; the conversion rules against
their stated properties; the whole predictor against the FP64 predictor (its
logits and the coded bits/byte on a trained model), so a dropped term, a
wrong index or a wrong sign anywhere in the step fails; and the integer
softmax table against the float quantiser's rule.
"""
import math
import os

import numpy as np
import pytest

from synth import ModelConfig, init_weights, records_f32_mix, records_structured64, raw_normal_f32
from oracle import intpipe as ip
from oracle import model as om
from oracle import coder as oc

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
RNG = np.random.default_rng(2511)


def test_rounding_rules_special_cases():
    # round half up: 1.5 -> 2, -1.5 -> -1, -2.5 -> -2; left shift for negative s
    assert ip.rs(3, 1) == 2 and ip.rs(-3, 1) == -1 and ip.rs(-5, 1) == -2 and ip.rs(5, -2) == 20
    assert ip.rs(7, 0) == 7 and ip.rs(-(1 << 40), 40) == -1 and ip.rs((1 << 39) - 1, 40) == 0
    assert ip.fdiv(-7, 2) == -4 and ip.fdiv(7, 2) == 3
    assert ip.rdiv(-5, 2) == -2 and ip.rdiv(5, 2) == 3 and ip.rdiv(-7, 2) == -3


def test_isqrt_is_the_floor_square_root():
    v = np.concatenate([np.arange(0, 2000), RNG.integers(0, 1 << 62, 2000)])
    s = ip.isqrt(v)
    for a, r in zip(v.tolist(), s.tolist()):
        assert r * r <= a < (r + 1) * (r + 1)


def test_constants_are_the_stated_values():
    """Each table entry within half a unit of its real value (Q30)."""
    for k in range(16):
        assert abs(int(ip.T16[k]) - 2 ** (k / 16) * 2 ** 30) <= 0.5
    for c, k in zip((ip.C1, ip.C2, ip.C3, ip.C4), range(1, 5)):
        assert abs(c - math.log(2) ** k / math.factorial(k) * 2 ** 30) <= 0.5
    assert abs(ip.LOG2E - 2 ** 30 / math.log(2)) <= 0.5
    for k in range(17):
        assert abs(int(ip.LNC[k]) - math.log1p(k / 16) * 2 ** 30) <= 0.5
    assert abs(ip.H5 - 2 ** 30 / 5) <= 0.5 and abs(ip.H3 - 2 ** 30 / 3) <= 0.5


def test_exp2_fraction_within_4_units():
    """Degree-4 Taylor on [0, 1/16): truncation (ln2/16)^5/120 ~ 1.3e-9
    relative, plus five roundings: within 4 units of 2^-30."""
    g = np.concatenate([[0, 1, (1 << 26) - 1, 1 << 26, (1 << 30) - 1], RNG.integers(0, 1 << 30, 50000)])
    ref = np.array([2 ** (x / 2 ** 30) * 2 ** 30 for x in g.tolist()])
    assert np.abs(ip.exp2_frac(g) - ref).max() <= 4
    assert ip.exp2_frac(np.array([0]))[0] == 1 << 30


def test_exp_of_nonpositive_argument():
    """exp(x) in Q30 within 2 units absolute for x in [-64, 0]; exactly 2^30 at
    0; monotone non-increasing; below 2^-46 it is 0."""
    x = np.concatenate([[0, -1, -(64 << 24), -(70 << 24)], -RNG.integers(0, 64 << 24, 50000)])
    e = ip.exp_neg_q24(x)
    assert np.abs(e - np.exp(x / 2 ** 24) * 2 ** 30).max() <= 2
    assert ip.exp_neg_q24(np.array([0]))[0] == 1 << 30
    xs = np.sort(x)
    assert np.all(np.diff(ip.exp_neg_q24(xs)) >= 0)
    assert ip.exp_neg_q24(np.array([-(50 << 24)]))[0] == 0


def test_sigmoid_silu_log1p_softplus_bounds():
    u = RNG.integers(-(1 << 23) + 1, 1 << 23, 50000)
    u[:5] = [0, 1, -1, (1 << 23) - 1, -(1 << 23) + 1]
    uf = u / 4096.0
    with np.errstate(over="ignore"):
        sig = 1.0 / (1.0 + np.exp(-uf))
    assert np.abs(ip.sigmoid_q30(u) - sig * 2 ** 30).max() <= 2
    assert np.abs(ip.silu_q12(u) - uf * sig * 4096).max() <= 1
    w = np.concatenate([[0, 1, 1 << 26, (1 << 30) - 1, 1 << 30], RNG.integers(0, (1 << 30) + 1, 50000)])
    assert np.abs(ip.log1p_q30(w) - np.log1p(w / 2 ** 30) * 2 ** 30).max() <= 16
    sp = om.softplus(uf) * 2 ** 20
    assert np.abs(ip.softplus_q20(u) - np.minimum(sp, 2 ** 30)).max() <= 1
    assert np.all(ip.softplus_q20(u) >= 0)


def test_layer_norm_against_float64():
    """Integer LayerNorm of Q12 rows within 2^-10 of the float64 LayerNorm
    (gain 1, bias 0), and with a gain and bias within 2^-9 + 2^-10 |g|."""
    for D in (64, 256, 512):
        r = np.round(RNG.normal(0, 3, (8, D)) * 4096).astype(np.int64)
        r[0] = 5                                            # constant row: variance 0, eps keeps it finite
        g = np.full(D, 4096, dtype=np.int64)
        b = np.zeros(D, dtype=np.int64)
        n = ip.layer_norm(r, g, b) / 4096.0
        ref = om.layer_norm(r / 4096.0, np.ones(D), np.zeros(D))
        assert np.abs(n - ref).max() <= 2 ** -10, D
        gf = RNG.uniform(-2, 2, D)
        bf = RNG.uniform(-1, 1, D)
        n2 = ip.layer_norm(r, ip.fixq(gf, 12, ip.SAT23), ip.fixq(bf, 12, ip.SAT23)) / 4096.0
        ref2 = om.layer_norm(r / 4096.0, gf, bf)
        assert np.abs(n2 - ref2).max() <= 2 ** -9 + 2 ** -10 * 2, D


def test_dynamic_int8_input():
    a = np.round(RNG.normal(0, 1, (64, 300)) * np.exp(RNG.uniform(-3, 12, (64, 1)))).astype(np.int64)
    a[0] = 0
    a[1, :] = 0
    a[1, 3] = -200                                           # 200 needs e = 1
    a8, e = ip.quant8(a)
    assert np.all(np.abs(a8) <= 127)
    assert e[0] == 0 and np.all(a8[0] == 0) and e[1] == 1 and a8[1, 3] == -100
    m = np.abs(a).max(axis=1)
    # e is the smallest shift that brings max |a| below 128
    assert np.all((m >> e) < 128) and np.all((e == 0) | ((m >> np.maximum(e - 1, 0)) >= 128))
    err = np.abs(a8 * (2.0 ** e[:, None]) - a)
    assert np.all(err <= 2.0 ** e[:, None] / 2 + 2.0 ** e[:, None] * (np.abs(a8) == 127))


def test_projection_weight_conversion():
    W = RNG.normal(0, 1, (40, 70)) * np.exp(RNG.uniform(-6, 3, (40, 1)))
    W[0] = 0.0
    W[1, 5] = 127.0                                          # p = 0 exactly
    P = ip.conv_proj(W)
    w8, p = P["w8"], P["p"]
    assert p[0] == 0 and np.all(w8[0] == 0) and p[1] == 0
    assert np.all(np.abs(w8) <= 127)
    rows = np.arange(2, 40)
    mx = np.abs(w8[rows]).max(axis=1)
    assert np.all((mx >= 64) & (mx <= 127))                  # the largest power of two that fits
    assert np.all(np.abs(w8 * 2.0 ** -p[:, None] - W) <= 2.0 ** -(p[:, None] + 1))


def test_A_from_A_log():
    cfg = ModelConfig(64, 2)
    w = init_weights(cfg, 4243)
    IM = ip.convert(cfg, w)
    A_log = om.Weights(cfg, w).layer(1)["A_log"]
    ref = -np.exp(A_log)
    assert np.all(np.abs(IM["layers"][1]["A"] / 4096.0 - ref) <= 1e-7 * np.abs(ref) + 2 ** -13)


def test_tables_against_the_float_quantiser():
    """Sum M, every bin >= 1, equal at the maximum-shifted softmax to the float
    quantiser's bins within one unit (the remainder bin aside)."""
    lg = np.round(RNG.normal(0, 3, (50, 256)) * 4096).astype(np.int64)
    lg[0] = 0                                                 # uniform: 256 each
    lg[1] = -(1 << 23) + 1
    lg[1, 7] = (1 << 23) - 1                                  # one dominant symbol
    f = ip.tables(lg)
    assert np.all(f.sum(axis=1) == ip.M) and np.all(f >= 1)
    assert np.all(f[0] == 256)
    assert f[1, 7] == ip.M - 255 and np.all(np.delete(f[1], 7) == 1)
    for row_l, row_f in zip(lg[2:], f[2:]):
        q = oc.quantise(om.softmax(row_l / 4096.0))
        d = np.abs(q - row_f)
        a = int(np.argmax(row_f))
        assert np.all(np.delete(d, a) <= 1)


def test_step_logits_against_fp64_seed_init():
    """d_model 64 x 2 layers, seed-init weights, three stream types: integer
    logits within 0.1 of the FP64 predictor's at every position."""
    cfg = ModelConfig(64, 2)
    w = init_weights(cfg, 4243)
    seqs = np.stack([records_f32_mix(120, 3), records_structured64(120, 4), raw_normal_f32(120, 5)])
    lg, tb = ip.stream_tables(ip.convert(cfg, w), seqs)
    ref = om.stream_logits(om.Weights(cfg, w), seqs)
    assert np.abs(lg / 4096.0 - ref).max() <= 0.1
    assert np.all(tb.sum(-1) == ip.M)


@pytest.mark.parametrize("gen", [records_f32_mix, records_structured64])
def test_coded_bits_on_trained_model_within_half_percent(gen):
    """The oracle-trained d_model 256 x 3 model (sharp predictions, about 5
    bits/byte): the integer tables code within 0.5 % of the FP64 ideal."""
    cfg = ModelConfig(256, 3)
    w = np.load(os.path.join(GOLDEN, "cfg2_oracle_trained_f16.npy")).astype(np.float32)
    seqs = np.stack([gen(200, 7331 + b) for b in range(2)])
    _, tb = ip.stream_tables(ip.convert(cfg, w), seqs)
    p64 = om.softmax(om.stream_logits(om.Weights(cfg, w), seqs))
    tgt = seqs[:, 1:].astype(np.int64)[..., None]
    ideal = float(-np.log2(np.take_along_axis(p64, tgt, -1)).sum())
    coded = float(-np.log2(np.take_along_axis(tb, tgt, -1) / 65536.0).sum())
    assert ideal / tgt.size < 6.5
    assert coded <= ideal * 1.005


def test_round_trip_through_the_integer_tables():
    cfg = ModelConfig(64, 2)
    IM = ip.convert(cfg, init_weights(cfg, 4243))
    chunk = records_f32_mix(90, 11)
    _, tb = ip.stream_tables(IM, chunk[None])
    payload = oc.encode_with_tables(chunk[1:], tb[0])
    assert ip.decode_chunk(IM, int(chunk[0]), payload, chunk.size) == chunk.tobytes()


def test_planted_mistakes_fail_the_trained_model_gate():
    """The whole-model pin is sensitive: each plausible mistake, planted in a
    copy of the oracle's integer model (the D skip dropped, B and C swapped,
    the conv taps reversed, A halved), pushes the coded bits on the trained
    model past the 0.5 % gate that the clean model meets."""
    import copy
    cfg = ModelConfig(256, 3)
    w = np.load(os.path.join(GOLDEN, "cfg2_oracle_trained_f16.npy")).astype(np.float32)
    seqs = records_f32_mix(120, 7331)[None]
    p64 = om.softmax(om.stream_logits(om.Weights(cfg, w), seqs))
    tgt = seqs[:, 1:].astype(np.int64)[..., None]
    ideal = float(-np.log2(np.take_along_axis(p64, tgt, -1)).sum())

    def loss(IMx):
        _, tb = ip.stream_tables(IMx, seqs)
        return float(-np.log2(np.take_along_axis(tb, tgt, -1) / 65536.0).sum()) / ideal - 1.0

    IM = ip.convert(cfg, w)
    assert loss(IM) <= 0.005
    R, N = cfg.dt_rank, cfg.d_state
    swap = np.r_[0:R, R + N:R + 2 * N, R:R + N]
    mistakes = {
        "D dropped": lambda L: L["D"].fill(0),
        "B and C swapped": lambda L: L.update(x={"w8": L["x"]["w8"][swap], "p": L["x"]["p"][swap]}),
        "conv taps reversed": lambda L: L.update(cw=L["cw"][:, ::-1].copy()),
        "A halved": lambda L: L.update(A=L["A"] // 2),
    }
    for name, plant in mistakes.items():
        bad = copy.deepcopy(IM)
        for L in bad["layers"]:
            plant(L)
        assert loss(bad) > 0.005, name
