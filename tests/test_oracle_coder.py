"""Pins of the oracle's histogram, CDF and range coder (CPU only).

Each test checks the oracle against something other than itself: a closed
form derived from the coder equations (uniform tables code bytes verbatim),
brute force over every short string, the code-length identity of the
Theoretical Framework (coded bytes ~ sum -log_256 Q), and the histogram
invariants the Range coding section requires (strictly positive, sum M).
"""
import numpy as np
import pytest

from oracle import coder
from oracle.coder import M, quantise, cdf, encode_with_tables, decode_with_tables, ideal_bits
from oracle.model import softmax


def rand_table(rng, support=256, peak=None):
    p = np.zeros(256)
    idx = rng.choice(256, support, replace=False)
    p[idx] = rng.dirichlet(np.full(support, 0.5))
    if peak is not None:
        p = (1 - peak) * p
        p[idx[0]] += peak
    return quantise(p)


# ---------------------------------------------------------------- P1 closed form
def test_uniform_tables_code_bytes_verbatim():
    """f = 256 everywhere: L = s 2^24, R = 2^24 after each symbol, so its top
    byte s is emitted and the state returns to (0, 2^32); no flush bytes."""
    rng = np.random.default_rng(0)
    syms = rng.integers(0, 256, 5000)
    f = np.full(256, 256)
    payload = encode_with_tables(syms, [f] * len(syms))
    assert payload == bytes(syms.astype(np.uint8))
    assert decode_with_tables(payload, [f] * len(syms)) == list(syms)


def test_uniform_empty_and_single():
    f = np.full(256, 256)
    assert encode_with_tables([], []) == b""
    assert encode_with_tables([7], [f]) == b"\x07"


# ---------------------------------------------------------------- P2 brute force
@pytest.mark.parametrize("seed", [1, 2])
def test_every_two_symbol_string_round_trips(seed):
    rng = np.random.default_rng(seed)
    f1, f2 = rand_table(rng), rand_table(rng, peak=0.9)
    seen = set()
    for a in range(256):
        for b in range(256):
            pl = encode_with_tables([a, b], [f1, f2])
            assert decode_with_tables(pl, [f1, f2]) == [a, b]
            seen.add((pl, ))
    # distinct strings give distinct (decodable) payloads given the tables
    assert len(seen) == 256 * 256


def test_every_three_symbol_string_small_support():
    rng = np.random.default_rng(3)
    tabs = [rand_table(rng, support=16) for _ in range(3)]
    sup = [np.nonzero(f > 1)[0][:16] for f in tabs]
    # every string over the high-probability supports, plus the floor symbols 0 and 255
    alph = [sorted(set(list(sp) + [0, 255])) for sp in sup]
    for a in alph[0]:
        for b in alph[1]:
            for c in alph[2]:
                pl = encode_with_tables([a, b, c], tabs)
                assert decode_with_tables(pl, tabs) == [a, b, c]


# ---------------------------------------------------------------- P3 length bound
@pytest.mark.parametrize("kind", ["random", "peaked", "uniform", "floor"])
def test_length_within_code_length_identity(kind):
    """payload bytes <= sum(-log2 f(s)/M)/8 * (1 + 1e-3) + 2."""
    rng = np.random.default_rng(11)
    n = 4000
    if kind == "uniform":
        tabs = [np.full(256, 256)] * n
        syms = rng.integers(0, 256, n)
    elif kind == "peaked":
        tabs, syms = [], []
        for _ in range(n):
            s = int(rng.integers(0, 256))
            p = np.zeros(256)
            p[s] = 1.0
            tabs.append(quantise(p))          # f(s) = M - 255
            syms.append(s)
    elif kind == "floor":                     # always code a probability-floor symbol
        tabs, syms = [], []
        for _ in range(n):
            p = np.zeros(256)
            p[0] = 1.0
            tabs.append(quantise(p))
            syms.append(int(rng.integers(1, 256)))
    else:
        tabs = [rand_table(rng, support=int(rng.integers(2, 257))) for _ in range(n)]
        syms = [int(rng.choice(256, p=f / M)) for f in tabs]
    pl = encode_with_tables(syms, tabs)
    ib = ideal_bits(syms, tabs)
    assert len(pl) <= ib / 8 * (1 + 1e-3) + 2, (len(pl), ib / 8)
    assert decode_with_tables(pl, tabs) == list(syms)
    if kind == "peaked":
        # the floor costs log2(M / (M - 255)) ~ 0.0056 bits per symbol
        assert len(pl) <= n * 0.0057 / 8 + 2


# ---------------------------------------------------------------- P4 invariants
def test_state_invariants_every_step():
    rng = np.random.default_rng(5)
    enc = coder.Encoder()
    syms, tabs = [], []
    for _ in range(3000):
        f = rand_table(rng, support=int(rng.integers(1, 257)))
        s = int(rng.integers(0, 256))
        C = cdf(f)
        enc.encode(int(C[s]), int(f[s]))
        assert coder.BOT <= enc.R <= 2 ** 32 and enc.L + enc.R <= 2 ** 32
        syms.append(s)
        tabs.append(f)
    pl = enc.finish()
    dec = coder.Decoder(pl)
    for s, f in zip(syms, tabs):
        C = cdf(f)
        x = dec.target()
        assert C[s] <= x < C[s + 1]
        assert dec.decode(C) == s


def test_flush_uses_at_most_two_bytes():
    rng = np.random.default_rng(9)
    for _ in range(300):
        n = int(rng.integers(1, 30))
        tabs = [rand_table(rng) for _ in range(n)]
        syms = [int(rng.integers(0, 256)) for _ in range(n)]
        enc = coder.Encoder()
        for s, f in zip(syms, tabs):
            C = cdf(f)
            enc.encode(int(C[s]), int(f[s]))
        before = len(enc.out)
        pl = enc.finish()
        assert len(pl) - before <= 2
        assert decode_with_tables(pl, tabs) == syms


# ---------------------------------------------------------------- P5 histogram
def test_quantiser_invariants():
    rng = np.random.default_rng(2)
    for _ in range(500):
        logits = rng.normal(0, rng.uniform(0.1, 30), 256)
        p = softmax(logits)
        f = quantise(p)
        assert f.sum() == M and f.min() >= 1
        g = np.floor(p * M)
        a = int(np.argmax(np.maximum(g, 1)))
        # every bin but the largest is exactly max(1, floor(p M))
        mask = np.arange(256) != a
        assert np.array_equal(f[mask], np.maximum(g, 1)[mask])
        C = cdf(f)
        assert C[0] == 0 and C[256] == M and np.all(np.diff(C) >= 1)


def test_quantiser_special_cases():
    assert np.array_equal(quantise(np.full(256, 1 / 256)), np.full(256, 256))
    p = np.zeros(256)
    p[37] = 1.0
    f = quantise(p)
    assert f[37] == M - 255 and np.all(np.delete(f, 37) == 1)
    # ties resolve to the lowest index
    p = np.zeros(256)
    p[[10, 20]] = 0.5
    f = quantise(p)
    # 254 floor bins of 1 push the sum 254 over M; the lowest-index largest bin absorbs it
    assert f[10] == M // 2 - 254 and f[20] == M // 2 and f.sum() == M


def test_quantiser_float32_inputs_are_exact():
    """floor(p * 2^16) is exact for float32 p: the GPU and the oracle agree on
    the histogram whenever they see the same float32 probabilities."""
    rng = np.random.default_rng(4)
    for _ in range(100):
        p32 = softmax(rng.normal(0, 5, 256)).astype(np.float32)
        f = quantise(p32)
        g = np.floor(p32.astype(np.float64) * 65536.0)
        g2 = np.array([int(np.float32(v) * np.float32(65536.0)) for v in p32])
        assert np.array_equal(g, g2)
        assert f.sum() == M


# ---------------------------------------------------------------- P6 softmax
def test_softmax_normalised_and_shift_invariant():
    rng = np.random.default_rng(6)
    l = rng.normal(0, 10, (50, 256))
    p = softmax(l)
    assert np.allclose(p.sum(-1), 1.0, atol=1e-14, rtol=0)
    assert np.allclose(softmax(l + 123.0), p, atol=1e-13, rtol=0)
    import torch
    assert np.allclose(torch.softmax(torch.from_numpy(l), -1).numpy(), p, atol=1e-14, rtol=0)
