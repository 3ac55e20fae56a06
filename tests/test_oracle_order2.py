"""Pins of the oracle's adaptive order-2 context-count model (CPU only)."""
import numpy as np

from synth import records_f32_mix, raw_normal_f32
from oracle import order2
from oracle.coder import M


def test_empty_context_is_uniform():
    assert np.array_equal(order2.table(np.zeros(256, dtype=np.int64)), np.full(256, 256))


def test_kt_estimate_closed_form():
    """One observation of byte 7: f(7) = floor(3M/258), the others floor(M/258),
    the remainder to byte 7."""
    n = np.zeros(256, dtype=np.int64)
    n[7] = 1
    f = order2.table(n)
    other = M // 258
    assert np.all(np.delete(f, 7) == other)
    assert f[7] == M - 255 * other
    assert f.sum() == M and f.min() >= 1


def test_round_trip_and_cost():
    for data in (records_f32_mix(3000, 1), raw_normal_f32(2000, 2), np.zeros(500, np.uint8),
                 np.arange(256, dtype=np.uint8)):
        first, pl, ib = order2.compress_chunk(data)
        assert order2.decompress_chunk(first, pl, len(data)) == bytes(data)
        assert len(pl) <= ib / 8 * (1 + 1e-3) + 2


def test_constant_stream_cost_is_logarithmic():
    """KT on a constant stream: the n-th repeat costs -log2((2n+1)/(2n+256)),
    about 255 / (2 n ln 2) bits, so 20000 repeats cost ~ 184 ln(20000) bits
    plus the floor cost log2(M / (M - 255)) per byte: well under 200 bytes."""
    data = np.full(20000, 0x41, np.uint8)
    _, pl, ib = order2.compress_chunk(data)
    n = np.arange(1, 20000)
    kt = -np.log2(np.minimum((2 * (n - 1) + 1) / (2 * (n - 1) + 256), (M - 255) / M)).sum()
    assert ib <= kt + 256 and len(pl) < 200


def test_halving_keeps_counts_positive():
    m = order2.Order2()
    for _ in range(order2.HALVE_AT + 5):
        m.update(1, 2, 3)
    r = m.row(1, 2)
    assert 0 < r.sum() < order2.HALVE_AT and r[3] == r.sum()
