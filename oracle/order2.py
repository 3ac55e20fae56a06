"""Adaptive order-2 context-count model (test infrastructure only).

Not in the paper: a classical statistical predictor (the paper's Theoretical
Framework names PPM-style context models as the traditional alternative) that
drives the same integer range coder, used as a per-chunk fallback and as a
bits/byte yardstick for the learned predictor.

Rule (the reading taken here): the context of byte y_t is (y_{t-2}, y_{t-1})
with bytes before the chunk start taken as 0.  Counts n[ctx, a] start at 0.
The histogram is the Krichevsky-Trofimov estimate
    f(a) = max(1, floor(M (2 n(a) + 1) / (2 T + 256))),   T = sum_a n(a),
followed by the same remainder rule as the neural histogram (M - sum f added
to the largest f, lowest index on ties).  T = 0 gives f = 256 everywhere.
After coding s, n[ctx, s] += 1; when T reaches 2**16 every count of that
context becomes ceil(n / 2).
"""
from __future__ import annotations

import numpy as np

from .coder import M, Encoder, Decoder, cdf

HALVE_AT = 1 << 16


def table(counts_row) -> np.ndarray:
    n = np.asarray(counts_row, dtype=np.int64)
    T = int(n.sum())
    f = np.maximum((M * (2 * n + 1)) // (2 * T + 256), 1)
    d = M - int(f.sum())
    a = int(np.argmax(f))
    f[a] += d
    assert f[a] >= 1
    return f


class Order2:
    def __init__(self):
        self.counts = {}

    def row(self, c2, c1):
        key = (c2, c1)
        if key not in self.counts:
            self.counts[key] = np.zeros(256, dtype=np.int64)
        return self.counts[key]

    def update(self, c2, c1, s):
        r = self.row(c2, c1)
        r[s] += 1
        if r.sum() >= HALVE_AT:
            r[:] = (r + 1) // 2


def compress_chunk(chunk) -> tuple[int, bytes, float]:
    chunk = bytes(chunk)
    if not chunk:
        return -1, b"", 0.0
    m = Order2()
    enc = Encoder()
    ib = 0.0
    for t in range(1, len(chunk)):
        c2 = chunk[t - 2] if t >= 2 else 0
        c1 = chunk[t - 1]
        f = table(m.row(c2, c1))
        C = cdf(f)
        s = chunk[t]
        ib += -np.log2(f[s] / M)
        enc.encode(int(C[s]), int(f[s]))
        m.update(c2, c1, s)
    return chunk[0], enc.finish(), ib


def decompress_chunk(first_byte, payload, length) -> bytes:
    if length == 0:
        return b""
    m = Order2()
    dec = Decoder(payload)
    out = bytearray([first_byte])
    for t in range(1, length):
        c2 = out[t - 2] if t >= 2 else 0
        c1 = out[t - 1]
        s = dec.decode(cdf(table(m.row(c2, c1))))
        out.append(s)
        m.update(c2, c1, s)
    return bytes(out)


def tables_for(chunk) -> list[np.ndarray]:
    """The integer histogram used for each coded byte of ``chunk`` (for parity)."""
    chunk = bytes(chunk)
    m = Order2()
    out = []
    for t in range(1, len(chunk)):
        c2 = chunk[t - 2] if t >= 2 else 0
        c1 = chunk[t - 1]
        out.append(table(m.row(c2, c1)))
        m.update(c2, c1, chunk[t])
    return out
