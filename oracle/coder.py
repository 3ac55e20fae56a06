"""Integer histogram, CDF and range coder in Python integers (test infrastructure only).

Follows the paper's Range coding section: probabilities are quantised to a
strictly positive histogram f summing to M = 2**B, C(a) = sum_{x<a} f(x); the
encoder keeps (L, R) on a w-bit ring, updates
L <- L + floor(R C(s) / M), R <- floor(R (C(s+1) - C(s)) / M), and emits the
top byte while it is fixed (E = L + R - 1 has the same top byte as L), shifting
both L and R left by 8; the decoder forms x = floor(((X - L + 1) M - 1) / R),
finds s with C(s) <= x < C(s+1), applies the same update and shifts the next
payload byte into its code value X on every emitted byte.

Readings where the paper is silent (each listed in the design notes):
* w = 32, B = 16; L is kept mod 2**32 but R is never reduced mod 2**w
  (R in [1, 2**32]), otherwise R = 2**24 would wrap to 0 on a shift.
* start state L = 0, R = 2**32; decoder code value X = first four payload
  bytes, big-endian; bytes past the end of the payload read as 0.
* straddle ("underflow") case: when the top bytes differ but R < 2**16, R is
  cut to the distance from L to the next multiple of 2**16 (carry-less
  coder); the following iterations then emit bytes.
* flush: the smallest k in {0, 1, 2} such that V = ceil(L / 2**(32-8k)) *
  2**(32-8k) <= L + R - 1; the top k bytes of V are emitted.
* histogram rule: f(a) = max(1, floor(p(a) M)); the difference M - sum f is
  added to the largest f (lowest index on ties).
"""
from __future__ import annotations

import numpy as np

W_BITS = 32
B_BITS = 16
M = 1 << B_BITS
TOP = 1 << (W_BITS - 8)
BOT = 1 << 16
MASK = (1 << W_BITS) - 1


# ----------------------------------------------------------------------------
# histogram and CDF
# ----------------------------------------------------------------------------
def quantise(p) -> np.ndarray:
    """Strictly positive integer histogram f with sum M from probabilities p [256].

    floor(p * M) is exact for any binary float p (M is a power of two), so the
    result depends only on the float values passed in.
    """
    p = np.asarray(p)
    assert p.shape == (256,)
    g = np.floor(p.astype(np.float64) * M).astype(np.int64)
    f = np.maximum(g, 1)
    d = M - int(f.sum())
    a = int(np.argmax(f))              # lowest index among ties
    f[a] += d
    assert f[a] >= 1, "remainder rule would empty the largest bin"
    return f


def cdf(f) -> np.ndarray:
    """C(0) = 0, C(a+1) = C(a) + f(a); C(256) = M."""
    c = np.zeros(257, dtype=np.int64)
    c[1:] = np.cumsum(f)
    assert c[256] == M
    return c


# ----------------------------------------------------------------------------
# encoder
# ----------------------------------------------------------------------------
class Encoder:
    def __init__(self):
        self.L = 0
        self.R = 1 << W_BITS
        self.out = bytearray()

    def encode(self, c_lo: int, f: int):
        """Code one symbol whose CDF interval is [c_lo, c_lo + f) of M."""
        L, R = self.L, self.R
        assert 1 <= f and c_lo + f <= M
        L = L + (R * c_lo) // M
        R = (R * f) // M
        assert R >= 1 and L + R <= (1 << W_BITS)
        while True:
            if L // TOP == (L + R - 1) // TOP:
                self.out.append(L // TOP)
                L = (L << 8) & MASK
                R = R << 8
            elif R < BOT:
                R = BOT - (L % BOT)
            else:
                break
        assert BOT <= R <= (1 << W_BITS) and L + R <= (1 << W_BITS)
        self.L, self.R = L, R

    def finish(self) -> bytes:
        L, R = self.L, self.R
        for k in range(3):
            s = W_BITS - 8 * k
            V = -(-L // (1 << s)) * (1 << s)
            if V <= L + R - 1:
                for i in range(k):
                    self.out.append((V >> (W_BITS - 8 - 8 * i)) & 0xFF)
                return bytes(self.out)
        raise AssertionError("flush needs more than two bytes")


class Decoder:
    def __init__(self, payload: bytes):
        self.buf = bytes(payload)
        self.pos = 0
        self.L = 0
        self.R = 1 << W_BITS
        self.X = 0
        for _ in range(4):
            self.X = (self.X << 8) | self._next()

    def _next(self) -> int:
        b = self.buf[self.pos] if self.pos < len(self.buf) else 0
        self.pos += 1
        return b

    def target(self) -> int:
        """x = floor(((X - L + 1) M - 1) / R) in [0, M)."""
        x = ((self.X - self.L + 1) * M - 1) // self.R
        assert 0 <= x < M
        return x

    def decode(self, C) -> int:
        x = self.target()
        s = int(np.searchsorted(C, x, side="right")) - 1     # C(s) <= x < C(s+1)
        assert C[s] <= x < C[s + 1]
        L, R = self.L, self.R
        L = L + (R * int(C[s])) // M
        R = (R * int(C[s + 1] - C[s])) // M
        while True:
            if L // TOP == (L + R - 1) // TOP:
                L = (L << 8) & MASK
                R = R << 8
                self.X = ((self.X << 8) & MASK) | self._next()
            elif R < BOT:
                R = BOT - (L % BOT)
            else:
                break
        self.L, self.R = L, R
        return s


# ----------------------------------------------------------------------------
# whole-stream helpers on explicit tables
# ----------------------------------------------------------------------------
def encode_with_tables(symbols, tables) -> bytes:
    """Encode symbols[i] with integer histogram tables[i] (each [256], sum M)."""
    enc = Encoder()
    for s, f in zip(symbols, tables):
        C = cdf(f)
        enc.encode(int(C[s]), int(f[s]))
    return enc.finish()


def decode_with_tables(payload: bytes, tables) -> list[int]:
    dec = Decoder(payload)
    return [dec.decode(cdf(f)) for f in tables]


def ideal_bits(symbols, tables) -> float:
    """sum -log2(f(s)/M) over the coded symbols (the tables actually coded)."""
    tot = 0.0
    for s, f in zip(symbols, tables):
        tot += -np.log2(f[s] / M)
    return tot


# ----------------------------------------------------------------------------
# model-driven compression of one chunk (the paper's per-stream procedure)
# ----------------------------------------------------------------------------
def compress_chunk(step_fn, chunk) -> tuple[int, bytes, float]:
    """Compress one chunk: the first byte is stored raw, bytes 2..l are coded.

    step_fn(y_prev) -> probabilities [256] of the next byte (stateful).
    Returns (first_byte, payload, ideal_bits).
    """
    chunk = bytes(chunk)
    if len(chunk) == 0:
        return -1, b"", 0.0
    enc = Encoder()
    ib = 0.0
    for t in range(len(chunk) - 1):
        f = quantise(step_fn(chunk[t]))
        C = cdf(f)
        s = chunk[t + 1]
        ib += -np.log2(f[s] / M)
        enc.encode(int(C[s]), int(f[s]))
    return chunk[0], enc.finish(), ib


def decompress_chunk(step_fn, first_byte: int, payload: bytes, length: int) -> bytes:
    if length == 0:
        return b""
    dec = Decoder(payload)
    out = bytearray([first_byte])
    for _ in range(length - 1):
        f = quantise(step_fn(out[-1]))
        out.append(dec.decode(cdf(f)))
    return bytes(out)
