"""Seeded record-stream generators (inputs only; no compressor arithmetic).

Three stream families, each serialised little-endian and row-major so that a
byte sequence is the causal serialisation of a table (paper, Theoretical
Framework: rows are serialised into a causal byte sequence):

* ``records_f32_mix``: 20-byte records of physics-like columns
  (pT ~ Exp(mean 20), eta ~ U[-2.5, 2.5], phi ~ U[-pi, pi] as float32,
  nHits ~ Poisson(12) and a run number that changes every 1000 records as
  int32).
* ``records_structured64``: 64-byte records with slowly varying counters,
  repeated detector IDs and quantised float16 kinematics with Gaussian
  jitter: a highly structured stream.
* ``raw_normal_f32``: a low-structure stream of float32 values ~ N(0, 1).

All generators use NumPy's PCG64 via ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import numpy as np

REC_F32_MIX = np.dtype([("pt", "<f4"), ("eta", "<f4"), ("phi", "<f4"),
                        ("nhits", "<i4"), ("run", "<i4")])


def records_f32_mix(n_bytes: int, seed: int) -> np.ndarray:
    """``n_bytes`` bytes of 20-byte physics records, truncated at the end."""
    rng = np.random.default_rng(seed)
    n_rec = (n_bytes + REC_F32_MIX.itemsize - 1) // REC_F32_MIX.itemsize
    rec = np.empty(n_rec, dtype=REC_F32_MIX)
    rec["pt"] = rng.exponential(20.0, n_rec).astype(np.float32)
    rec["eta"] = rng.uniform(-2.5, 2.5, n_rec).astype(np.float32)
    rec["phi"] = rng.uniform(-np.pi, np.pi, n_rec).astype(np.float32)
    rec["nhits"] = rng.poisson(12.0, n_rec).astype(np.int32)
    run0 = int(rng.integers(100000, 1000000))
    rec["run"] = (run0 + np.arange(n_rec) // 1000).astype(np.int32)
    return np.frombuffer(rec.tobytes(), dtype=np.uint8)[:n_bytes].copy()


REC_S64 = np.dtype([("event", "<u8"), ("run", "<u4"), ("lumi", "<u4"),
                    ("ts", "<u8"), ("det", "<u2", (8,)), ("kin", "<f2", (12,))])
assert REC_S64.itemsize == 64


def records_structured64(n_bytes: int, seed: int, event0: int | None = None) -> np.ndarray:
    """``n_bytes`` bytes of 64-byte structured records (one chunk's worth).

    40 bytes of counters and IDs: event number (+1 per record), run (changes
    every 2**20 events), lumi block (event // 1000), a timestamp advancing by
    25 + U{0..3}, and 8 detector IDs cycling through a fixed 16-entry table
    with a period-8 pattern and swap probability 0.01.  24 bytes of
    kinematics: 4 objects x (pT, eta, phi) as float16, per-chunk base values
    plus N(0, 1% of base) jitter, quantised to a grid (pT 0.25, eta/phi 1/256).
    """
    rng = np.random.default_rng(seed)
    n_rec = (n_bytes + 63) // 64
    if event0 is None:
        event0 = int(rng.integers(0, 1 << 40))
    ev = np.uint64(event0) + np.arange(n_rec, dtype=np.uint64)
    rec = np.zeros(n_rec, dtype=REC_S64)
    rec["event"] = ev
    rec["run"] = (300000 + (ev >> np.uint64(20))).astype(np.uint32)
    rec["lumi"] = (ev // np.uint64(1000)).astype(np.uint32)
    ts0 = int(rng.integers(1 << 40, 1 << 41))
    rec["ts"] = np.uint64(ts0) + np.cumsum(25 + rng.integers(0, 4, n_rec)).astype(np.uint64)
    table = np.array([0x1A01, 0x1A02, 0x1A03, 0x1A04, 0x2B10, 0x2B11, 0x2B12, 0x2B13,
                      0x3C20, 0x3C21, 0x3C22, 0x3C23, 0x4D30, 0x4D31, 0x4D32, 0x4D33],
                     dtype=np.uint16)
    pattern = np.array([0, 3, 5, 6, 9, 10, 12, 15])
    phase = (np.arange(n_rec)[:, None] + np.arange(8)[None, :]) % 8
    idx = pattern[phase]
    swap = rng.random((n_rec, 8)) < 0.01
    idx = np.where(swap, rng.integers(0, 16, (n_rec, 8)), idx)
    rec["det"] = table[idx]
    base_pt = rng.uniform(10.0, 200.0, 4)
    base_eta = rng.uniform(-2.4, 2.4, 4)
    base_phi = rng.uniform(-3.1, 3.1, 4)
    kin = np.empty((n_rec, 12), dtype=np.float64)
    for o in range(4):
        pt = base_pt[o] + rng.normal(0.0, 0.01 * base_pt[o], n_rec)
        eta = base_eta[o] + rng.normal(0.0, 0.01 * abs(base_eta[o]) + 1e-3, n_rec)
        phi = base_phi[o] + rng.normal(0.0, 0.01 * abs(base_phi[o]) + 1e-3, n_rec)
        kin[:, 3 * o + 0] = np.round(pt / 0.25) * 0.25
        kin[:, 3 * o + 1] = np.round(eta * 256.0) / 256.0
        kin[:, 3 * o + 2] = np.round(phi * 256.0) / 256.0
    rec["kin"] = kin.astype(np.float16)
    return np.frombuffer(rec.tobytes(), dtype=np.uint8)[:n_bytes].copy()


def raw_normal_f32(n_bytes: int, seed: int) -> np.ndarray:
    """``n_bytes`` bytes of little-endian float32 ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    n = (n_bytes + 3) // 4
    v = rng.standard_normal(n).astype("<f4")
    return np.frombuffer(v.tobytes(), dtype=np.uint8)[:n_bytes].copy()


def split_fixed(data: np.ndarray, chunk_len: int) -> list[np.ndarray]:
    """Split a byte stream into consecutive chunks of ``chunk_len`` (last may be short)."""
    return [data[i:i + chunk_len] for i in range(0, len(data), chunk_len)]


def chunk_lengths_uniform(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """``n`` chunk lengths uniform on the integers [lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, n).astype(np.int64)


def chunk_lengths_heavy(n: int, seed: int, lo: int = 16384, ratio: float = 64.0,
                        gamma: float = 2.415) -> np.ndarray:
    """``n`` lengths floor(lo * ratio**(u**gamma)), u ~ U[0, 1): 16 KiB .. 1 MiB, mean ~128 KiB."""
    rng = np.random.default_rng(seed)
    u = rng.random(n)
    return np.floor(lo * ratio ** (u ** gamma)).astype(np.int64)


def mixed_chunks(lengths, seed: int) -> list[tuple[int, np.ndarray]]:
    """Chunks whose stream type is (index mod 3): f32-mix records, structured-64
    records, raw N(0,1) float32.  Returns (type, bytes) pairs."""
    out = []
    for i, n in enumerate(lengths):
        kind = i % 3
        s = seed * 1_000_003 + i
        if kind == 0:
            out.append((0, records_f32_mix(int(n), s)))
        elif kind == 1:
            out.append((1, records_structured64(int(n), s)))
        else:
            out.append((2, raw_normal_f32(int(n), s)))
    return out
