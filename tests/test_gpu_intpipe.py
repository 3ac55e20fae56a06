"""The integer-only pipeline on the GPU against the integer oracle, bit for bit.

* Integer tables and Q12 logits equal to oracle/intpipe.py's at every position
  (d_model 64 x 2, 128 x 3, 256 x 3 with oracle-trained weights, 512 x 2), sizes
  spanning ragged thread tiles (d_inner 128 .. 1024 over 256 threads).
* Payloads equal to the oracle coder's bytes on the oracle's tables, and the
  CPU oracle decodes the GPU's payloads: a stream encoded on the GPU decodes
  on another device.
* Round trip through the device entry points with empty, one-byte and
  uneven chunks, and at the benchmark's full batch (256 x 64 KiB of 20-byte
  records, d_model 256 x 3), with sampled chunk prefixes' tables against the
  oracle.
* Containers written with dtype int8 carry the integer pipeline's numerics id
  and round-trip, also with the per-chunk order-2 / raw fallback; the CPU
  oracle decodes such a container from its bytes alone.
"""
import os

import numpy as np
import pytest
import torch

from synth import ModelConfig, init_weights, records_f32_mix, records_structured64, raw_normal_f32
from oracle import intpipe as ip
from oracle import coder as oc

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
CFG1 = ModelConfig(64, 2)
CFG2 = ModelConfig(256, 3)


def boa():
    import paper_2511_11337_amd as b
    return b


def trained():
    return np.load(os.path.join(GOLDEN, "cfg2_oracle_trained_f16.npy")).astype(np.float32)


def gpu_tables(cfg, w, seqs):
    q = boa().QModel(boa().Model(cfg, w))
    tb, lg = boa().int_tables(q, torch.from_numpy(np.ascontiguousarray(seqs)).cuda())
    return tb.cpu().numpy().view(np.uint16).astype(np.int64), lg.cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("case", ["d64_seed", "d128_seed", "d256_trained", "d512_seed"])
def test_tables_and_logits_equal_oracle(case):
    if case == "d64_seed":
        cfg, w, T = CFG1, init_weights(CFG1, 4243), 160
    elif case == "d128_seed":
        cfg = ModelConfig(128, 3)
        w, T = init_weights(cfg, 4245), 90
    elif case == "d256_trained":
        cfg, w, T = CFG2, trained(), 120
    else:
        cfg = ModelConfig(512, 2)
        w, T = init_weights(cfg, 4247), 40
    seqs = np.stack([records_f32_mix(T, 21), records_structured64(T, 22), raw_normal_f32(T, 23)])
    print(f"[gpu] integer tables {case}: {seqs.shape}", flush=True)
    tb, lg = gpu_tables(cfg, w, seqs)
    ref_lg, ref_tb = ip.stream_tables(ip.convert(cfg, w), seqs)
    bad = np.argwhere(lg != ref_lg)
    assert bad.size == 0, f"{len(bad)} logits differ, first at {bad[:3].tolist()}"
    assert np.array_equal(tb, ref_tb)


def test_payloads_equal_oracle_and_oracle_decodes_gpu_payloads():
    """GPU-encoded chunks: payload bytes equal the oracle coder's on the
    oracle's integer tables, and the CPU oracle decodes them."""
    w = trained()
    m = boa().Model(CFG2, w)
    q = boa().QModel(m)
    IM = ip.convert(CFG2, w)
    chunks = [records_f32_mix(150, 31), records_structured64(97, 32), raw_normal_f32(64, 33), np.array([7], np.uint8)]
    lens = [c.size for c in chunks]
    data = np.concatenate(chunks)
    print("[gpu] integer encode, oracle decode", flush=True)
    pl, po, ln = boa().int_encode_dev(q, torch.from_numpy(data).cuda(), lens)
    pay, lnh = pl.cpu().numpy(), ln.cpu().numpy().astype(np.int64)
    for i, c in enumerate(chunks):
        gpu_bytes = bytes(pay[po[i]:po[i] + lnh[i]])
        if c.size > 1:
            _, tb = ip.stream_tables(IM, c[None])
            assert gpu_bytes == oc.encode_with_tables(c[1:], tb[0]), i
        else:
            assert gpu_bytes == b""
        assert ip.decode_chunk(IM, int(c[0]), gpu_bytes, c.size) == c.tobytes(), i


def test_round_trip_edges_on_gpu():
    m = boa().Model(CFG1, init_weights(CFG1, 4243))
    q = boa().QModel(m)
    rng = np.random.default_rng(5)
    lens = [0, 1, 2, 3, 300, 0, 1000, 17]
    data = np.concatenate([records_f32_mix(n, 40 + i) if n else np.zeros(0, np.uint8) for i, n in enumerate(lens)]
                          + [rng.integers(0, 256, 5).astype(np.uint8)])
    lens.append(5)
    print(f"[gpu] integer round trip edges {lens}", flush=True)
    d = torch.from_numpy(data).cuda()
    pl, po, ln = boa().int_encode_dev(q, d, lens)
    lnh = ln.cpu().numpy().astype(np.uint32).astype(np.uint64)
    assert np.all(lnh != 0xFFFFFFFF)
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    first = np.array([data[o] if n else 0 for o, n in zip(off, lens)], np.uint8)
    out = boa().int_decode_dev(q, pl, po, lnh, first, lens)
    assert torch.equal(out[:data.size], d)


def test_full_benchmark_batch_round_trip_and_sampled_tables():
    """256 x 64 KiB of 20-byte records, d_model 256 x 3 (oracle-trained): round
    trip exact; the first 256 bytes of two chunks give the oracle's tables."""
    w = trained()
    q = boa().QModel(boa().Model(CFG2, w))
    data = records_f32_mix(256 * 65536, 1338)
    lens = np.full(256, 65536, dtype=np.uint64)
    d = torch.from_numpy(data).cuda()
    print("[gpu] integer full batch encode", flush=True)
    pl, po, ln = boa().int_encode_dev(q, d, lens)
    lnh = ln.cpu().numpy().astype(np.uint32).astype(np.uint64)
    assert np.all(lnh != 0xFFFFFFFF)
    print(f"[gpu] integer full batch: {8 * lnh.sum() / (data.size - 256):.4f} bits/byte; decode", flush=True)
    out = boa().int_decode_dev(q, pl, po, lnh, data[::65536].copy(), lens)
    assert torch.equal(out[:data.size], d)
    seqs = np.stack([data[0:256], data[200 * 65536:200 * 65536 + 256]])
    tb, lg = gpu_tables(CFG2, w, seqs)
    ref_lg, ref_tb = ip.stream_tables(ip.convert(CFG2, w), seqs)
    assert np.array_equal(lg, ref_lg) and np.array_equal(tb, ref_tb)


def test_int8_container_round_trip_with_fallback():
    """compress / decompress with dtype int8: the container carries the
    integer pipeline's numerics id and round-trips, with the per-chunk
    fallback to order-2 and raw storage mixed in."""
    m = boa().Model(CFG2, trained())
    rng = np.random.default_rng(9)
    chunks = [records_f32_mix(3000, 1), np.tile(np.array([0x41, 0x7F], np.uint8), 1500),
              rng.integers(0, 256, 2500).astype(np.uint8), records_structured64(2048, 2), np.array([5], np.uint8),
              np.zeros(0, np.uint8), records_f32_mix(700, 3)]
    lens = [len(c) for c in chunks]
    data = np.concatenate(chunks).tobytes()
    print("[gpu] int8 container", flush=True)
    for fb in (False, True):
        blob = boa().compress(m, data, chunk_lens=lens, dtype="int8", fallback=fb)
        assert boa().container_info(blob)["numerics_id"] == boa().numerics_id("int8")
        assert boa().decompress(m, blob) == data
        if fb:
            _, coder = boa().last_chunk_stats(len(lens))
            assert coder[0] == 0 and coder[1] == 1 and coder[2] == 2


def test_cpu_oracle_decodes_an_int8_container():
    """Encode on the GPU, decode on the CPU from the file alone: the container
    written with dtype int8 is parsed here (64-byte header, 32-byte index
    records, payloads) and every chunk is decoded by the integer oracle; each
    matches its index CRC-32 and the input."""
    import struct
    import zlib
    w = trained()
    m = boa().Model(CFG2, w)
    IM = ip.convert(CFG2, w)
    chunks = [records_f32_mix(120, 51), records_structured64(90, 52), raw_normal_f32(60, 53), np.array([9], np.uint8)]
    data = np.concatenate(chunks)
    print("[gpu] int8 container decoded by the CPU oracle", flush=True)
    blob = boa().compress(m, data.tobytes(), chunk_lens=[c.size for c in chunks], dtype="int8")
    n = struct.unpack_from("<Q", blob, 48)[0]
    assert n == len(chunks)
    base = 64 + 32 * n
    out, coders = b"", []
    for i in range(n):
        length, po, size, crc, first, coder = struct.unpack_from("<QQIIBB", blob, 64 + 32 * i)
        pay = blob[base + po:base + po + size]
        # raw storage (the coded form was not smaller): bytes 2..len verbatim
        chunk = bytes([first]) + pay if coder == 2 else ip.decode_chunk(IM, first, pay, length)
        assert zlib.crc32(chunk) == crc, i
        out += chunk
        coders.append(coder)
    assert coders[0] == 0 and coders[1] == 0          # the record chunks are model-coded
    assert out == data.tobytes()
