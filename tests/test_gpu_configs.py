"""The larger workload shapes at sizes a test can run, through the C ABI.

* Structured-record batch (64-byte records of counters, cycling detector IDs
  and quantised half-precision kinematics; chunk lengths uniform in a range):
  2048 uneven chunks in BF16 through the batched encoder and the fused
  decoder, round trip exact; BF16 bits/byte within 0.5 % of the FP64 ideal on
  an oracle subsample of 16 chunks.
* Mixed-stream FP8 workload (d_model 512 x 4 layers; the three stream types in
  turn; heavy-tailed chunk lengths): round trip exact in FP8 and BF16, also at
  the workload's full 32768 chunks (lengths scaled down); FP8 bits/byte loss
  against FP64 per stream type.
* The benchmark's own batch (256 x 64 KiB of 20-byte records, d_model 256 x
  3 layers) at full size in the launch shape it times, BF16 and FP8: round
  trip exact, every payload within its ideal-cost bound, and two sampled
  chunks' payloads equal to the oracle coder's bytes.

Apart from the benchmark batch, chunk lengths are the workload's laws scaled
down from KiB to bytes.
"""
import numpy as np
import pytest
import torch

from synth import (ModelConfig, init_weights, records_f32_mix, records_structured64, raw_normal_f32,
                   chunk_lengths_uniform, chunk_lengths_heavy, mixed_chunks)
from oracle import model as om
from oracle import coder as oc

pytestmark = pytest.mark.gpu

CFG2 = ModelConfig(d_model=256, n_layers=3)
CFG5 = ModelConfig(d_model=512, n_layers=4)


def boa():
    import paper_2511_11337_amd as b
    return b


def loss_vs_fp64(m, cfg, W, seqs, dtype):
    """(coded bits, FP64 ideal bits) of the GPU tables on teacher-forced lanes."""
    _, _, tb = boa().logits(m, torch.from_numpy(seqs).cuda(), dtype=dtype, want_probs=True, want_tables=True)
    tb = tb.cpu().numpy().view(np.uint16).astype(np.int64)
    p64 = om.softmax(om.stream_logits(W, seqs))
    tgt = seqs[:, 1:].astype(np.int64)[..., None]
    ideal = -np.log2(np.take_along_axis(p64, tgt, -1)).sum()
    coded = -np.log2(np.take_along_axis(tb, tgt, -1) / 65536.0).sum()
    return coded, ideal


@pytest.fixture(scope="module")
def m2():
    print("[gpu] cfg2-shape model", flush=True)
    return boa().Model(CFG2, init_weights(CFG2, 4246))


@pytest.fixture(scope="module")
def m5():
    print("[gpu] cfg5-shape model", flush=True)
    return boa().Model(CFG5, init_weights(CFG5, 4247))


def test_structured_batch_2048_uneven_chunks_bf16(m2):
    lens = chunk_lengths_uniform(2048, 32, 256, 1337 + 4)
    data = np.concatenate([records_structured64(int(n), 5000 + i) for i, n in enumerate(lens)])
    print(f"[gpu] structured batch: {lens.size} chunks, {data.size} bytes", flush=True)
    blob = boa().compress(m2, data.tobytes(), chunk_lens=lens, dtype="bf16")
    assert boa().decompress(m2, blob) == data.tobytes()
    # the per-step decoder on the same container agrees
    assert boa().decompress(m2, blob, decode_kernel="steps") == data.tobytes()


def test_structured_bf16_loss_on_oracle_subsample(m2):
    seqs = np.stack([records_structured64(1024, 7331 + i) for i in range(16)])
    coded, ideal = loss_vs_fp64(m2, CFG2, om.Weights(CFG2, init_weights(CFG2, 4246)), seqs, "bf16")
    print(f"[gpu] structured bf16: coded {coded / seqs[:, 1:].size:.4f} bits/byte, "
          f"fp64 ideal {ideal / seqs[:, 1:].size:.4f}, loss {100 * (coded / ideal - 1):.3f}%")
    assert coded <= ideal * 1.005


@pytest.mark.parametrize("dtype", ["fp8", "bf16"])
def test_mixed_streams_d512_round_trip(m5, dtype):
    lens = chunk_lengths_heavy(48, 1337 + 5, lo=16, ratio=64.0)
    chunks = mixed_chunks(lens, 1337 + 5)
    data = np.concatenate([c for _, c in chunks])
    print(f"[gpu] mixed streams {dtype}: {len(lens)} chunks, {data.size} bytes", flush=True)
    blob = boa().compress(m5, data.tobytes(), chunk_lens=lens, dtype=dtype)
    assert boa().container_info(blob)["numerics_id"] == boa().numerics_id(dtype)
    assert boa().decompress(m5, blob) == data.tobytes()


def test_mixed_streams_d512_fp8_at_full_chunk_count(m5):
    """The mixed-stream workload's 32768 chunks (its heavy-tailed length law
    divided by 256: 64 B .. 4 KiB) in FP8 through the device entry points in
    the library's own launch shape: every byte comes back and every chunk's
    payload is within 2 bytes + 1e-3 of its ideal cost -sum log2(f/M)."""
    lens = chunk_lengths_heavy(32768, 1337 + 5, lo=64, ratio=64.0).astype(np.uint64)
    chunks = mixed_chunks(lens, 1337 + 5)
    data = np.concatenate([c for _, c in chunks])
    print(f"[gpu] mixed streams at full chunk count: {lens.size} chunks, {data.size} bytes, "
          f"{boa().plan_lanes(lens)} lanes", flush=True)
    d = torch.from_numpy(data).cuda()
    pl, po, ln, ib = boa().encode_dev(m5, d, lens, dtype="fp8", ideal=True)
    lnh = ln.cpu().numpy().astype(np.uint32).astype(np.uint64)
    assert np.all(lnh <= ib.cpu().numpy()[:lens.size] / 8 * (1 + 1e-3) + 2)
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    out = boa().decode_dev(m5, pl, po, lnh, data[off], lens, dtype="fp8", decode_kernel="fused")
    assert torch.equal(out[:data.size], d)


def test_mixed_streams_d512_fp8_loss_per_stream_type(m5):
    W = om.Weights(CFG5, init_weights(CFG5, 4247))
    for name, gen in [("records", records_f32_mix), ("structured64", records_structured64),
                      ("raw_normal_f32", raw_normal_f32)]:
        seqs = np.stack([gen(96, 900 + b) for b in range(2)])
        coded, ideal = loss_vs_fp64(m5, CFG5, W, seqs, "fp8")
        loss = coded / ideal - 1
        print(f"[gpu] d512 fp8 {name}: coded {coded / seqs[:, 1:].size:.4f} bits/byte, "
              f"fp64 ideal {ideal / seqs[:, 1:].size:.4f}, loss {100 * loss:.3f}%")
        assert loss <= 0.05


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_cfg2_full_batch_round_trip_in_bench_shape(dtype):
    """The benchmark's own workload at full size (16 MiB of records as 256 x
    64 KiB chunks, d_model 256 x 3 layers) in the launch shape it times
    (encoder tile 512, fused decoder with one lane per workgroup): every byte
    comes back, every chunk's payload is within 2 bytes + 1e-3 of its own
    ideal cost -sum log2(f/M) (property that holds at any size), and two
    sampled chunks' payloads equal the oracle coder's bytes on the GPU tables
    of those chunks alone."""
    cfg = ModelConfig(d_model=256, n_layers=3)
    m = boa().Model(cfg, init_weights(cfg, 4244))
    n, L = 256, 65536
    data = records_f32_mix(n * L, 1338)
    d = torch.from_numpy(data).cuda()
    lens = np.full(n, L, dtype=np.uint64)
    print(f"[gpu] cfg2 full batch {dtype}", flush=True)
    pl, po, ln, ib = boa().encode_dev(m, d, lens, dtype=dtype, tile_t=512, ideal=True)
    lnh = ln.cpu().numpy().astype(np.uint32).astype(np.uint64)
    ibh = ib.cpu().numpy()[:n]
    assert np.all(lnh <= ibh / 8 * (1 + 1e-3) + 2)
    pay = pl.cpu().numpy()
    for i in (0, 201):
        c = data[i * L:(i + 1) * L]
        tb = boa().logits(m, torch.from_numpy(c[None]).cuda(), dtype=dtype, want_tables=True)[-1]
        tabs = tb[0].cpu().numpy().view(np.uint16).astype(np.int64)
        a, b = int(po[i]), int(po[i]) + int(lnh[i])
        assert bytes(pay[a:b]) == oc.encode_with_tables(c[1:], tabs)
    out = boa().decode_dev(m, pl, po, lnh, data[::L].copy(), lens, dtype=dtype, decode_kernel="fused", fused_lanes=1)
    assert torch.equal(out[:n * L], d)
