"""The larger workload shapes at sizes a test can run, through the C ABI.

* Structured-record batch (64-byte records of counters, cycling detector IDs
  and quantised half-precision kinematics; chunk lengths uniform in a range):
  2048 uneven chunks in BF16 through the batched encoder and the fused
  decoder, round trip exact; BF16 bits/byte within 0.5 % of the FP64 ideal on
  an oracle subsample of 16 chunks.
* Mixed-stream FP8 workload (d_model 512 x 4 layers; the three stream types in
  turn; heavy-tailed chunk lengths): round trip exact in FP8 and BF16; FP8
  bits/byte loss against FP64 per stream type.

Chunk lengths are the workload's laws scaled down from KiB to bytes.
"""
import numpy as np
import pytest
import torch

from synth import (ModelConfig, init_weights, records_f32_mix, records_structured64, raw_normal_f32,
                   chunk_lengths_uniform, chunk_lengths_heavy, mixed_chunks)
from oracle import model as om

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
