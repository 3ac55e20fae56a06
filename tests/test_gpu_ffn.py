"""The paper's block variant on the GPU, through the C ABI: each Mamba block
followed by Algorithm 1's sub-layer r <- LayerNorm(FFN(r)), FFN(r) =
W2 GELU(W1 r + b1) + b2 (hidden width 4 d_model), against the FP64 oracle.

* FP32 logits within 1e-3 of the oracle over several time tiles with a
  ragged tail, and in the decoder's one-row-per-lane shape, for a small model
  and for the paper's own model (d_model 256, one layer, about 1.10 M
  parameters);
* BF16 and FP8 projections: integer tables independent of the launch shape,
  FP8 logits following the FP8-mode oracle;
* compress -> decompress is the identity in every dtype (the per-step
  decoder; the fused decoder declines models with the sub-layer).
"""
import numpy as np
import pytest
import torch

from synth import ModelConfig, init_weights, records_f32_mix, records_structured64, raw_normal_f32, param_count
from oracle import model as om

pytestmark = pytest.mark.gpu

SMALL = ModelConfig(d_model=64, n_layers=2, ffn_mult=4)
PAPER = ModelConfig(d_model=256, n_layers=1, ffn_mult=4)


def boa():
    import paper_2511_11337_amd as b
    return b


@pytest.fixture(scope="module")
def models():
    print("[gpu] ffn models", flush=True)
    return {c: (boa().Model(c, init_weights(c, s)), init_weights(c, s)) for c, s in ((SMALL, 61), (PAPER, 62))}


def test_paper_model_size():
    n = param_count(PAPER)
    assert boa().Config.of(PAPER).n_params == n
    assert 1.09e6 < n < 1.11e6            # "about 4.5 MB" of float32 weights
    print(f"[gpu] paper model: {n} parameters, {4 * n / 2 ** 20:.2f} MiB")


@pytest.mark.parametrize("which", ["small", "paper"])
@pytest.mark.parametrize("tile", [1, 64, 300])
def test_ffn_logits_fp32_match_oracle(models, which, tile):
    cfg = SMALL if which == "small" else PAPER
    m, w = models[cfg]
    print(f"[gpu] ffn logits {which} tile {tile}", flush=True)
    seqs = np.stack([records_f32_mix(301, 71), records_structured64(301, 72), raw_normal_f32(301, 73)])
    lg = boa().logits(m, torch.from_numpy(seqs).cuda(), dtype="f32", tile_t=tile).cpu().numpy()
    ref = om.stream_logits(om.Weights(cfg, w), seqs)
    err = np.abs(lg - ref)
    print(f"[gpu] {which} max |dlogit| {err.max():.3e}")
    assert err.max() <= 1e-3


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_ffn_tables_do_not_depend_on_launch_shape(models, dtype):
    m, _ = models[PAPER]
    seqs = np.stack([records_f32_mix(131, 80 + b) for b in range(20)])
    d = torch.from_numpy(seqs).cuda()
    _, _, a = boa().logits(m, d, dtype=dtype, want_probs=True, want_tables=True, tile_t=1)
    _, _, b = boa().logits(m, d, dtype=dtype, want_probs=True, want_tables=True, tile_t=50)
    _, _, c = boa().logits(m, d, dtype=dtype, want_probs=True, want_tables=True, tile_t=130)   # 2600 rows
    assert torch.equal(a, b)
    assert torch.equal(a, c)


def test_ffn_fp8_logits_follow_fp8_oracle(models):
    m, w = models[PAPER]
    seqs = np.stack([records_f32_mix(160, 31), raw_normal_f32(160, 32)])
    lg = boa().logits(m, torch.from_numpy(seqs).cuda(), dtype="fp8").cpu().numpy()
    ref = om.stream_logits(om.Weights(PAPER, w), seqs, proj="fp8")
    err = np.abs(lg - ref)
    print(f"[gpu] ffn fp8 |dlogit| max {err.max():.3e} mean {err.mean():.3e}")
    assert err.mean() <= 2e-3
    assert err.max() <= 0.1


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_ffn_round_trip(models, dtype):
    m, _ = models[PAPER]
    print(f"[gpu] ffn round trip {dtype}", flush=True)
    lens = [1500, 1, 0, 2, 777, 2048]
    data = np.concatenate([records_f32_mix(lens[0], 1), records_f32_mix(1, 2), np.zeros(0, np.uint8),
                           records_structured64(2, 3), raw_normal_f32(lens[4], 4),
                           records_structured64(lens[5], 5)]).tobytes()
    blob = boa().compress(m, data, chunk_lens=lens, dtype=dtype, max_lanes=4)
    assert boa().decompress(m, blob) == data
    with pytest.raises(boa().BoaError) as e:
        boa().decompress(m, blob, decode_kernel="fused")
    assert e.value.name == "BOA_E_UNSUPPORTED"
