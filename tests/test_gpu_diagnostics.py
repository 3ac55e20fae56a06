"""GPU predictor diagnostics through the C ABI against the oracle.

The kernel reads the probabilities the coder quantises; the oracle's
diagnostics of those same probabilities (returned by the logits call) must
match bit for bit: confusion counts, rank histogram and reliability bins,
whose confidence sums are exact integers.  Against the FP64 model's own
probabilities only what is robust to rounding is compared: the true-byte
totals exactly, Top-k and ECE within a tolerance.  Launch shapes with several
tiles and a ragged tail, one position per lane, one bin, and bad bin counts
are covered.
"""
import numpy as np
import pytest
import torch

from synth import ModelConfig, init_weights, records_f32_mix, records_structured64
from oracle import diagnostics as dg
from oracle import model as om

pytestmark = pytest.mark.gpu

CFG1 = ModelConfig(d_model=64, n_layers=2)


def boa():
    import paper_2511_11337_amd as b
    return b


@pytest.fixture(scope="module")
def m1():
    print("[gpu] diagnostics model cfg1", flush=True)
    return boa().Model(CFG1, init_weights(CFG1, 4243))


def seqs_of(B, T, seed):
    gens = [records_f32_mix, records_structured64]
    return np.stack([gens[b % 2](T, seed + b) for b in range(B)])


@pytest.mark.parametrize("dtype,tile,n_bins", [("f32", 0, 10), ("f32", 64, 15), ("bf16", 97, 10), ("fp8", 0, 1)])
def test_diagnostics_equal_oracle_on_gpu_probabilities(m1, dtype, tile, n_bins):
    print(f"[gpu] diagnostics {dtype} tile={tile} bins={n_bins}", flush=True)
    seqs = seqs_of(5, 333, 70)
    d = torch.from_numpy(seqs).cuda()
    got = boa().diagnostics(m1, d, dtype=dtype, n_bins=n_bins, tile_t=tile)
    _, pr = boa().logits(m1, d, dtype=dtype, tile_t=tile, want_probs=True)
    p = pr.cpu().numpy().reshape(-1, 256)
    y = seqs[:, 1:].reshape(-1).astype(np.int64)
    ref = dg.all_diagnostics(p, y, n_bins)
    assert np.array_equal(got["confusion"], ref["confusion"])
    assert np.array_equal(got["rank_hist"], ref["rank_hist"])
    assert np.array_equal(got["calibration"], ref["calibration"])
    assert got["positions"] == y.size
    assert abs(got["ece"] - ref["ece"]) < 1e-12 and got["top1"] == ref["top1"]


def test_diagnostics_close_to_fp64_model(m1):
    seqs = seqs_of(4, 400, 90)
    got = boa().diagnostics(m1, torch.from_numpy(seqs).cuda(), dtype="f32")
    p64 = om.softmax(om.stream_logits(om.Weights(CFG1, init_weights(CFG1, 4243)), seqs)).reshape(-1, 256)
    y = seqs[:, 1:].reshape(-1).astype(np.int64)
    ref = dg.all_diagnostics(p64, y, 10)
    print(f"[gpu] top1 {got['top1']:.4f} vs {ref['top1']:.4f}, ece {got['ece']:.5f} vs {ref['ece']:.5f}")
    assert np.array_equal(got["confusion"].sum(axis=1), ref["confusion"].sum(axis=1))   # true-byte totals
    for k in ("top1", "top5", "top10"):
        assert abs(got[k] - ref[k]) <= 0.01
    assert abs(got["ece"] - ref["ece"]) <= 0.01


def test_diagnostics_edge_cases(m1):
    two = torch.from_numpy(seqs_of(3, 2, 5)).cuda()                    # one position per lane
    g = boa().diagnostics(m1, two, n_bins=1)
    assert g["positions"] == 3 and g["calibration"][0, 0] == 3
    one = torch.from_numpy(seqs_of(2, 1, 5)).cuda()                    # no positions
    g = boa().diagnostics(m1, one)
    assert g["positions"] == 0 and g["confusion"].sum() == 0 and g["ece"] == 0.0
    for bad in (0, 1025):
        with pytest.raises(boa().BoaError) as e:
            boa().diagnostics(m1, two, n_bins=bad)
        assert e.value.name == "BOA_E_ARG"
