"""GPU checks of the fused persistent decoder through the C ABI.

The encoder (time-tiled kernels) writes the payloads; the fused decoder must
rebuild every byte exactly -- which it can only do if it builds the same
integer frequency table as the encoder at every step -- for each model width,
each projection dtype (FP32, BF16, FP8) and each supported lanes-per-workgroup count
(1 to 16: up to a full 16-row MFMA tile of live lanes), with
uneven chunks, chunks of length 0, 1 and 2, lanes that run several chunks back
to back and lane counts that are not a multiple of the workgroup's lanes;
and, with the output buffer filled beforehand with wrong bytes, that every
decoded byte is written.
"""
import numpy as np
import pytest
import torch

from synth import ModelConfig, init_weights, records_f32_mix, raw_normal_f32, records_structured64

pytestmark = pytest.mark.gpu

LENS = [700, 1, 2, 0, 129, 3, 1000, 64, 257, 33, 2]


def boa():
    import paper_2511_11337_amd as b
    return b


def make_data(lens, seed):
    gens = [records_f32_mix, records_structured64, raw_normal_f32]
    parts = [gens[i % 3](n, seed + i) if n else np.zeros(0, np.uint8) for i, n in enumerate(lens)]
    return np.concatenate(parts)


def encode(m, data, lens, dtype, max_lanes=0):
    cl = np.asarray(lens, dtype=np.uint64)
    d = torch.from_numpy(data.copy()).cuda()
    pl, po, ln, _ = boa().encode_dev(m, d, cl, dtype=dtype, max_lanes=max_lanes)
    lnh = ln.cpu().numpy().astype(np.uint32).astype(np.uint64)
    off = np.concatenate([[0], np.cumsum(cl)[:-1]]).astype(np.int64)
    firsts = [int(data[o]) if n else 0 for o, n in zip(off, lens)]
    return pl, po, lnh, firsts, cl


@pytest.fixture(scope="module")
def models():
    out = {}
    for d, l, seed in [(64, 2, 4243), (128, 1, 77), (256, 3, 4244), (512, 1, 91)]:
        print(f"[gpu] model d_model={d} n_layers={l}", flush=True)
        cfg = ModelConfig(d_model=d, n_layers=l)
        out[d] = boa().Model(cfg, init_weights(cfg, seed))
    return out


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("d_model", [64, 128, 256, 512])
def test_fused_decode_every_lane_count(models, d_model, dtype):
    m = models[d_model]
    data = make_data(LENS, 100 + d_model)
    pl, po, lnh, firsts, cl = encode(m, data, LENS, dtype)
    lane_counts = [1, 2, 4, 8, 16] if d_model <= 256 else [1, 2, 4, 8]
    for g in lane_counts:
        for max_lanes in (0, 3):            # 3 lanes: several chunks back to back per lane
            print(f"[gpu] fused decode d_model={d_model} {dtype} G={g} max_lanes={max_lanes}", flush=True)
            out = boa().decode_dev(m, pl, po, lnh, firsts, cl, dtype=dtype, max_lanes=max_lanes,
                                   decode_kernel="fused", fused_lanes=g)
            got = out.cpu().numpy()[:data.size]
            bad = np.nonzero(got != data)[0]
            assert bad.size == 0, f"G={g} max_lanes={max_lanes}: first mismatch at byte {bad[:1]}"


def test_fused_matches_step_decoder_cfg2(models):
    """cfg2 shape (d_model 256 x 3 layers), 24 lanes of 1.5 KiB: the fused and
    the step-graph decoder both return the input."""
    m = models[256]
    lens = [1536] * 23 + [777]
    data = np.concatenate([records_f32_mix(n, 500 + i) for i, n in enumerate(lens)])
    for dtype in ("f32", "bf16"):
        pl, po, lnh, firsts, cl = encode(m, data, lens, dtype)
        print(f"[gpu] cfg2 fused vs steps {dtype}", flush=True)
        a = boa().decode_dev(m, pl, po, lnh, firsts, cl, dtype=dtype, decode_kernel="fused")
        b = boa().decode_dev(m, pl, po, lnh, firsts, cl, dtype=dtype, decode_kernel="steps")
        assert np.array_equal(a.cpu().numpy()[:data.size], data)
        assert np.array_equal(b.cpu().numpy()[:data.size], data)


def test_fused_container_round_trip(models):
    m = models[64]
    data = make_data(LENS, 9).tobytes()
    blob = boa().compress(m, data, chunk_lens=LENS, max_lanes=5)
    assert boa().decompress(m, blob, decode_kernel="fused") == data
    assert boa().decompress(m, blob, decode_kernel="fused", fused_lanes=8) == data
    assert boa().decompress(m, blob, decode_kernel="steps") == data


def test_fused_rejects_bad_lane_counts(models):
    m = models[512]
    data = make_data([100, 50], 3)
    pl, po, lnh, firsts, cl = encode(m, data, [100, 50], "f32")
    with pytest.raises(boa().BoaError) as e:
        boa().decode_dev(m, pl, po, lnh, firsts, cl, decode_kernel="fused", fused_lanes=3)
    assert e.value.name == "BOA_E_ARG"


def test_fused_rejects_lane_counts_beyond_lds():
    """d_model 512: 16 lanes per workgroup need more LDS than a CU has; the
    automatic choice picks a count that fits (16 layers: state in device
    memory for every lane count above one)."""
    cfg = ModelConfig(d_model=512, n_layers=16)
    m = boa().Model(cfg, init_weights(cfg, 5))
    data = make_data([40, 30], 4)
    pl, po, lnh, firsts, cl = encode(m, data, [40, 30], "f32")
    with pytest.raises(boa().BoaError) as e:
        boa().decode_dev(m, pl, po, lnh, firsts, cl, decode_kernel="fused", fused_lanes=16)
    assert e.value.name == "BOA_E_ARG"
    out = boa().decode_dev(m, pl, po, lnh, firsts, cl, decode_kernel="fused")      # auto picks a count that fits
    assert np.array_equal(out.cpu().numpy()[:data.size], data)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("d_model", [64, 256])
def test_fused_writes_every_decoded_byte(models, d_model, dtype):
    """The decoded bytes leave the decoder in 64-byte blocks gathered across
    steps: with the output buffer filled beforehand with the complement of
    the expected bytes, every byte must still come out right -- chunk edges on
    and beside 64-byte boundaries, chunks sharing a block, several chunks per
    lane."""
    m = models[d_model]
    lens = LENS + [63, 64, 65, 127, 128, 191, 66, 1, 0, 200]
    data = make_data(lens, 300 + d_model)
    pl, po, lnh, firsts, cl = encode(m, data, lens, dtype)
    for g in (1, 2, 8, 16):
        for max_lanes in (0, 3):
            print(f"[gpu] prefilled output d_model={d_model} {dtype} G={g} max_lanes={max_lanes}", flush=True)
            out = torch.from_numpy(~data).cuda()
            boa().decode_dev(m, pl, po, lnh, firsts, cl, dtype=dtype, max_lanes=max_lanes,
                             decode_kernel="fused", fused_lanes=g, out=out)
            got = out.cpu().numpy()
            bad = np.nonzero(got != data)[0]
            assert bad.size == 0, f"G={g} max_lanes={max_lanes}: first wrong byte at {bad[:1]}"
