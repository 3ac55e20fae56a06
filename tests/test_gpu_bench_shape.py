"""The benchmark's workload in the launch shapes it times, through the C ABI.

* The precision-plus-batching workload at full size (8192 chunks, lengths
  uniform in [32 KiB, 256 KiB], 1.12 GiB of 64-byte structured records; the
  trained d_model 256 x 3 layer model; BF16) in the benchmark's launch shape
  (the tuned table's: encoder tile 256, fused decoder with 16 lanes per
  workgroup; 8192 lanes, caller-owned workspaces): every byte comes back, every chunk's payload is
  within 2 bytes + 1e-3 of its own ideal cost -sum log2(f/M) (a property that
  holds at any size), and the payloads of the two shortest chunks equal the
  oracle coder's bytes on those chunks' GPU tables.
* The same laws scaled down (8192 chunks of 256..2048 bytes) at 8 and 16
  lanes per workgroup and with the per-step decoder: identical bytes.
* The autotuner returns a launch shape that round-trips and is cached.
"""
import os

import numpy as np
import pytest
import torch

from synth import records_structured64, chunk_lengths_uniform
from oracle import coder as oc

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MODELS = os.path.join(ROOT, "paper_2511_11337_amd", "models")


def boa():
    import paper_2511_11337_amd as b
    return b


def trained_model():
    for name in ("records64_d256x3.boam", "records20_d256x3.boam"):
        p = os.path.join(MODELS, name)
        if os.path.exists(p):
            return boa().Model.load(p)
    pytest.skip("no trained model file")


def workload(n, lo, hi, seed):
    lens = chunk_lengths_uniform(n, lo, hi, seed).astype(np.uint64)
    data = np.concatenate([records_structured64(int(x), seed * 1000003 + i) for i, x in enumerate(lens)])
    return data, lens


def test_full_batch_in_bench_shape():
    m = trained_model()
    data, lens = workload(8192, 32768, 262144, 1341)          # the benchmark's own batch
    print(f"[gpu] full batch: {lens.size} chunks, {data.size} bytes", flush=True)
    d = torch.from_numpy(data).cuda()
    from paper_2511_11337_amd import autotune
    shape = autotune.tune(m, d, lens, dtype="bf16", use_cache=False)        # the bench's shape
    tile, g = shape["tile_t"], shape["fused_lanes"] or 16
    print(f"[gpu] full batch shape {shape}", flush=True)
    ws_e = boa().workspace_size(m, lens, "encode", dtype="bf16", tile_t=tile)
    ws_d = boa().workspace_size(m, lens, "decode", dtype="bf16", decode_kernel="fused", fused_lanes=g)
    w_e = torch.empty(ws_e, dtype=torch.uint8, device="cuda")
    pl, po, ln, ib = boa().encode_dev(m, d, lens, dtype="bf16", tile_t=tile, ideal=True, workspace=w_e)
    del w_e
    lnh = ln.cpu().numpy().astype(np.uint32).astype(np.uint64)
    ibh = ib.cpu().numpy()[:lens.size]
    assert np.all(lnh <= ibh / 8 * (1 + 1e-3) + 2)
    print("[gpu] full batch encoded", flush=True)
    pay = pl.cpu().numpy()
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    for i in np.argsort(lens, kind="stable")[:2]:
        c = data[off[i]:off[i] + int(lens[i])]
        tb = boa().logits(m, torch.from_numpy(c[None]).cuda(), dtype="bf16", want_tables=True)[-1]
        tabs = tb[0].cpu().numpy().view(np.uint16).astype(np.int64)
        a, b = int(po[i]), int(po[i]) + int(lnh[i])
        assert bytes(pay[a:b]) == oc.encode_with_tables(c[1:], tabs), i
    w_d = torch.empty(ws_d, dtype=torch.uint8, device="cuda")
    out = boa().decode_dev(m, pl, po, lnh, data[off], lens, dtype="bf16", decode_kernel="fused", fused_lanes=g,
                           workspace=w_d)
    assert torch.equal(out[:data.size], d)


def test_scaled_batch_every_decoder_shape():
    m = trained_model()
    data, lens = workload(8192, 256, 2048, 2341)
    d = torch.from_numpy(data).cuda()
    pl, po, ln, _ = boa().encode_dev(m, d, lens, dtype="bf16", tile_t=256, ideal=False)
    lnh = ln.cpu().numpy().astype(np.uint32).astype(np.uint64)
    firsts = data[np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)]
    for kw in (dict(decode_kernel="fused", fused_lanes=8), dict(decode_kernel="fused", fused_lanes=16),
               dict(decode_kernel="steps")):
        print(f"[gpu] scaled batch decode {kw}", flush=True)
        out = boa().decode_dev(m, pl, po, lnh, firsts, lens, dtype="bf16", **kw)
        assert torch.equal(out[:data.size], d), kw


def test_autotuner_shape_round_trips_and_is_cached(tmp_path, monkeypatch):
    from paper_2511_11337_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    monkeypatch.setattr(autotune, "TABLE", str(tmp_path / "none.json"))
    m = trained_model()
    data, lens = workload(512, 512, 4096, 3341)
    d = torch.from_numpy(data).cuda()
    t = autotune.tune(m, d, lens, dtype="bf16", sample_bytes=512)
    assert t["tile_t"] in autotune.TILES and t["decode_kernel"] in ("fused", "steps")
    assert (tmp_path / "tune.json").exists()
    assert autotune.tune(m, d, lens, dtype="bf16", sample_bytes=512) == t       # from the cache
    pl, po, ln, _ = boa().encode_dev(m, d, lens, dtype="bf16", tile_t=t["tile_t"], ideal=False)
    lnh = ln.cpu().numpy().astype(np.uint32).astype(np.uint64)
    firsts = data[np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)]
    out = boa().decode_dev(m, pl, po, lnh, firsts, lens, dtype="bf16", use_graph=t["use_graph"],
                           decode_kernel=t["decode_kernel"], fused_lanes=t["fused_lanes"])
    assert torch.equal(out[:data.size], d)
