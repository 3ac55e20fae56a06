"""The allocation-free decode entry point against boa_decode_dev, through the C ABI.

boa_decode_noalloc_dev carves every device buffer of the call from the
library's fixed per-device scratch array.  Its output must equal that of
boa_decode_dev (fused decoder, library-allocated buffers) byte for byte, and
the original chunks: on two calls in a row, the second with fewer and
shorter chunks (the scratch array keeps the first call's contents), with the
output buffers filled beforehand with wrong bytes.  A call that needs more
than the array holds fails with BOA_E_ARG.
"""
import ctypes as C

import numpy as np
import pytest
import torch

from synth import ModelConfig, init_weights, records_f32_mix, records_structured64, raw_normal_f32

pytestmark = pytest.mark.gpu


def boa():
    import paper_2511_11337_amd as b
    return b


def decode_with(fn_name, m, pl, po, lnh, firsts, cl, dtype, fused_lanes, fill):
    from paper_2511_11337_amd import _lib, _layout, _opts
    lib = _lib.load()
    cl, off, _, _ = _layout(cl)
    po = np.ascontiguousarray(po, dtype=np.uint64)
    ln = np.ascontiguousarray(lnh, dtype=np.uint64)
    fb = np.ascontiguousarray(firsts, dtype=np.uint8)
    out = torch.full((max(int(cl.sum()), 1),), fill, dtype=torch.uint8, device="cuda")
    o = _opts(dtype, 0, 0, decode_kernel="fused", fused_lanes=fused_lanes)
    args = [m.handle, pl.data_ptr(), po.ctypes.data_as(_lib.U64P), ln.ctypes.data_as(_lib.U64P), fb.ctypes.data,
            off.ctypes.data_as(_lib.U64P), cl.ctypes.data_as(_lib.U64P), cl.size, C.byref(o), out.data_ptr()]
    if fn_name == "boa_decode_dev":
        args += [None, 0]
    rc = getattr(lib, fn_name)(*args, int(torch.cuda.current_stream().cuda_stream))
    return rc, out


def encode(m, lens, seed, dtype):
    gens = [records_f32_mix, records_structured64, raw_normal_f32]
    data = np.concatenate([gens[i % 3](n, seed + i) if n else np.zeros(0, np.uint8) for i, n in enumerate(lens)])
    cl = np.asarray(lens, dtype=np.uint64)
    pl, po, ln, _ = boa().encode_dev(m, torch.from_numpy(data).cuda(), cl, dtype=dtype)
    lnh = ln.cpu().numpy().astype(np.uint32).astype(np.uint64)
    off = np.concatenate([[0], np.cumsum(cl)[:-1]]).astype(np.int64)
    firsts = [int(data[o]) if n else 0 for o, n in zip(off, lens)]
    return data, pl, po, lnh, firsts, cl


@pytest.mark.parametrize("dtype,fused_lanes", [("bf16", 1), ("f32", 2)])
def test_noalloc_decode_equals_decode_dev(dtype, fused_lanes):
    print(f"[gpu] no-alloc decode {dtype} lanes/wg {fused_lanes}", flush=True)
    cfg = ModelConfig(d_model=64, n_layers=2)
    m = boa().Model(cfg, init_weights(cfg, 4243))
    first = [900, 1, 0, 2, 333, 1500, 64, 7, 2048, 3]
    second = [100, 2, 0, 257, 1]
    for k, lens in enumerate((first, second)):
        data, pl, po, lnh, firsts, cl = encode(m, lens, 50 + 10 * k, dtype)
        rc_a, a = decode_with("boa_decode_noalloc_dev", m, pl, po, lnh, firsts, cl, dtype, fused_lanes, 0xA5)
        assert rc_a == 0, boa()._lib.load().boa_last_error()
        rc_b, b = decode_with("boa_decode_dev", m, pl, po, lnh, firsts, cl, dtype, fused_lanes, 0x5A)
        assert rc_b == 0
        n = int(cl.sum())
        assert torch.equal(a[:n], b[:n])
        assert np.array_equal(a[:n].cpu().numpy(), data)


def test_noalloc_rejects_calls_beyond_the_scratch():
    from paper_2511_11337_amd import _lib
    cfg = ModelConfig(d_model=64, n_layers=2)
    m = boa().Model(cfg, init_weights(cfg, 4243))
    n = 40000                                     # ~70 B per chunk: more than 2 MiB
    cl = np.full(n, 2, dtype=np.uint64)
    pl = torch.zeros(64 * n, dtype=torch.uint8, device="cuda")
    po = np.arange(n, dtype=np.uint64) * 64
    lnh = np.zeros(n, dtype=np.uint64)
    rc, _ = decode_with("boa_decode_noalloc_dev", m, pl, po, lnh, np.zeros(n, np.uint8), cl, "f32", 0, 0)
    assert rc == -1                               # BOA_E_ARG
    assert "needs" in _lib.load().boa_last_error().decode()
