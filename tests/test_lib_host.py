"""Host-side checks of libboa (no GPU needed): every symbol include/boa.h
declares is exported, and the error paths that need no device behave."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2511_11337_amd", "libboa.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libboa.so not built")


def declared_functions():
    hdr = open(os.path.join(ROOT, "include", "boa.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(boa_[a-z0-9_]+)\s*\(", hdr)))


def test_every_declared_symbol_is_exported():
    from paper_2511_11337_amd import _lib
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    # the ctypes table covers exactly the declared ABI
    assert set(names) == set(_lib.SIGNATURES)


def test_param_count_matches_layout():
    from paper_2511_11337_amd import Config
    from synth import ModelConfig, param_count
    for d, l in [(64, 2), (256, 3), (512, 4), (128, 1)]:
        assert Config(d, l).n_params == param_count(ModelConfig(d, l))
    # with the feed-forward sub-layer (hidden ffn_mult * d_model <= 1024)
    for d, l, f in [(64, 2, 4), (256, 1, 4), (512, 1, 2)]:
        assert Config(d, l, ffn_mult=f).n_params == param_count(ModelConfig(d, l, ffn_mult=f))
    assert Config(512, 1, ffn_mult=4).n_params == 0
    # unsupported shapes report 0
    assert Config(96, 2).n_params == 0


def test_container_errors_without_device():
    from paper_2511_11337_amd import _lib, container_info, BoaError
    with pytest.raises(BoaError) as e:
        container_info(b"not a container" * 8)
    assert e.value.name == "BOA_E_FORMAT"
    with pytest.raises(BoaError) as e:
        container_info(b"\x00" * 10)
    assert e.value.name == "BOA_E_FORMAT"


def test_numerics_id_encodes_dtype():
    from paper_2511_11337_amd import numerics_id
    assert numerics_id("f32") != numerics_id("bf16")
    assert numerics_id("f32") & 0xFF == 0 and numerics_id("bf16") & 0xFF == 1


def test_model_create_without_gpu_is_an_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_2511_11337_amd import Model, Config, BoaError
    from synth import ModelConfig, init_weights
    w = init_weights(ModelConfig(64, 2), 1)
    with pytest.raises(BoaError) as e:
        Model(Config(64, 2), w)
    assert e.value.name in ("BOA_E_UNSUPPORTED", "BOA_E_DEVICE")


def test_bad_config_rejected():
    from paper_2511_11337_amd import _lib
    lib = _lib.load()
    c = _lib.boa_config(64, 2, 8, 4, 2)       # d_state 8 unsupported
    h = C.c_void_p()
    w = np.zeros(10, np.float32)
    rc = lib.boa_model_create(C.byref(c), w.ctypes.data, w.size, 0, C.byref(h))
    assert rc == -1


def _struct_fields(name):
    hdr = open(os.path.join(ROOT, "include", "boa.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + ";", hdr).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        typ, names = decl.split(None, 1)
        fields += [n.strip() for n in names.split(",")]
    return fields


def test_ctypes_structs_match_header():
    """The binding's structs list the header's fields in order (an ABI drift
    would pass garbage options silently)."""
    from paper_2511_11337_amd import _lib
    for cname, ct in [("boa_config", _lib.boa_config), ("boa_run_opts", _lib.boa_run_opts)]:
        assert [f[0] for f in ct._fields_] == _struct_fields(cname), cname


def _container(lens, total, coder=0, pay=b""):
    """A container with a valid index CRC around the given index records
    (layout of include/boa.h: 64-byte header, 32-byte records, payloads)."""
    import struct
    import zlib
    n = len(lens)
    idx = b"".join(struct.pack("<QQIIBB6x", L, 0, 0, 0, 0, coder) for L in lens)
    hdr = bytearray(64)
    hdr[0:4] = b"BOA1"
    struct.pack_into("<I", hdr, 4, 1)
    struct.pack_into("<QIBB", hdr, 8, 1234, 0, 32, 16)
    struct.pack_into("<QQQQ", hdr, 24, total, lens[0] if n else 0, lens[-1] if n else 0, n)
    struct.pack_into("<I", hdr, 56, zlib.crc32(bytes(hdr[:56]) + idx))
    return bytes(hdr) + idx + pay


def test_crafted_index_lengths_are_rejected():
    """Chunk lengths come from the container: three lengths of about 6e18
    add up to 2 modulo 2^64, which must not pass as a 2-byte container; nor
    may lengths that overshoot or undershoot the total, or a chunk beyond the
    decoder's 2^31 - 1 byte limit."""
    from paper_2511_11337_amd import container_info, BoaError
    big = 6148914691236517206                      # 3 x big = 2 (mod 2^64)
    cases = [([big, big, big], 2), ([5, 7], 10), ([5, 4], 10), ([1 << 31], 1 << 31)]
    for lens, total in cases:
        with pytest.raises(BoaError) as e:
            container_info(_container(lens, total))
        assert e.value.name == "BOA_E_CORRUPT", (lens, total)
    info = container_info(_container([5, 5], 10))     # consistent: accepted (payload sizes 0)
    assert info["n_chunks"] == 2 and info["total_len"] == 10
    bad = bytearray(_container([5, 5], 10))
    bad[64] ^= 1                                      # index byte changed: CRC catches it
    with pytest.raises(BoaError) as e:
        container_info(bytes(bad))
    assert e.value.name == "BOA_E_CRC"


def test_split_and_payload_layout():
    from paper_2511_11337_amd import _chunk_lens, _layout
    assert _chunk_lens(0).tolist() == []
    assert _chunk_lens(10, chunk_len=4).tolist() == [4, 4, 2]
    assert _chunk_lens(8, chunk_len=4).tolist() == [4, 4]
    assert _chunk_lens(3, chunk_len=4).tolist() == [3]
    lens = np.array([5, 0, 1, 7], dtype=np.uint64)
    cl, off, poff, cap = _layout(lens)
    assert off.tolist() == [0, 5, 5, 6]
    assert cap.tolist() == [2 * n + 64 for n in lens.tolist()]
    assert poff.tolist() == [0, 74, 138, 204]


def test_diagnostics_summary_equals_oracle():
    """Top-k and ECE from the GPU kernel's counts, computed by the library,
    against the oracle's definitions on the same counts."""
    import ctypes as C
    from paper_2511_11337_amd import _lib
    from oracle import diagnostics as od
    rng = np.random.default_rng(4)
    for n_bins in (1, 10, 15):
        hist = rng.integers(0, 1000, 256).astype(np.uint32)
        hist[rng.integers(0, 256, 40)] = 0
        cnt = rng.integers(0, 500, n_bins)
        cnt[0] = 0
        cor = (cnt * rng.random(n_bins)).astype(np.int64)
        conf = ((np.arange(n_bins) + rng.random(n_bins)) / n_bins * cnt * 2.0 ** 32).astype(np.uint64)
        cal = np.stack([cnt, cor, conf], axis=1).astype(np.uint64)
        topk = np.zeros(256)
        ece, pos = C.c_double(), C.c_uint64()
        _lib.check(_lib.load().boa_diagnostics_summary(np.ascontiguousarray(hist).ctypes.data,
                                                       np.ascontiguousarray(cal).ctypes.data, n_bins,
                                                       topk.ctypes.data, C.byref(ece), C.byref(pos)))
        assert pos.value == int(hist.sum())
        for k in (1, 5, 10, 256):
            assert abs(topk[k - 1] - od.topk(hist.astype(np.int64), k)) <= 1e-15
        ref = od.ece(cal.astype(np.int64))
        assert abs(ece.value - ref) <= 1e-12, (ece.value, ref)


def _lpt_makespan(steps, lanes):
    """Longest-first onto the least-loaded lane (ties: lowest lane)."""
    import heapq
    h = [(0, i) for i in range(lanes)]
    for s in sorted(steps, reverse=True):
        load, i = heapq.heappop(h)
        heapq.heappush(h, (load + s, i))
    return max(x[0] for x in h)


def test_plan_lanes():
    """boa_plan_lanes: an explicit cap gives min(coded chunks, cap); the
    library's own choice is the largest candidate whose LPT schedule keeps the
    idle rows within 5 % (checked against an independent LPT simulation)."""
    import paper_2511_11337_amd as boa
    from synth import chunk_lengths_uniform
    assert boa.plan_lanes([]) == 0
    assert boa.plan_lanes([0, 1, 1]) == 0                      # nothing to code
    assert boa.plan_lanes([5, 1, 7], 8) == 2
    assert boa.plan_lanes(np.full(300, 1000), 64) == 64
    assert boa.plan_lanes(np.full(100, 1000)) == 100             # one chunk each, no idle rows
    assert boa.plan_lanes(np.full(10000, 1000)) == 5000          # two equal chunks per lane
    for n, lo, hi, seed in [(8192, 32768, 262144, 1341), (3000, 100, 5000, 7), (20000, 512, 4096, 9)]:
        lens = chunk_lengths_uniform(n, lo, hi, seed).astype(np.uint64)
        lanes = boa.plan_lanes(lens)
        steps = [int(x) - 1 for x in lens if x > 1]
        idle = 1.0 - sum(steps) / (lanes * _lpt_makespan(steps, lanes))
        assert 1 <= lanes <= min(len(steps), 8192)
        assert idle <= 0.05, (n, lanes, idle)
        top = min(len(steps), 8192)
        if lanes < top:                                          # the full count would idle more than 5 %
            assert 1.0 - sum(steps) / (top * _lpt_makespan(steps, top)) > 0.05
    assert boa.plan_lanes(chunk_lengths_uniform(8192, 32768, 262144, 1341)) == 4096   # the bench's batch


def test_int8_numerics_id_is_the_integer_pipelines_own():
    """Containers of the integer-only pipeline carry its version alone (no
    kernel version, no device), so any build that follows its rules accepts
    them; the float dtypes' ids differ from it."""
    import paper_2511_11337_amd as boa
    nid = boa.numerics_id("int8")
    assert nid == (0x101 << 8) | 3
    assert nid not in {boa.numerics_id(d) for d in ("f32", "bf16", "fp8")}


def test_container_parser_fuzz():
    """The container index is untrusted input: truncations at every length
    and random index and header fields (with the CRC recomputed, so parsing
    goes past the checksum) return a defined status and never read outside
    the buffer (each case is copied into an exactly sized allocation, so the
    host-sanitizer build of the library would report any overread)."""
    import ctypes as C
    import struct
    import zlib
    from paper_2511_11337_amd import _lib
    lib = _lib.load()
    codes = {0, -4, -5, -7}

    def info(blob):
        buf = np.frombuffer(blob, dtype=np.uint8).copy() if blob else np.zeros(0, np.uint8)
        n, t, fp, nid = C.c_uint64(), C.c_uint64(), C.c_uint64(), C.c_uint32()
        return lib.boa_container_info(buf.ctypes.data if buf.size else None, len(blob), C.byref(n), C.byref(t),
                                       C.byref(fp), C.byref(nid))

    good = _container([5, 9, 1], 15, pay=b"\x00" * 24)
    assert info(good) == 0
    for cut in range(len(good) - 24):               # header and index cut short
        assert info(good[:cut]) in codes - {0}, cut
    rng = np.random.default_rng(77)
    for _ in range(400):
        b = bytearray(good)
        for _ in range(int(rng.integers(1, 4))):
            rec = int(rng.integers(0, 3))
            field = int(rng.choice([0, 8, 16, 20, 25]))          # length, payload offset / size, crc, coder
            width = 8 if field < 16 else (4 if field < 24 else 1)
            val = int(rng.integers(0, 1 << 63)) if rng.random() < 0.5 else int(rng.integers(0, 64))
            b[64 + 32 * rec + field:64 + 32 * rec + field + width] = (val % (1 << (8 * width))).to_bytes(width, "little")
        if rng.random() < 0.3:                                     # header: total, chunk count
            struct.pack_into("<Q", b, int(rng.choice([24, 48])), int(rng.integers(0, 1 << 40)))
        struct.pack_into("<I", b, 56, zlib.crc32(bytes(b[:56]) + bytes(b[64:64 + 96])))
        assert info(bytes(b)) in codes
