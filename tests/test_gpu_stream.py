"""Streaming compressor through the C ABI: bytes pushed in pieces of random
size become shards of lanes x chunk_len bytes, each bit-identical to the
one-shot container of the same bytes, handed out in input order; the shards
decompress back to the stream.  Covers a partial last group and a short last
chunk, several worker counts, shards taken while pushing, an empty stream and
push after finish."""
import numpy as np
import pytest

from synth import ModelConfig, init_weights, records_f32_mix, records_structured64

pytestmark = pytest.mark.gpu

CFG1 = ModelConfig(d_model=64, n_layers=2)


def boa():
    import paper_2511_11337_amd as b
    return b


@pytest.fixture(scope="module")
def m1():
    print("[gpu] stream model cfg1", flush=True)
    return boa().Model(CFG1, init_weights(CFG1, 4243))


def stream_bytes(n, seed):
    a = records_f32_mix(n // 2, seed)
    b = records_structured64(n - n // 2, seed + 1)
    return np.concatenate([a, b]).tobytes()


def run_stream(m, data, chunk, lanes, workers, seed, dtype="f32"):
    r = np.random.default_rng(seed)
    shards = []
    with boa().StreamCompressor(m, chunk_len=chunk, lanes=lanes, workers=workers, dtype=dtype) as st:
        i = 0
        while i < len(data):
            k = int(r.integers(1, 100_000))
            st.push(data[i:i + k])
            i += k
            shards.extend(st.shards(wait=False))               # whatever is done so far
        st.finish()
        shards.extend(st.shards(wait=True))
    return shards


@pytest.mark.parametrize("workers", [1, 2, 4])
def test_stream_shards_equal_one_shot_containers(m1, workers):
    chunk, lanes = 16384, 8
    data = stream_bytes(10 * chunk * lanes + 3 * chunk + 1234, 77)   # 10 full groups, a partial one, short last chunk
    print(f"[gpu] stream workers={workers}: {len(data)} bytes", flush=True)
    shards = run_stream(m1, data, chunk, lanes, workers, 5)
    g = chunk * lanes
    assert len(shards) == 11
    for i, sh in enumerate(shards):
        assert sh == boa().compress(m1, data[i * g:(i + 1) * g], chunk_len=chunk), f"shard {i}"
    assert boa().decompress_shards(m1, shards) == data


def test_stream_bf16_round_trip(m1):
    data = stream_bytes(300_001, 91)
    shards = run_stream(m1, data, 4096, 16, 2, 6, dtype="bf16")
    assert len(shards) == (len(data) + 65535) // 65536
    assert boa().decompress_shards(m1, shards) == data


def test_stream_edge_cases(m1):
    with boa().StreamCompressor(m1, chunk_len=1024, lanes=4) as st:       # nothing pushed
        st.finish()
        assert list(st.shards()) == []
    with boa().StreamCompressor(m1, chunk_len=1024, lanes=4) as st:       # shorter than one chunk
        st.push(b"\x01\x02\x03")
        assert st.next_shard(wait=True) is None                          # nothing in flight before finish
        st.finish()
        sh = list(st.shards())
        assert len(sh) == 1 and boa().decompress_shards(m1, sh) == b"\x01\x02\x03"
        with pytest.raises(boa().BoaError) as e:
            st.push(b"x")
        assert e.value.name == "BOA_E_ARG"
    for bad in (dict(chunk_len=0), dict(lanes=0), dict(workers=0), dict(workers=9)):
        with pytest.raises(boa().BoaError) as e:
            boa().StreamCompressor(m1, **{**dict(chunk_len=1024, lanes=4, workers=2), **bad})
        assert e.value.name == "BOA_E_ARG"
