"""HBM traffic of the fused decoder from rocprofv3 hardware counters.

Two counter runs of the same bench command, one collecting FETCH_SIZE and one
WRITE_SIZE (KiB per dispatch, the L2's reads from and writes to memory), each
also see a plain copy kernel of known size that the bench launches first
(``bench.py --copy-calibration``: 256 MiB read, 256 MiB written).  The copy's
counter reading over its known bytes is the counter's scale; the fused
decoder's reading divided by that scale is its HBM traffic per launch.

The record is keyed by a hash of the sources the fused decoder is built from,
so the bench reports the traffic only while the kernel is the one that was
counted.

    python -m paper_2511_11337_amd.counters FETCH.csv WRITE.csv OUT.json [KERNEL]

The counter runs need not run bench.py itself: `encode PATH` compresses the
bench's batch (same generator, seed, model and tuned launch shape) and saves
the payloads; `decode PATH`, run under the counter profiler, launches the
same 256 MiB calibration copy and then the bench's decoder launch on those
payloads with plain launches (no kernel timers), and checks the round trip.
Only the decode process runs under the profiler.

    python -m paper_2511_11337_amd.counters encode /tmp/batch.npz
    rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR -o run -- \
        python3 -m paper_2511_11337_amd.counters decode /tmp/batch.npz
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["decode_fused.hip", "hotpath_common.h", "device_common.h", "boa_internal.h"]
COPY_BYTES = 256 << 20          # what the calibration copy reads, and writes
# the bench's fused decoder: bf16, d_model 256, 16 lanes per workgroup, state in device memory
KERNEL = "k_dec_fused<1, 256, 512, 16, 16, false>"


def source_hash() -> str:
    h = hashlib.sha256()
    for f in SOURCES:
        with open(os.path.join(_HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _dispatches(path: str, counter: str):
    """[(dispatch id, kernel name, grid size, value)] of one counter."""
    out = []
    with open(path, newline="") as fh:
        for row in csv.DictReader(fh):
            if row.get("Counter_Name") != counter:
                continue
            out.append((int(row["Dispatch_Id"]), row["Kernel_Name"], int(row.get("Grid_Size", 0) or 0),
                        float(row["Counter_Value"])))
    out.sort()
    return out


def measure(path: str, counter: str, kernel: str = KERNEL):
    """(copy reading, fused decoder reading) in KiB: the first dispatch of the
    run is the calibration copy; the fused decoder is its last dispatch of
    the largest grid (the timed batch launch)."""
    ds = _dispatches(path, counter)
    if not ds:
        raise SystemExit(f"{path}: no {counter} rows")
    copy = ds[0]
    fused = [d for d in ds if kernel in d[1]]
    if not fused:
        raise SystemExit(f"{path}: no {kernel} dispatch")
    big = max(d[2] for d in fused)
    dec = [d for d in fused if d[2] == big][-1]
    return copy, dec


def _bench_setup(dtype="bf16"):
    """The bench's batch, trained model and tuned launch shape."""
    import torch
    root = os.path.dirname(_HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import bench
    import paper_2511_11337_amd as boa
    from paper_2511_11337_amd.autotune import tune
    m = boa.Model.load(bench.MODEL_FILE)
    data, lens = bench.make_workload(bench.N_CHUNKS, bench.LEN_LO, bench.LEN_HI)
    d = torch.from_numpy(data).cuda()
    shape = tune(m, d, lens, dtype=dtype, use_cache=False)
    return boa, m, data, lens, d, shape


def encode_batch(path: str, dtype: str = "bf16"):
    import numpy as np
    import torch
    boa, m, data, lens, d, shape = _bench_setup(dtype)
    payload, poff, plen, _ = boa.encode_dev(m, d, lens, dtype=dtype, tile_t=shape["tile_t"], ideal=False)
    torch.cuda.synchronize()
    np.savez(path, payload=payload.cpu().numpy(), poff=np.asarray(poff, dtype=np.uint64),
             plen=plen.cpu().numpy().astype(np.uint32).astype(np.uint64))
    print(f"[counters] encoded {data.size} bytes, payload {int(plen.cpu().numpy().astype(np.uint64).sum())} B, "
          f"shape {shape}", flush=True)


def decode_batch(path: str, dtype: str = "bf16"):
    import numpy as np
    import torch
    src = torch.empty(64 << 20, dtype=torch.float32, device="cuda")     # the calibration copy: 256 MiB each way
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst
    boa, m, data, lens, d, shape = _bench_setup(dtype)
    z = np.load(path)
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    out = boa.decode_dev(m, torch.from_numpy(z["payload"]).cuda(), z["poff"], z["plen"], data[off].copy(), lens,
                         dtype=dtype, decode_kernel=shape["decode_kernel"], fused_lanes=shape["fused_lanes"],
                         use_graph=shape["use_graph"])
    torch.cuda.synchronize()
    ok = bool(torch.equal(out[:data.size], d))
    print(f"[counters] decoded {data.size} bytes with {shape}: round trip {'ok' if ok else 'FAILED'}", flush=True)
    if not ok:
        raise SystemExit(3)


def main(argv):
    if argv and argv[0] in ("encode", "decode"):
        (encode_batch if argv[0] == "encode" else decode_batch)(argv[1], *(argv[2:3]))
        return
    fetch_csv, write_csv, out_json = argv[:3]
    kernel = argv[3] if len(argv) > 3 else KERNEL
    cf, df = measure(fetch_csv, "FETCH_SIZE", kernel)
    cw, dw = measure(write_csv, "WRITE_SIZE", kernel)
    f_scale = cf[3] * 1024.0 / COPY_BYTES
    w_scale = cw[3] * 1024.0 / COPY_BYTES
    rec = {
        "kernel": kernel,
        "source_sha256": source_hash(),
        "copy_kernel": cf[1][:120],
        "copy_bytes": COPY_BYTES,
        "copy_fetch_kib": cf[3], "copy_write_kib": cw[3],
        "fetch_scale": f_scale, "write_scale": w_scale,
        "grid_size": df[2],
        "fetch_kib": df[3], "write_kib": dw[3],
        "hbm_bytes_per_launch": df[3] * 1024.0 / f_scale + dw[3] * 1024.0 / w_scale,
    }
    with open(out_json, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main(sys.argv[1:])
