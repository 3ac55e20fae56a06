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


def main(argv):
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
