"""The hardware-counter traffic record (paper_2511_11337_amd/counters.py),
on synthetic counter CSVs: the first dispatch is the calibration copy, the
fused decoder's reading is its last largest-grid dispatch, and each counter
is scaled by the copy's reading over the copy's known bytes."""
import csv
import json

from paper_2511_11337_amd import counters


def write_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for did, name, grid, val in rows:
            w.writerow({"Dispatch_Id": did, "Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter,
                        "Counter_Value": val})


def test_traffic_record_from_synthetic_counters(tmp_path):
    k = "void boa::" + counters.KERNEL + "(boa::FusedArgs)"
    copy = "void at::native::vectorized_elementwise_kernel<4>"
    f = tmp_path / "f.csv"
    w = tmp_path / "w.csv"
    # copy reads 256 MiB but the counter reports half; writes report in full
    write_csv(f, "FETCH_SIZE", [(3, k, 2048, 999.0), (1, copy, 1 << 24, 131072.0), (7, k, 131072, 5000.0),
                                (9, k, 512, 1.0), (5, "other", 64, 12.0)])
    write_csv(w, "WRITE_SIZE", [(1, copy, 1 << 24, 262144.0), (7, k, 131072, 8000.0), (3, k, 2048, 1.0)])
    out = tmp_path / "t.json"
    counters.main([str(f), str(w), str(out)])
    rec = json.loads(out.read_text())
    assert rec["fetch_scale"] == 0.5 and rec["write_scale"] == 1.0
    assert rec["grid_size"] == 131072 and rec["fetch_kib"] == 5000.0 and rec["write_kib"] == 8000.0
    assert rec["hbm_bytes_per_launch"] == 5000.0 * 1024 / 0.5 + 8000.0 * 1024
    assert rec["source_sha256"] == counters.source_hash()
