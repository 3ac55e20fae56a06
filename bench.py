#!/usr/bin/env python3
"""Benchmark of the BOA Constrictor hot path on one MI355X.

Workload (default): the precision-plus-batching workload -- 8192 independent
chunks with lengths uniform in [32 KiB, 256 KiB] (about 1.12 GiB) of 64-byte
structured records (counters, cycling detector IDs, quantised float16
kinematics with jitter), compressed and decompressed by the byte-level Mamba
predictor (d_model 256, 3 layers, d_state 16, d_conv 4, expand 2) trained on
device by the library's own kernels -- the training recipe on 64 MiB of
20-byte records, then the same recipe on 64 MiB of 64-byte structured
records (model files under paper_2511_11337_amd/models/) -- with BF16
projections, FP32 accumulation, FP32 scan and softmax, integer CDF.

One step = the whole hot path over that batch with inputs already resident in
HBM: encode every chunk (model forward over every position, histograms,
range coding) and decode it again (fused persistent decoder: model step,
histogram, range decoding, feedback of the decoded byte), each with a
workspace allocated once before the timed region.  The round trip is checked
for byte identity outside the timed region.  No warm-up step by default: one
step takes about two minutes, the encoder's kernels are launched thousands of
times in it, and the decoder is one launch of a minute (so its own first-launch
cost is noise); the timed decoder launch is then the only launch of its kernel
in the run, which a kernel trace of this command can be checked against.
Launch shapes come from the tuned table shipped for this device
(paper_2511_11337_amd/tuned.json), or from a sweep over prefixes of every
chunk (--retune, or a device the table lacks).

Beside the headline: compression ratio and storage-saving rate, coded and
ideal bits/byte, the BF16 bits/byte loss against the FP64 oracle on a
subsample, the plain FP32 single-stream GPU path (one lane), FP32 and FP8
batched runs on a subsample, kernel times of the timed step with the
dominant kernel's roofline, streaming compress, predictor diagnostics, and
the FP64 CPU oracle timed on a bounded sample.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

D_MODEL, N_LAYERS = 256, 3
N_CHUNKS, LEN_LO, LEN_HI, DATA_SEED = 8192, 32768, 262144, 1341
MIX_SEED = 1342                                            # the mixed-stream FP8 workload (data seed 1337 + 5)
MODEL_FILE = os.path.join(ROOT, "paper_2511_11337_amd", "models", "records64_d256x3.boam")
BASE_MODEL_FILE = os.path.join(ROOT, "paper_2511_11337_amd", "models", "records20_d256x3.boam")
PEAK = {"f32": 157.3, "bf16": 2500.0, "fp8": 5000.0}      # dense MFMA TFLOP/s
HBM_PEAK = 8000.0                                          # GB/s
# transcendentals: 256 CUs x 4 SIMDs x 16 lanes at quarter rate x 2.4 GHz
EXP_PEAK = 256 * 4 * 16 / 4 * 2.4e9
KIND_NAMES = ["embed", "in_proj", "mixer", "out_proj", "head", "decode", "quant", "encode", "fused_decoder", "ffn"]
K_COUNT = len(KIND_NAMES)
K_FUSED = 8


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def per_byte_work(D: int = D_MODEL, L: int = N_LAYERS):
    """Per coded byte: projection FLOPs on MFMA (in_proj, x_proj, dt_proj,
    out_proj per layer and the head), mixer FLOPs (conv, scan, gate) and
    transcendentals (exp of the scan per (d, n); softplus, SiLU x 2 per
    channel; 256 exps of the softmax)."""
    Di, N, R = 2 * D, 16, (D + 15) // 16
    proj = L * 2.0 * (2 * Di * D + (R + 2 * N) * Di + R * Di + D * Di) + 2.0 * 256 * D
    mixer = L * (8.0 * Di + 6.0 * Di * N + 4.0 * Di)
    trans = L * (Di * N + 3.0 * Di) + 256.0
    return proj, mixer, trans


def state_bytes_per_lane(D: int = D_MODEL, L: int = N_LAYERS):
    """FP32 conv window (3 taps) and scan state (16 per channel) of one stream
    over all layers."""
    return L * 2 * D * (3 + 16) * 4


def traffic_record(kernel: str, workload: str):
    """HBM bytes per launch of the fused decoder from the committed counter
    record of this workload, while the kernel's sources are the ones counted."""
    from paper_2511_11337_amd import counters
    path = os.path.join(ROOT, "profiles", f"traffic_k_dec_fused_{workload}.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    if rec.get("source_sha256") != counters.source_hash() or kernel not in rec.get("kernel", ""):
        return None
    return rec


def make_mixed(n_chunks: int, scale: int):
    """The mixed-stream FP8 workload's batch: chunk lengths
    floor(16384 / scale * 64^(u^2.415)) (mean 128 KiB / scale), stream type =
    chunk index mod 3 (20-byte records, 64-byte records, raw float32)."""
    from synth import chunk_lengths_heavy, mixed_chunks
    lens = chunk_lengths_heavy(n_chunks, MIX_SEED, lo=16384 // scale, ratio=64.0).astype(np.uint64)
    chunks = mixed_chunks(lens, MIX_SEED)
    return np.concatenate([c for _, c in chunks]), lens


def make_workload(n_chunks: int, lo: int, hi: int):
    from synth import records_structured64, chunk_lengths_uniform
    lens = chunk_lengths_uniform(n_chunks, lo, hi, DATA_SEED).astype(np.uint64)
    data = np.concatenate([records_structured64(int(n), DATA_SEED * 1000003 + i) for i, n in enumerate(lens)])
    return data, lens


def cpu_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def oracle_sample(W, chunks):
    """FP64 oracle compress + decompress of equal-length chunks (one lane each);
    returns (seconds, ideal bits -sum log2 p64, cost -sum log2 f64(s)/M of the oracle's own
    integer tables, coded payload bytes)."""
    from oracle import model as om, coder as oc
    lanes, nbytes = chunks.shape
    t0 = time.perf_counter()
    S = om.StreamState(W.cfg, lanes)
    encs = [oc.Encoder() for _ in range(lanes)]
    ideal = tab = 0.0
    for t in range(nbytes - 1):
        p = om.softmax(om.step(W, S, chunks[:, t]))
        for b in range(lanes):
            s = int(chunks[b, t + 1])
            ideal -= float(np.log2(p[b, s]))
            f = oc.quantise(p[b])
            tab -= float(np.log2(f[s] / oc.M))
            c = oc.cdf(f)
            encs[b].encode(int(c[s]), int(f[s]))
    payloads = [e.finish() for e in encs]
    S = om.StreamState(W.cfg, lanes)
    decs = [oc.Decoder(pl) for pl in payloads]
    out = np.zeros_like(chunks)
    out[:, 0] = chunks[:, 0]
    for t in range(nbytes - 1):
        p = om.softmax(om.step(W, S, out[:, t]))
        for b in range(lanes):
            out[b, t + 1] = decs[b].decode(oc.cdf(oc.quantise(p[b])))
    dt = time.perf_counter() - t0
    assert np.array_equal(out, chunks)
    return dt, ideal, tab, sum(len(p) for p in payloads)


# v_dot4_i32_i8 rate: 256 CUs x 4 SIMDs x 16 lanes x 4 multiply-adds (8 ops) per cycle x 2.4 GHz
DOT4_PEAK_TOPS = 256 * 4 * 16 * 8 * 2.4e9 / 1e12


def int_ops_per_byte(D: int = D_MODEL, L: int = N_LAYERS) -> int:
    """INT8 multiply-adds x 2 of one step of the integer pipeline: in_proj,
    x_proj, dt_proj, out_proj per layer, then the head."""
    Di, R = 2 * D, -(-D // 16)
    return 2 * (L * (2 * Di * D + (R + 32) * Di + Di * R + D * Di) + 256 * D)


def int_leg(m, sub, d_sub, sub_lens, sub_len, n_chunks):
    """The integer-only pipeline (device-independent tables) encoding and
    decoding the subsample; each call allocates its chunk state and waits."""
    import torch
    import paper_2511_11337_amd as boa
    q = boa.QModel(m)
    boa.int_encode_dev(q, d_sub[:2 * sub_len], sub_lens[:2])          # first launch outside the timing
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pq, oq, lq = boa.int_encode_dev(q, d_sub, sub_lens)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lqh = lq.cpu().numpy().astype(np.uint32).astype(np.uint64)
    t2 = time.perf_counter()
    outq = boa.int_decode_dev(q, pq, oq, lqh, sub[::sub_len], sub_lens)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ops = int_ops_per_byte() * (sub.size - n_chunks)
    tops = ops / (t3 - t2) / 1e12
    return {"value": sub.size / (t1 - t0 + t3 - t2) / 1e6, "encode_MBps": sub.size / (t1 - t0) / 1e6,
            "decode_MBps": sub.size / (t3 - t2) / 1e6,
            "coded_bits_per_byte": int(lqh.sum()) * 8 / (sub.size - n_chunks),
            "round_trip_ok": bool(torch.equal(outq[:sub.size], d_sub)),
            "roofline": {"bound": "alu", "kernel": "k_int_chunk<256> (decode)", "achieved": tops,
                         "peak": DOT4_PEAK_TOPS, "unit": "TOP/s (INT8 dot products)", "frac": tops / DOT4_PEAK_TOPS,
                         "ops_per_byte": int_ops_per_byte()},
            "sample": f"first {sub_len // 1024} KiB of every chunk ({sub.size / 2 ** 20:.0f} MiB), one workgroup "
                      f"per chunk, wall clock of the synchronous calls (their state allocation included)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--dtype", default="bf16", choices=["f32", "bf16", "fp8"],
                    help="projection dtype of the batched run (the metric's target is batched BF16)")
    ap.add_argument("--chunks", type=int, default=N_CHUNKS)
    ap.add_argument("--len-lo", type=int, default=LEN_LO)
    ap.add_argument("--len-hi", type=int, default=LEN_HI)
    ap.add_argument("--model", default=MODEL_FILE)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the subsample comparison runs, streaming compress and diagnostics")
    ap.add_argument("--fixed-shape", default="",
                    help="skip the autotuner: 'tile,fused_lanes' (e.g. 64,8); for hardware-counter runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first launch a plain 256 MiB copy (read + write) for hardware-counter scaling")
    ap.add_argument("--workload", default="structured64", choices=["structured64", "mixed"],
                    help="structured64: the 1.12 GiB batch of 64-byte records (default); mixed: the mixed-stream "
                         "FP8 workload (--chunks, default 32768, lengths divided by --scale; a d_model 512 x 4 "
                         "model trained on the mixed stream, --model)")
    ap.add_argument("--scale", type=int, default=1, help="mixed workload: chunk lengths divided by this")
    ap.add_argument("--retune", action="store_true",
                    help="sweep the launch shapes instead of taking the tuned table shipped for this device")
    ap.add_argument("--int8-only", action="store_true",
                    help="run only the integer-only pipeline on the subsample (first 4 KiB of every chunk) and "
                         "print its record; for the kernel trace of that kernel")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path (asked for {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2511_11337_amd as boa
    from paper_2511_11337_amd import _lib
    from paper_2511_11337_amd.autotune import tune, in_table

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if not os.path.exists(args.model):
        print(f"trained model {args.model} missing: python -m paper_2511_11337_amd.recipe --out {args.model}",
              file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 256 MiB read, 256 MiB written")
    m = boa.Model.load(args.model)
    Dm, Lm = m.cfg.d_model, m.cfg.n_layers
    mixed = args.workload == "mixed"
    if not mixed:
        assert (Dm, Lm) == (D_MODEL, N_LAYERS)
    t0 = time.perf_counter()
    if mixed:
        data, lens = make_mixed(args.chunks if args.chunks != N_CHUNKS else 32768, args.scale)
    else:
        data, lens = make_workload(args.chunks, args.len_lo, args.len_hi)
    total = int(data.size)
    n_chunks = int(lens.size)
    log(f"{n_chunks} chunks, {total} bytes ({total / 2 ** 30:.3f} GiB) generated in {time.perf_counter() - t0:.1f} s")
    d_data = torch.from_numpy(data).cuda()
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    firsts = data[off].copy()
    if args.int8_only:
        sub_len = 4096
        sub = np.concatenate([data[o:o + sub_len] for o in off])
        rec = int_leg(m, sub, torch.from_numpy(sub).cuda(), np.full(n_chunks, sub_len, dtype=np.uint64), sub_len,
                      n_chunks)
        print(json.dumps({"int8_pipeline_subsample": rec}), flush=True)
        return

    if args.fixed_shape:
        tile, g = (int(x) for x in args.fixed_shape.split(","))
        tuned = {"tile_t": tile, "decode_kernel": "fused", "fused_lanes": g, "use_graph": False}
        tuned_from = "--fixed-shape"
    else:
        tuned = tune(m, d_data, lens, dtype=args.dtype, use_cache=False, use_table=not args.retune)
        tuned_from = "tuned table" if not args.retune and in_table(m, args.dtype, n_chunks) else "sweep"
    log("launch shape", tuned, "from", tuned_from)
    dec_kw = dict(use_graph=tuned["use_graph"], decode_kernel=tuned["decode_kernel"], fused_lanes=tuned["fused_lanes"])
    ws_e = boa.workspace_size(m, lens, "encode", dtype=args.dtype, tile_t=tuned["tile_t"])
    ws_d = boa.workspace_size(m, lens, "decode", dtype=args.dtype, **{k: dec_kw[k] for k in
                                                                     ("decode_kernel", "fused_lanes")})
    w_enc = torch.empty(max(ws_e, 1), dtype=torch.uint8, device="cuda")
    w_dec = torch.empty(max(ws_d, 1), dtype=torch.uint8, device="cuda")
    out = torch.empty(total, dtype=torch.uint8, device="cuda")
    log(f"workspaces: encode {ws_e / 2 ** 20:.1f} MiB, decode {ws_d / 2 ** 20:.1f} MiB")

    def enc():
        return boa.encode_dev(m, d_data, lens, dtype=args.dtype, tile_t=tuned["tile_t"], ideal=True, workspace=w_enc)

    def dec(payload, poff, plen_h):
        return boa.decode_dev(m, payload, poff, plen_h, firsts, lens, dtype=args.dtype, out=out, workspace=w_dec,
                              **dec_kw)

    for i in range(args.warmup):
        log("warmup", i)
        payload, poff, plen, ib = enc()
        dec(payload, poff, plen.cpu().numpy().astype(np.uint32).astype(np.uint64))
    torch.cuda.synchronize()
    lib = _lib.load()
    t_enc = t_dec = 0.0
    enc_ms = np.zeros(K_COUNT)
    enc_n = np.zeros(K_COUNT, dtype=np.uint64)
    dec_ms = np.zeros(K_COUNT)
    dec_n = np.zeros(K_COUNT, dtype=np.uint64)
    for i in range(args.steps):
        log("step", i)
        # every launch of the step is bracketed by GPU timestamps on its own stream
        lib.boa_prof_read(None, None, 1)
        lib.boa_prof_enable((1 << K_COUNT) - 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        payload, poff, plen, ib = enc()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plen_h = plen.cpu().numpy().astype(np.uint32).astype(np.uint64)
        ms, n = np.zeros(K_COUNT), np.zeros(K_COUNT, dtype=np.uint64)
        lib.boa_prof_read(ms.ctypes.data, n.ctypes.data, 1)
        enc_ms += ms
        enc_n += n
        t2 = time.perf_counter()
        dec(payload, poff, plen_h)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        ms, n = np.zeros(K_COUNT), np.zeros(K_COUNT, dtype=np.uint64)
        lib.boa_prof_read(ms.ctypes.data, n.ctypes.data, 1)
        lib.boa_prof_enable(0)
        dec_ms += ms
        dec_n += n
        t_enc += t1 - t0
        t_dec += t3 - t2
        log(f"step {i}: encode {t1 - t0:.3f} s, decode {t3 - t2:.3f} s")
    ok = bool(torch.equal(out, d_data))
    pay = plen_h.astype(np.int64)
    pay = np.where(pay == 0xFFFFFFFF, np.iinfo(np.int64).max, pay)
    stored = np.minimum(pay, np.maximum(lens.astype(np.int64) - 1, 0))        # raw when coding does not pay
    container = 64 + 32 * n_chunks + int(stored.sum())
    coded = int(np.minimum(pay, np.iinfo(np.int64).max).sum())
    ideal = float(ib.cpu().numpy()[:n_chunks].sum())
    coded_positions = total - n_chunks
    ms_step = (t_enc + t_dec) / args.steps * 1e3
    enc_MBps = total * args.steps / t_enc / 1e6
    dec_MBps = total * args.steps / t_dec / 1e6
    res = {
        "metric": "encode/decode MB/s on 1 GPU at fixed bits/byte; batched BF16 vs plain FP32",
        "value": total / (ms_step / 1e3) / 1e6,
        "unit": "MB/s (1e6 uncompressed bytes/s, encode+decode round trip)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": (f"{n_chunks} chunks, lengths uniform in [{args.len_lo // 1024}, "
                                f"{args.len_hi // 1024}] KiB ({total / 2 ** 30:.3f} GiB) of 64-byte structured "
                                f"records; byte Mamba d_model {D_MODEL} x {N_LAYERS} layers trained on device "
                                f"(recipe on 20-byte records, then on 64-byte records)") if not mixed else
                               (f"{n_chunks} mixed-stream chunks (20-byte records, 64-byte records, raw float32 in "
                                f"turn), lengths floor(16384 / {args.scale} * 64^(u^2.415)) "
                                f"({total / 2 ** 20:.1f} MiB); byte Mamba d_model {Dm} x {Lm} layers "
                                f"({os.path.basename(args.model)})"),
                   "chunks": n_chunks, "bytes": total, "lanes": boa.plan_lanes(lens), "projections": args.dtype},
        "encode_MBps": enc_MBps,
        "decode_MBps": dec_MBps,
        "compression_ratio": total / container,
        "storage_saving_rate_MBps": (total - container) / (t_enc / args.steps) / 1e6,
        "container_bytes": container,
        "coded_bits_per_byte": coded * 8 / coded_positions,
        "ideal_bits_per_byte": ideal / coded_positions,
        "round_trip_ok": ok,
        "autotuned": tuned, "launch_shape_from": tuned_from,
        "workspace_bytes": {"encode": ws_e, "decode": ws_d},
    }

    _, _, _, ib2 = boa.order2_encode(d_data, lens)
    res["order2_bits_per_byte"] = float(ib2.cpu().numpy()[:n_chunks].sum()) / coded_positions
    del ib2

    # ---------------------------------------------------------------- kernel times and roofline
    share = {}
    for k in range(K_COUNT):
        if dec_n[k]:
            share[("decode", k)] = dec_ms[k]
        if enc_n[k]:
            share[("encode", k)] = enc_ms[k]
    res["kernel_time_ms_per_step"] = {f"{ph}:{KIND_NAMES[k]}": round(float(v) / args.steps, 2)
                                      for (ph, k), v in sorted(share.items(), key=lambda kv: -kv[1])}
    (phase, kind), _ = max(share.items(), key=lambda kv: kv[1])
    tab_ms, tab_n = (dec_ms, dec_n) if phase == "decode" else (enc_ms, enc_n)
    avg_s = tab_ms[kind] / tab_n[kind] / 1e3
    proj, mixer, trans = per_byte_work(Dm, Lm)
    if kind == K_FUSED:
        # Thousands of lanes' FP32 conv and scan state (114 KiB each) cannot
        # stay on chip, so every decoded byte reads and writes its lane's state
        # in HBM: that stream, the decoded byte and the payload read are the
        # kernel's algorithmic HBM bytes, and HBM is its roofline.
        positions = coded_positions                      # one launch decodes every chunk
        g = tuned["fused_lanes"]
        kname = f"k_dec_fused<{ {'f32': 0, 'bf16': 1, 'fp8': 2}[args.dtype] }, {Dm}, {2 * Dm}, " \
                f"{(Dm + 15) // 16}, {g}, {'true' if g == 1 and Dm <= 256 else 'false'}>"
        per_pos = 2.0 * state_bytes_per_lane(Dm, Lm) + 1.0 + coded * 1.0 / positions
        hbm = per_pos * positions
        achieved = hbm / avg_s / 1e9
        rec = traffic_record(kname, f"{args.dtype}_{n_chunks}x{args.len_lo // 1024}-{args.len_hi // 1024}KiB")
        res["roofline"] = {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK, "unit": "GB/s",
            "frac": achieved / HBM_PEAK, "traffic": rec["hbm_bytes_per_launch"] if rec else None,
            "kernel": kname, "avg_launch_us": avg_s * 1e6, "positions_per_launch": positions,
            "bytes_per_position": per_pos, "work_per_launch": hbm,
            "bytes_note": "per decoded byte: FP32 conv window and scan state of every layer read and written "
                          f"({2 * state_bytes_per_lane(Dm, Lm)} B), the decoded byte, the payload bits / 8",
            "mfma": {"flops_per_position": proj, "achieved_tflops": proj * positions / avg_s / 1e12,
                     "peak_tflops": PEAK[args.dtype], "frac": proj * positions / avg_s / 1e12 / PEAK[args.dtype]},
            "exp_valu": {"transcendentals_per_position": trans, "achieved_per_s": trans * positions / avg_s,
                         "peak_per_s": EXP_PEAK, "frac": trans * positions / avg_s / EXP_PEAK},
            "lanes_per_workgroup": g,
        }
        if rec:
            res["roofline"]["traffic_source"] = {k: rec[k] for k in ("fetch_kib", "write_kib", "fetch_scale",
                                                                      "write_scale") if k in rec}
    else:
        rows = coded_positions
        flops = (proj if kind in (1, 3, 4) else mixer) * rows
        achieved = flops / avg_s / 1e12
        pk = PEAK[args.dtype] if kind in (1, 3, 4) else 157.3
        res["roofline"] = {"bound": "mfma" if kind in (1, 3, 4) else "alu", "achieved": achieved, "peak": pk,
                           "unit": "TFLOP/s", "frac": achieved / pk, "traffic": None,
                           "kernel": f"{phase} {KIND_NAMES[kind]}", "avg_launch_us": avg_s * 1e6}
    # the round trip against the per-byte ceilings of the method's own work
    hbm_dec = HBM_PEAK * 1e9 / (2.0 * state_bytes_per_lane(Dm, Lm)) / 1e6
    res["ceilings_MBps"] = {"mfma": PEAK[args.dtype] * 1e12 / proj / 1e6, "exp_valu": EXP_PEAK / trans / 1e6,
                            "decode_hbm_state": hbm_dec, "decode_frac_of_hbm_state": dec_MBps / hbm_dec,
                            "decode_frac_of_exp_valu": dec_MBps / (EXP_PEAK / trans / 1e6),
                            "encode_frac_of_exp_valu": enc_MBps / (EXP_PEAK / trans / 1e6)}

    # ---------------------------------------------------------------- FP64 comparison per stream type (mixed)
    if mixed:
        from synth import ModelConfig
        from oracle import model as om, coder as oc
        W = om.Weights(ModelConfig(Dm, Lm), m.get_weights())
        per_type = {}
        for t, name in enumerate(("records20", "records64", "raw_f32")):
            log(f"FP64 oracle on the {name} sample")
            idx = [c for c in range(t, n_chunks, 3) if lens[c] >= 1024][:4]
            smp = np.stack([data[off[c]:off[c] + 1024] for c in idx])
            _, _, tbt = boa.logits(m, torch.from_numpy(smp).cuda(), dtype=args.dtype, want_probs=True,
                                   want_tables=True)
            tbt = tbt.cpu().numpy().view(np.uint16).astype(np.int64)
            tg = smp[:, 1:].astype(np.int64)[..., None]
            gpu_c = float(-np.log2(np.take_along_axis(tbt, tg, -1) / 65536.0).sum())
            p64 = om.softmax(om.stream_logits(W, smp))
            f64 = np.stack([np.stack([oc.quantise(p64[b, i]) for i in range(p64.shape[1])]) for b in range(len(idx))])
            ora_c = float(-np.log2(np.take_along_axis(f64, tg, -1) / oc.M).sum())
            npos_t = tg.size
            per_type[name] = {"gpu_table_bits_per_byte": gpu_c / npos_t, "fp64_table_bits_per_byte": ora_c / npos_t,
                              "loss_frac": gpu_c / ora_c - 1.0}
        res["bits_per_byte_loss_vs_fp64_by_type"] = {"dtype": args.dtype, **per_type,
                                                      "sample": "4 chunks x first 1 KiB per stream type"}
    else:
        # ---------------------------------------------------------------- FP64 subsample and CPU oracle
        sub_chunks, sub_bytes = 16, 2048
        pick = np.linspace(0, n_chunks - 1, sub_chunks).astype(np.int64)
        sample = np.stack([data[off[c]:off[c] + sub_bytes] for c in pick])
        _, _, tb = boa.logits(m, torch.from_numpy(sample).cuda(), dtype=args.dtype, want_probs=True, want_tables=True)
        tb = tb.cpu().numpy().view(np.uint16).astype(np.int64)
        tgt = sample[:, 1:].astype(np.int64)[..., None]
        gpu_bits = float(-np.log2(np.take_along_axis(tb, tgt, -1) / 65536.0).sum())
        if os.path.exists(BASE_MODEL_FILE) and os.path.abspath(args.model) != os.path.abspath(BASE_MODEL_FILE):
            mb = boa.Model.load(BASE_MODEL_FILE)
            _, _, tb0 = boa.logits(mb, torch.from_numpy(sample).cuda(), dtype=args.dtype, want_probs=True,
                                   want_tables=True)
            tb0 = tb0.cpu().numpy().view(np.uint16).astype(np.int64)
            npos0 = sample.shape[0] * (sample.shape[1] - 1)
            res["base_model_coded_bits_per_byte"] = {
                "value": float(-np.log2(np.take_along_axis(tb0, tgt, -1) / 65536.0).sum()) / npos0,
                "model": "trained on 20-byte records only (before fine-tuning on 64-byte records)",
                "sample": f"{sub_chunks} chunks x first {sub_bytes} B"}
            del mb
        if not args.no_cpu_baseline:
            log("cpu baseline (FP64 oracle)")
            from synth import ModelConfig
            from oracle import model as om
            W = om.Weights(ModelConfig(D_MODEL, N_LAYERS), m.get_weights())
            dt, ideal64, tab64, coded64 = oracle_sample(W, sample)
            try:
                from threadpoolctl import threadpool_info
                cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
            except Exception:  # pragma: no cover
                cores = 1
            npos = sample.shape[0] * (sample.shape[1] - 1)
            res["cpu_baseline"] = {
                "value": sample.size / dt / 1e6, "unit": "MB/s (encode+decode round trip)", "cores": int(cores),
                "kind": "oracle", "cpu": cpu_info(), "host_threads": os.cpu_count(),
                "sample": f"{sub_chunks} chunks x first {sub_bytes} B of the same batch, FP64 NumPy model step + "
                          f"Python-integer range coder, compress and decompress ({dt:.1f} s)",
                "fp64_table_bits_per_byte": tab64 / npos, "oracle_payload_bits_per_byte": coded64 * 8 / npos}
            # like for like: the cost -sum log2 f(s)/M of the GPU's integer tables against that of the
            # oracle's FP64 tables under the same quantiser (the minimum-frequency floor caps the cost of
            # confident misses in both); -sum log2 p64 beside it
            res["bits_per_byte_loss_vs_fp64"] = {
                "dtype": args.dtype, "gpu_table_bits_per_byte": gpu_bits / npos,
                "fp64_table_bits_per_byte": tab64 / npos, "loss_frac": gpu_bits / tab64 - 1.0,
                "fp64_softmax_bits_per_byte": ideal64 / npos,
                "sample": f"{sub_chunks} chunks x first {sub_bytes} B (same prefixes as cpu_baseline)"}

    # ---------------------------------------------------------------- plain FP32 single stream
    one_len = 16384
    one = d_data[:one_len].clone()
    pl1, po1, ln1, _ = boa.encode_dev(m, one, [one_len], dtype="f32", ideal=False)
    ln1h = ln1.cpu().numpy().astype(np.uint32).astype(np.uint64)
    boa.decode_dev(m, pl1, po1, ln1h, data[:1], [one_len], dtype="f32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pl1, po1, ln1, _ = boa.encode_dev(m, one, [one_len], dtype="f32", ideal=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out1 = boa.decode_dev(m, pl1, po1, ln1h, data[:1], [one_len], dtype="f32")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    assert torch.equal(out1[:one_len], one)
    res["single_stream_fp32"] = {"encode_MBps": one_len / (t1 - t0) / 1e6, "decode_MBps": one_len / (t2 - t1) / 1e6,
                                 "round_trip_MBps": one_len / (t2 - t0) / 1e6,
                                 "sample": f"1 lane x {one_len // 1024} KiB (first chunk's prefix), FP32"}
    res["batched_vs_single_stream_fp32"] = res["value"] / res["single_stream_fp32"]["round_trip_MBps"]

    if not args.no_extras:
        # ------------------------------------------------------------ other dtypes on a subsample
        sub_len = 4096
        sub = np.concatenate([data[o:o + sub_len] for o in off])
        d_sub = torch.from_numpy(sub).cuda()
        sub_lens = np.full(n_chunks, sub_len, dtype=np.uint64)
        for dt_name in [x for x in ("f32", "fp8") if x != args.dtype]:
            tq = tune(m, d_sub, sub_lens, dtype=dt_name, use_cache=False, sample_bytes=2048,
                      use_table=not args.retune)
            kw = dict(use_graph=tq["use_graph"], decode_kernel=tq["decode_kernel"], fused_lanes=tq["fused_lanes"])
            for rep in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                pq, oq, lq, iq = boa.encode_dev(m, d_sub, sub_lens, dtype=dt_name, tile_t=tq["tile_t"], ideal=True)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                lqh = lq.cpu().numpy().astype(np.uint32).astype(np.uint64)
                t2 = time.perf_counter()
                outq = boa.decode_dev(m, pq, oq, lqh, sub[::sub_len], sub_lens, dtype=dt_name, **kw)
                torch.cuda.synchronize()
                t3 = time.perf_counter()
            res[f"{dt_name}_batched_subsample"] = {
                "value": sub.size / (t1 - t0 + t3 - t2) / 1e6, "encode_MBps": sub.size / (t1 - t0) / 1e6,
                "decode_MBps": sub.size / (t3 - t2) / 1e6,
                "coded_bits_per_byte": int(lqh.sum()) * 8 / (sub.size - n_chunks),
                "ideal_bits_per_byte": float(iq.cpu().numpy()[:n_chunks].sum()) / (sub.size - n_chunks),
                "round_trip_ok": bool(torch.equal(outq[:sub.size], d_sub)), "autotuned": tq,
                "sample": f"first {sub_len // 1024} KiB of every chunk ({sub.size / 2 ** 20:.0f} MiB)"}
        # ------------------------------------------------------------ integer-only pipeline, same subsample
        res["int8_pipeline_subsample"] = int_leg(m, sub, d_sub, sub_lens, sub_len, n_chunks)
        del d_sub
        # ------------------------------------------------------------ streaming compress
        st_bytes = data[:64 << 20].tobytes()
        t0 = time.perf_counter()
        shards = []
        with boa.StreamCompressor(m, chunk_len=65536, lanes=512, workers=2, dtype=args.dtype) as st:
            for i in range(0, len(st_bytes), 1 << 20):
                st.push(st_bytes[i:i + (1 << 20)])
                shards.extend(st.shards(wait=False))
            st.finish()
            shards.extend(st.shards(wait=True))
        t_st = time.perf_counter() - t0
        res["streaming_compress"] = {"MBps": len(st_bytes) / t_st / 1e6, "shards": len(shards),
                                     "compressed_bytes": sum(len(x) for x in shards),
                                     "sample": "first 64 MiB of the batch pushed in 1 MiB pieces, 512 x 64 KiB "
                                               "chunks per shard, 2 workers; host memory in and out, H2D/D2H and "
                                               "container assembly included"}
        # ------------------------------------------------------------ diagnostics
        d_pre = torch.from_numpy(np.stack([data[o:o + 4096] for o in off[:1024]])).cuda()
        boa.diagnostics(m, d_pre, dtype=args.dtype, n_bins=10)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dg = boa.diagnostics(m, d_pre, dtype=args.dtype, n_bins=10)
        res["diagnostics"] = {"positions": dg["positions"], "top1": dg["top1"], "top5": dg["top5"],
                              "top10": dg["top10"], "ece": dg["ece"], "bins": 10,
                              "ms": (time.perf_counter() - t0) * 1e3,
                              "sample": f"1024 chunks x first 4 KiB, {args.dtype}"}

    print(json.dumps(res), flush=True)
    if not ok:
        sys.exit(3)


if __name__ == "__main__":
    main()
