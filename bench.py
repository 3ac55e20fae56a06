#!/usr/bin/env python3
"""Benchmark of the BOA Constrictor hot path on one MI355X.

Workload: 16 MiB of synthetic 20-byte physics records (float32 pT ~ Exp(20),
eta, phi, int32 nHits ~ Poisson(12), run number) split into 256 independent
64 KiB chunks; byte-level Mamba with d_model 256, 3 layers, d_state 16,
d_conv 4, expand 2 (1,446,656 parameters), seed-initialised float32 weights.

One step = the whole hot path over that batch with inputs already resident in
HBM: encode all 256 chunks (model forward over every position, histograms,
range coding) and decode them again step by step (model step, histogram,
range decoding, feedback of the decoded byte).  The round trip is checked for
byte identity outside the timed region.

The headline run uses BF16 projections (FP32 accumulation, FP32 scan and
softmax, integer CDF); the same batch with FP32 and with FP8 (E4M3)
projections, and one FP32 stream on its own, are reported beside it.  Launch shapes (encoder tile,
decoder kernel and lanes per workgroup) come from the autotuner.

After the timed steps a kernel-timing pass times every launch with GPU
start/stop timestamps: the encoder's kernel classes on the first 4 KiB of
every chunk (same lanes and tile, scaled to the full run), the fused decoder
on the full batch; the class with the largest share of GPU time is the
dominant kernel of the roofline object.  The CPU baseline is the FP64 oracle
on a bounded sample of the same stream.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

D_MODEL, N_LAYERS, CHUNK, N_CHUNKS = 256, 3, 65536, 256
DATA_SEED, W_SEED = 1338, 4244
PEAK = {"f32": {"mfma": 157.3, "alu": 157.3}, "bf16": {"mfma": 2500.0, "alu": 157.3},
        "fp8": {"mfma": 5000.0, "alu": 157.3}}
HBM_PEAK = 8000.0   # GB/s
KIND_NAMES = ["embed", "in_proj", "mixer", "out_proj", "head", "decode", "quant", "encode", "fused_decoder"]
K_COUNT = len(KIND_NAMES)
K_FUSED = 8


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def flops_per_row() -> float:
    """Model flops of one position: projections on MFMA plus the mixer's
    elementwise work (conv 8 Di, x_proj, dt_proj, scan 6 Di N, gate 4 Di)."""
    D, Di, N, R = D_MODEL, 2 * D_MODEL, 16, (D_MODEL + 15) // 16
    per_layer = 2.0 * 2 * Di * D + 2.0 * D * Di + 8.0 * Di + 2.0 * (R + 2 * N) * Di + 2.0 * R * Di + 6.0 * Di * N + 4.0 * Di
    return N_LAYERS * per_layer + 2.0 * 256 * D


def algorithmic(kind: int, rows: int, dtype: str):
    """(bound, flops or bytes per launch, unit) for a kernel class over `rows` rows."""
    D, Di, N, R = D_MODEL, 2 * D_MODEL, 16, (D_MODEL + 15) // 16
    if kind == K_FUSED:
        # the whole model at every decoded position; the projections dominate
        return "mfma", rows * flops_per_row(), "TFLOP/s"
    if kind == 1:
        return "mfma", 2.0 * rows * 2 * Di * D, "TFLOP/s"
    if kind == 3:
        return "mfma", 2.0 * rows * D * Di, "TFLOP/s"
    if kind == 4:
        return "mfma", 2.0 * rows * 256 * D, "TFLOP/s"
    if kind == 2:
        # conv 2*4*Di, x_proj 2*(R+2N)*Di, dt_proj 2*R*Di, scan 6*Di*N, gate 4*Di
        return "alu", rows * (8.0 * Di + 2.0 * (R + 2 * N) * Di + 2.0 * R * Di + 6.0 * Di * N + 4.0 * Di), "TFLOP/s"
    # coder / histogram / gather kernels: bytes they must move (logits in, bytes out)
    return "hbm", rows * (256 * 4.0 + 8.0), "GB/s"


# Per-CU rate at which one workgroup streams L2-resident data to registers
# with every CU streaming (measured with a plain streaming kernel: 256
# workgroups of 512 threads, 16 B loads, about 113 GB/s each)
CU_STREAM_PEAK = 113.0


def weight_bytes_per_step(dtype: str) -> float:
    """Bytes of weights one decoding step reads: in_proj, out_proj and head in
    the projection dtype; x_proj and dt_proj in bf16 (BF16 mode) or f32; conv,
    A, D, biases and LayerNorm parameters in f32."""
    D, Di, N, R = D_MODEL, 2 * D_MODEL, 16, (D_MODEL + 15) // 16
    pb = {"f32": 4, "bf16": 2, "fp8": 1}[dtype]
    xb = 2 if dtype == "bf16" else 4
    per_layer = pb * (2 * Di * D + D * Di) + xb * ((R + 2 * N) * Di + R * Di) + 4 * (5 * Di + N * Di + 3 * Di + 2 * D)
    return N_LAYERS * per_layer + pb * 256 * D + 4 * (256 + 2 * D + D)


def traffic_record(kind: int, dtype: str):
    """HBM bytes per launch of the fused decoder from the committed counter
    record (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the kernel
    is not the one that was counted."""
    if kind != K_FUSED or dtype != "bf16":
        return None
    path = os.path.join(ROOT, "profiles", "traffic_k_dec_fused_bf16_256x64KiB.json")
    if not os.path.exists(path):
        return None
    from paper_2511_11337_amd.counters import source_hash
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha256") != source_hash():
        return None
    return rec["hbm_bytes_per_launch"]


def cpu_baseline(data: np.ndarray, lanes: int = 8, nbytes: int = 4096):
    """FP64 oracle compress + decompress of `lanes` chunks of `nbytes` bytes."""
    from synth import ModelConfig, init_weights
    from oracle import model as om, coder as oc
    cfg = ModelConfig(D_MODEL, N_LAYERS)
    W = om.Weights(cfg, init_weights(cfg, W_SEED))
    chunks = np.stack([data[i * CHUNK:i * CHUNK + nbytes] for i in range(lanes)])
    t0 = time.perf_counter()
    S = om.StreamState(cfg, lanes)
    encs = [oc.Encoder() for _ in range(lanes)]
    for t in range(nbytes - 1):
        p = om.softmax(om.step(W, S, chunks[:, t]))
        for b in range(lanes):
            f = oc.quantise(p[b])
            c = oc.cdf(f)
            s = int(chunks[b, t + 1])
            encs[b].encode(int(c[s]), int(f[s]))
    payloads = [e.finish() for e in encs]
    S = om.StreamState(cfg, lanes)
    decs = [oc.Decoder(pl) for pl in payloads]
    out = np.zeros_like(chunks)
    out[:, 0] = chunks[:, 0]
    for t in range(nbytes - 1):
        p = om.softmax(om.step(W, S, out[:, t]))
        for b in range(lanes):
            out[b, t + 1] = decs[b].decode(oc.cdf(oc.quantise(p[b])))
    dt = time.perf_counter() - t0
    assert np.array_equal(out, chunks)
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        cores = 1
    return {"value": lanes * nbytes / dt / 1e6, "unit": "MB/s (encode+decode round trip)", "cores": int(cores),
            "kind": "oracle",
            "sample": f"{lanes} chunks x {nbytes} B of the same record stream, FP64 NumPy model step + "
                      f"Python-integer range coder, compress and decompress ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", default="bf16", choices=["f32", "bf16", "fp8"],
                    help="projection dtype of the batched run (the metric's target is batched BF16)")
    ap.add_argument("--no-fp32-batched", action="store_true", help="skip the FP32 batched comparison run")
    ap.add_argument("--no-fp8-batched", action="store_true", help="skip the FP8 batched comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--chunks", type=int, default=N_CHUNKS)
    ap.add_argument("--chunk-bytes", type=int, default=CHUNK)
    ap.add_argument("--fixed-shape", action="store_true",
                    help="skip the autotuner: encoder tile 512, fused decoder with one lane per workgroup "
                         "(the shape the autotuner picks for this batch); for hardware-counter runs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first launch a plain 256 MiB copy (read + write) for hardware-counter scaling")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path (asked for {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2511_11337_amd as boa
    from paper_2511_11337_amd import _lib
    from synth import ModelConfig, init_weights, records_f32_mix

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        # the run's first dispatch: reads and writes 256 MiB (counter scale)
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 256 MiB read, 256 MiB written")
    cfg = ModelConfig(D_MODEL, N_LAYERS)
    n_chunks, chunk = args.chunks, args.chunk_bytes
    total = chunk * n_chunks
    log("generating", total, "bytes")
    data = records_f32_mix(total, DATA_SEED)
    lens = np.full(n_chunks, chunk, dtype=np.uint64)
    m = boa.Model(cfg, init_weights(cfg, W_SEED))
    d_data = torch.from_numpy(data).cuda()
    firsts = data[::chunk].copy()

    from paper_2511_11337_amd.autotune import tune
    if args.fixed_shape:
        tuned = {"tile_t": 512, "decode_kernel": "fused", "fused_lanes": 1, "use_graph": False}
    else:
        tuned = tune(m, d_data, lens, dtype=args.dtype, use_cache=False)
    log("autotuned" if not args.fixed_shape else "fixed shape", tuned)

    def dec_opts(t):
        return dict(use_graph=t["use_graph"], decode_kernel=t["decode_kernel"], fused_lanes=t["fused_lanes"])

    def enc():
        return boa.encode_dev(m, d_data, lens, dtype=args.dtype, tile_t=tuned["tile_t"], ideal=True)

    def dec(payload, poff, plen_h):
        return boa.decode_dev(m, payload, poff, plen_h, firsts, lens, dtype=args.dtype, **dec_opts(tuned))

    for i in range(args.warmup):
        log("warmup", i)
        payload, poff, plen, ib = enc()
        dec(payload, poff, plen.cpu().numpy().astype(np.uint32).astype(np.uint64))
    torch.cuda.synchronize()
    t_enc = t_dec = 0.0
    for i in range(args.steps):
        log("step", i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        payload, poff, plen, ib = enc()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plen_h = plen.cpu().numpy().astype(np.uint32).astype(np.uint64)
        t2 = time.perf_counter()
        out = dec(payload, poff, plen_h)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        t_enc += t1 - t0
        t_dec += t3 - t2
        log(f"step {i}: encode {t1 - t0:.3f} s, decode {t3 - t2:.3f} s")
    ok = bool(torch.equal(out[:total], d_data))
    coded = int(plen_h.sum())
    ideal = float(ib.cpu().numpy()[:n_chunks].sum())
    ms_step = (t_enc + t_dec) / args.steps * 1e3
    res = {
        "metric": "encode/decode MB/s on 1 GPU at fixed bits/byte; batched BF16 vs plain FP32",
        "value": total / (ms_step / 1e3) / 1e6,
        "unit": "MB/s (1e6 uncompressed bytes/s, encode+decode round trip)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"{n_chunks} x {chunk // 1024} KiB chunks of 20-byte f32/i32 records, "
                               f"byte Mamba d_model {D_MODEL} x {N_LAYERS} layers, seed-init weights",
                   "chunks": n_chunks, "chunk_bytes": chunk, "lanes": n_chunks, "projections": args.dtype},
        "encode_MBps": total * args.steps / t_enc / 1e6,
        "decode_MBps": total * args.steps / t_dec / 1e6,
        "coded_bits_per_byte": coded * 8 / (total - n_chunks),
        "ideal_bits_per_byte": ideal / (total - n_chunks),
        "round_trip_ok": ok,
        "autotuned": tuned,
    }

    def batched(dt):
        """The same batch in another projection dtype: autotuned, one warm-up
        encode + decode, then one timed."""
        tdt = tune(m, d_data, lens, dtype=dt, use_cache=False)
        log(f"{dt} batched, autotuned", tdt)
        tt = []
        for i in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pq, oq, lq, iq = boa.encode_dev(m, d_data, lens, dtype=dt, tile_t=tdt["tile_t"], ideal=True)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            lqh = lq.cpu().numpy().astype(np.uint32).astype(np.uint64)
            t2 = time.perf_counter()
            outq = boa.decode_dev(m, pq, oq, lqh, firsts, lens, dtype=dt, **dec_opts(tdt))
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            tt.append((t1 - t0, t3 - t2))
        te, td = tt[-1]
        return {"value": total / (te + td) / 1e6, "encode_MBps": total / te / 1e6, "decode_MBps": total / td / 1e6,
                "coded_bits_per_byte": int(lqh.sum()) * 8 / (total - n_chunks),
                "ideal_bits_per_byte": float(iq.cpu().numpy()[:n_chunks].sum()) / (total - n_chunks),
                "round_trip_ok": bool(torch.equal(outq[:total], d_data)), "autotuned": tdt}

    if not args.no_fp32_batched and args.dtype != "f32":
        res["fp32_batched"] = batched("f32")
    if not args.no_fp8_batched and args.dtype != "fp8":
        res["fp8_batched"] = batched("fp8")

    # the plain comparator: the same kernels with one stream (one lane), FP32, on a 4 KiB chunk
    one = torch.from_numpy(data[:4096].copy()).cuda()
    pl1, po1, ln1, _ = boa.encode_dev(m, one, [4096], dtype="f32", ideal=False)
    ln1h = ln1.cpu().numpy().astype(np.uint32).astype(np.uint64)
    boa.decode_dev(m, pl1, po1, ln1h, data[:1], [4096], dtype="f32")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pl1, po1, ln1, _ = boa.encode_dev(m, one, [4096], dtype="f32", ideal=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out1 = boa.decode_dev(m, pl1, po1, ln1h, data[:1], [4096], dtype="f32")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    assert torch.equal(out1[:4096], one)
    res["single_stream_fp32"] = {"encode_MBps": 4096 / (t1 - t0) / 1e6, "decode_MBps": 4096 / (t2 - t1) / 1e6,
                                 "round_trip_MBps": 4096 / (t2 - t0) / 1e6, "sample": "1 lane x 4 KiB"}

    if not args.no_kernel_timing:
        # Encoder: same launch shapes on the first 4 KiB of every chunk, every
        # launch timed with GPU start/stop timestamps, scaled to the full run.
        # Decoder: the fused kernel is timed on the full batch (one launch);
        # the per-step kernels, when chosen, on the 4 KiB prefixes.
        sub = min(4096, chunk)
        sub_data = np.concatenate([data[i * chunk:i * chunk + sub] for i in range(n_chunks)])
        d_sub = torch.from_numpy(sub_data).cuda()
        sub_lens = np.full(n_chunks, sub, dtype=np.uint64)
        lib = _lib.load()
        lib.boa_prof_read(None, None, 1)
        lib.boa_prof_enable((1 << K_COUNT) - 1)
        boa.encode_dev(m, d_sub, sub_lens, dtype=args.dtype, tile_t=tuned["tile_t"], ideal=False)
        enc_ms = np.zeros(K_COUNT)
        enc_n = np.zeros(K_COUNT, dtype=np.uint64)
        lib.boa_prof_read(enc_ms.ctypes.data, enc_n.ctypes.data, 1)
        fused = tuned["decode_kernel"] == "fused"
        if fused:
            boa.decode_dev(m, payload, poff, plen_h, firsts, lens, dtype=args.dtype, **dec_opts(tuned))
            dec_scale = 1.0
        else:
            pl_s, po_s, ln_s, _ = boa.encode_dev(m, d_sub, sub_lens, dtype=args.dtype, ideal=False)
            lib.boa_prof_read(None, None, 1)
            boa.decode_dev(m, pl_s, po_s, ln_s.cpu().numpy().astype(np.uint32).astype(np.uint64),
                           sub_data[::sub], sub_lens, dtype=args.dtype, use_graph=False, decode_kernel="steps")
            dec_scale = (chunk - 1) / max(sub - 1, 1)
        dec_ms = np.zeros(K_COUNT)
        dec_n = np.zeros(K_COUNT, dtype=np.uint64)
        lib.boa_prof_read(dec_ms.ctypes.data, dec_n.ctypes.data, 1)
        lib.boa_prof_enable(0)
        steps_full = chunk - 1
        enc_tiles_sub = max(int(enc_n[1]) // N_LAYERS, 1)
        T_enc = (sub - 1 + enc_tiles_sub - 1) // enc_tiles_sub
        share = {}
        for k in range(K_COUNT):
            if dec_n[k]:
                share[("decode", k)] = dec_ms[k] * dec_scale
            if enc_n[k]:
                share[("encode", k)] = enc_ms[k] / max(sub - 1, 1) * steps_full
        (phase, kind), _ = max(share.items(), key=lambda kv: kv[1])
        ms_tab = dec_ms if phase == "decode" else enc_ms
        n_tab = dec_n if phase == "decode" else enc_n
        avg_s = ms_tab[kind] / n_tab[kind] / 1e3
        if kind == K_FUSED:
            rows = n_chunks * (chunk - 1)              # positions decoded by the one launch
        else:
            rows = n_chunks if phase == "decode" else n_chunks * T_enc
        bound, work, unit = algorithmic(kind, rows, args.dtype)
        if unit == "TFLOP/s":
            achieved = work / avg_s / 1e12
            peak = PEAK[args.dtype][bound]
        else:
            achieved = work / avg_s / 1e9
            peak = HBM_PEAK
        res["roofline"] = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                           "frac": achieved / peak, "traffic": traffic_record(kind, args.dtype),
                           "kernel": f"{phase} {KIND_NAMES[kind]}", "rows_per_launch": rows,
                           "avg_launch_us": avg_s * 1e6,
                           "work_per_launch": work}
        if kind == K_FUSED:
            # what bounds the fused decoder: every workgroup streams all weights
            # from L2 each step (one lane per workgroup at this batch)
            wb = weight_bytes_per_step(args.dtype)
            steps = chunk - 1
            res["roofline"]["weight_stream"] = {
                "bytes_per_step_per_workgroup": wb, "steps": steps,
                "achieved_GBps_per_CU": wb * steps / avg_s / 1e9,
                "measured_peak_GBps_per_CU": CU_STREAM_PEAK,
                "frac": wb * steps / avg_s / 1e9 / CU_STREAM_PEAK}
        res["kernel_time_us"] = {f"{ph}:{KIND_NAMES[k]}": round(float(ms_tab_k) * 1e3 / max(int(n_k), 1), 2)
                                 for ph, tab, ntab in (("encode", enc_ms, enc_n), ("decode", dec_ms, dec_n))
                                 for k, (ms_tab_k, n_k) in enumerate(zip(tab, ntab)) if n_k}

    # streaming compress (host bytes in, shards out): the batch pushed in
    # 1 MiB pieces, groups of 128 chunks, 2 workers; beside it the one-shot
    # host-level compress of the same bytes (both include the copies to and
    # from the GPU and the container assembly)
    hb = data.tobytes()
    boa.compress(m, hb[:4 * chunk], chunk_len=chunk, dtype=args.dtype)
    t0 = time.perf_counter()
    one = boa.compress(m, hb, chunk_len=chunk, dtype=args.dtype, tile_t=tuned["tile_t"])
    t_one = time.perf_counter() - t0
    t0 = time.perf_counter()
    shards = []
    with boa.StreamCompressor(m, chunk_len=chunk, lanes=128, workers=2, dtype=args.dtype, tile_t=tuned["tile_t"]) as st:
        for i in range(0, len(hb), 1 << 20):
            st.push(hb[i:i + (1 << 20)])
            shards.extend(st.shards(wait=False))
        st.finish()
        shards.extend(st.shards(wait=True))
    t_st = time.perf_counter() - t0
    res["streaming_compress"] = {"MBps": total / t_st / 1e6, "one_shot_host_MBps": total / t_one / 1e6,
                                 "shards": len(shards), "compressed_bytes": sum(len(x) for x in shards),
                                 "one_shot_bytes": len(one),
                                 "sample": "16 MiB pushed in 1 MiB pieces, 128 x 64 KiB chunks per shard, 2 workers; "
                                           "host memory in and out, H2D/D2H and container assembly included"}

    # predictor diagnostics (confusion, Top-k, reliability / ECE) of the
    # headline dtype on the first 4 KiB of every chunk
    sub = min(4096, chunk)
    d_pre = torch.from_numpy(np.stack([data[i * chunk:i * chunk + sub] for i in range(n_chunks)])).cuda()
    boa.diagnostics(m, d_pre, dtype=args.dtype, n_bins=10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dg = boa.diagnostics(m, d_pre, dtype=args.dtype, n_bins=10)
    t_dg = time.perf_counter() - t0
    res["diagnostics"] = {"positions": dg["positions"], "top1": dg["top1"], "top5": dg["top5"],
                          "top10": dg["top10"], "ece": dg["ece"], "bins": 10, "ms": t_dg * 1e3,
                          "sample": f"{n_chunks} chunks x {sub} B prefixes, {args.dtype}"}

    if not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle)")
        res["cpu_baseline"] = cpu_baseline(data)
    print(json.dumps(res), flush=True)
    if not ok:
        sys.exit(3)


if __name__ == "__main__":
    main()
