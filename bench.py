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

Prints one JSON line (see the design notes for the fields).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

D_MODEL, N_LAYERS, CHUNK, N_CHUNKS = 256, 3, 65536, 256
DATA_SEED, W_SEED = 1338, 4244


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--chunks", type=int, default=N_CHUNKS)
    ap.add_argument("--chunk-bytes", type=int, default=CHUNK)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path (asked for {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2511_11337_amd as boa
    from synth import ModelConfig, init_weights, records_f32_mix

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    cfg = ModelConfig(D_MODEL, N_LAYERS)
    n_chunks = args.chunks
    chunk = args.chunk_bytes
    total = chunk * n_chunks
    log("generating", total, "bytes")
    data = records_f32_mix(total, DATA_SEED)
    lens = np.full(n_chunks, chunk, dtype=np.uint64)
    w = init_weights(cfg, W_SEED)
    m = boa.Model(cfg, w)
    d_data = torch.from_numpy(data).cuda()
    stream = torch.cuda.current_stream()

    def one_step():
        payload, poff, plen, ib = boa.encode_dev(m, d_data, lens, dtype=args.dtype, ideal=False)
        plen_h = plen.cpu().numpy().astype(np.uint32).astype(np.uint64)
        out = boa.decode_dev(m, payload, poff, plen_h, data[::chunk], lens, dtype=args.dtype)
        return payload, poff, plen_h, out

    for i in range(args.warmup):
        log("warmup", i)
        payload, poff, plen_h, out = one_step()
    torch.cuda.synchronize()
    t_enc = t_dec = 0.0
    for i in range(args.steps):
        log("step", i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        payload, poff, plen, ib = boa.encode_dev(m, d_data, lens, dtype=args.dtype, ideal=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plen_h = plen.cpu().numpy().astype(np.uint32).astype(np.uint64)
        t2 = time.perf_counter()
        out = boa.decode_dev(m, payload, poff, plen_h, data[::chunk], lens, dtype=args.dtype)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        t_enc += t1 - t0
        t_dec += t3 - t2
    ok = bool(torch.equal(out[:total], d_data))
    comp = int(plen_h.sum()) + n_chunks * 33 + 64
    ms_step = (t_enc + t_dec) / args.steps * 1e3
    enc_mbps = total * args.steps / t_enc / 1e6
    dec_mbps = total * args.steps / t_dec / 1e6
    res = {
        "metric": "encode/decode MB/s on 1 GPU at fixed bits/byte; batched BF16 vs plain FP32",
        "value": total / (ms_step / 1e3) / 1e6,
        "unit": "MB/s (1e6 uncompressed bytes/s, encode+decode round trip)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"{n_chunks} x {chunk // 1024} KiB chunks of 20-byte f32/i32 records, "
                               f"byte Mamba d_model {D_MODEL} x {N_LAYERS} layers",
                   "chunks": n_chunks, "chunk_bytes": chunk, "d_model": D_MODEL, "n_layers": N_LAYERS},
        "encode_MBps": enc_mbps, "decode_MBps": dec_mbps,
        "bits_per_byte": comp * 8 / total, "round_trip_ok": ok,
    }
    print(json.dumps(res), flush=True)
    if not ok:
        sys.exit(3)


if __name__ == "__main__":
    main()
