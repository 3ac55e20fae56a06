"""The learned part's training recipe on one GPU, and its held-out judge.

    python -m paper_2511_11337_amd.recipe --out model.boam [--steps 2560] [--resume ckpt.boat]

Trains the d_model 256 x 3 layer predictor from its seeded initial weights on
64 MiB of the 20-byte record stream with the library's own forward and
backward kernels: AdamW at lr 1e-3 (betas 0.9 / 0.999, eps 1e-8, weight decay
0.01, 100-step linear warm-up, global-norm clipping at 1.0), batch 32
windows of 8192 bytes, BF16 projection operands with FP32 master weights
(paper, Models: cross-entropy training with sequence length, batch and
learning rate as the tunable choices).  Ten epochs over the 8192 windows are
2560 steps; the windows are shuffled every epoch by the library (seed 1340).
The 64 MiB are 512 independent record streams of 128 KiB, each with its own
run-number range (one long stream would let the model memorise a single
range).  A checkpoint with the AdamW moments is written every --ckpt-every
steps, and --resume continues from one exactly.

At the end the held-out judge runs: 16 MiB of records (seed 7331) as 256 x 64
KiB chunks, coded bits/byte of the trained model (FP32 and BF16), of the
starting model (seed-initialised, or --init) and of the adaptive order-2
model, against 8 for raw bytes.

--data records64 --init MODEL fine-tunes a trained model on 64 MiB of the
64-byte structured records with the same recipe (the precision-plus-batching
workload runs the 20-byte-record model on 64-byte records, which it has never
seen; fine-tuning on that stream is the reading taken for it).  There every
8 KiB window is a stream of its own, so the network cannot memorise a
stream's counters and base values and has to read them from the context.

--data mixed trains on the mixed stream of the FP8 workload: every 8 KiB
window is one stream, its type (20-byte records, 64-byte records, raw
float32 N(0, 1)) taking turns; with --d-model 512 --n-layers 4 --w-seed 4247
--steps 300 it is the brief training the FP8 workload's model gets.  Its
held-out judge is 16 MiB of mixed 64 KiB chunks, reported per stream type.
Everything runs in the library; this module only drives it and writes the
model file and a JSON log.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

D_MODEL, N_LAYERS, W_SEED = 256, 3, 4245
DATA_SEED, DATA_SEED64, DATA_SEED_MIX, HELD_SEED = 1340, 1344, 1345, 7331
TRAIN_BYTES, STREAM_BYTES, SEQ, BATCH = 64 << 20, 128 << 10, 8192, 32


def training_bytes(kind: str = "records20", total: int = TRAIN_BYTES, per_stream: int = STREAM_BYTES) -> np.ndarray:
    """Independent record streams of per_stream bytes: the 20-byte physics
    records, or the 64-byte structured records (each stream its own event
    range, base kinematics and timestamps), or the mixed stream (one 8 KiB
    window per stream, the three types in turn)."""
    from synth import records_f32_mix, records_structured64, mixed_chunks
    if kind == "mixed":
        return np.concatenate([c for _, c in mixed_chunks(np.full(total // SEQ, SEQ), DATA_SEED_MIX)])
    gen, seed = (records_f32_mix, DATA_SEED) if kind == "records20" else (records_structured64, DATA_SEED64)
    if kind == "records64":
        per_stream = SEQ          # every window its own stream: its bases and counters are seen once
    n = total // per_stream
    return np.concatenate([gen(per_stream, seed * 100003 + k) for k in range(n)])


def held_out(kind: str = "records20", nbytes: int = 16 << 20) -> np.ndarray:
    from synth import records_f32_mix, records_structured64, mixed_chunks
    if kind == "records20":
        return records_f32_mix(nbytes, HELD_SEED)
    if kind == "mixed":
        return np.concatenate([c for _, c in mixed_chunks(np.full(nbytes // 65536, 65536), HELD_SEED)])
    return np.concatenate([records_structured64(65536, HELD_SEED * 1000003 + i) for i in range(nbytes // 65536)])


def bits_per_byte_by_type(model, data: np.ndarray, chunk: int = 65536, dtype="f32") -> dict:
    """Coded bits/byte of the mixed held-out stream per stream type (chunk
    index mod 3: 20-byte records, 64-byte records, raw float32)."""
    import torch
    import paper_2511_11337_amd as boa
    lens = boa._chunk_lens(data.size, chunk_len=chunk)
    _, _, _, ib = boa.encode_dev(model, torch.from_numpy(data).cuda(), lens, dtype=dtype)
    ib = ib.cpu().numpy()[:lens.size]
    out = {}
    for t, name in enumerate(("records20", "records64", "raw_f32")):
        sel = np.arange(lens.size) % 3 == t
        out[name] = float(ib[sel].sum()) / float((lens[sel] - 1).sum())
    return out


def bits_per_byte(model, data: np.ndarray, chunk: int = 65536, dtype="f32") -> float:
    """Sum of -log2 f(s)/M over the coded bytes of every chunk (the integer
    tables the coder uses), per coded byte."""
    import torch
    import paper_2511_11337_amd as boa
    lens = boa._chunk_lens(data.size, chunk_len=chunk)
    d = torch.from_numpy(data).cuda()
    _, _, _, ib = boa.encode_dev(model, d, lens, dtype=dtype)
    return float(ib.cpu().numpy()[:lens.size].sum()) / (data.size - lens.size)


def order2_bits_per_byte(data: np.ndarray, chunk: int = 65536) -> float:
    import torch
    import paper_2511_11337_amd as boa
    lens = boa._chunk_lens(data.size, chunk_len=chunk)
    _, _, _, ib = boa.order2_encode(torch.from_numpy(data).cuda(), lens)
    return float(ib.cpu().numpy()[:lens.size].sum()) / (data.size - lens.size)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True, help="model file to write (BOAM)")
    ap.add_argument("--steps", type=int, default=2560, help="total optimiser steps (the recipe: 2560)")
    ap.add_argument("--resume", default=None, help="training checkpoint (BOAT) to continue from")
    ap.add_argument("--ckpt", default=None, help="checkpoint path written every --ckpt-every steps and at the end")
    ap.add_argument("--ckpt-every", type=int, default=500)
    ap.add_argument("--stop-after", type=int, default=0, help="stop this run after so many steps (0 = run to --steps)")
    ap.add_argument("--dtype", default="bf16", choices=["f32", "bf16"])
    ap.add_argument("--data", default="records20", choices=["records20", "records64", "mixed"],
                    help="training stream: 20-byte physics records (the recipe), 64-byte structured records, "
                         "or the mixed stream")
    ap.add_argument("--d-model", type=int, default=D_MODEL)
    ap.add_argument("--n-layers", type=int, default=N_LAYERS)
    ap.add_argument("--w-seed", type=int, default=W_SEED, help="seed of the initial weights")
    ap.add_argument("--init", default=None, help="model file to start from (fine-tuning); default: seeded init")
    ap.add_argument("--log", default=None, help="JSON log to write")
    ap.add_argument("--no-judge", action="store_true")
    args = ap.parse_args(argv)

    import torch
    import paper_2511_11337_amd as boa
    import paper_2511_11337_amd.train as tr
    from synth import ModelConfig, init_weights

    cfg = ModelConfig(args.d_model, args.n_layers)
    m = boa.Model.load(args.init) if args.init else boa.Model(cfg, init_weights(cfg, args.w_seed))
    cfg = m.cfg
    start_model = m.get_weights()
    if args.resume:
        tr.load_state(m, args.resume)
    start = tr.steps_done(m)
    t0 = time.perf_counter()
    data = training_bytes(args.data)
    end = args.steps if not args.stop_after else min(args.steps, start + args.stop_after)
    print(f"[recipe] {data.size} training bytes, windows of {SEQ}, batch {BATCH}, steps {start}..{end} of "
          f"{args.steps}", flush=True)
    # the library's train(model, bytes) in slices of 50 steps: it continues the
    # seeded window order from the model's own step count, so the slices (and
    # a resumed run) equal one uninterrupted call
    losses = []
    t_train = time.perf_counter()
    step = start
    while step < end:
        n = min(50, end - step)
        o = tr.opts(lr=1e-3, warmup=100, steps=n, batch=BATCH, seq_len=SEQ, chunk_t=256, dtype=args.dtype,
                    seed=DATA_SEED)
        losses.extend(tr.train(m, data, o).tolist())
        step += n
        print(f"[recipe] step {step}: loss {np.mean(losses[-n:]) / np.log(2):.4f} bits/byte, "
              f"{time.perf_counter() - t_train:.0f} s", flush=True)
        if args.ckpt and (step % args.ckpt_every == 0 or step == end):
            tr.save_state(m, args.ckpt)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t_train
    n_steps = end - start
    log = {"steps_done": end, "steps_this_run": n_steps, "dtype": args.dtype,
           "tokens_per_s": n_steps * BATCH * (SEQ - 1) / dt if n_steps else None,
           "ms_per_step": dt / n_steps * 1e3 if n_steps else None,
           "loss_bits_per_byte_every_50": [float(np.mean(losses[i:i + 50]) / np.log(2))
                                           for i in range(0, len(losses), 50)]}
    if end == args.steps:
        m.save(args.out)
        print(f"[recipe] wrote {args.out}", flush=True)
        if not args.no_judge:
            held = held_out(args.data)
            log["held_out_bits_per_byte"] = {
                "trained_f32": bits_per_byte(m, held, dtype="f32"),
                "trained_bf16": bits_per_byte(m, held, dtype="bf16"),
                ("start_model" if args.init else "seed_init"): bits_per_byte(boa.Model(cfg, start_model), held),
                "order2": order2_bits_per_byte(held), "raw": 8.0,
                "sample": f"16 MiB of {args.data} (seed {HELD_SEED}) as 256 x 64 KiB chunks"}
            if args.data == "mixed":
                log["held_out_bits_per_byte"]["by_type"] = {
                    dt: bits_per_byte_by_type(m, held, dtype=dt) for dt in ("f32", "bf16", "fp8")}
            print("[recipe] held-out bits/byte", log["held_out_bits_per_byte"], flush=True)
    log["wall_s"] = time.perf_counter() - t0
    if args.log:
        with open(args.log, "w") as fh:
            json.dump(log, fh, indent=1)
    return log


if __name__ == "__main__":
    main()
