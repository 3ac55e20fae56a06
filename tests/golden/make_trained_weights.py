"""Writes cfg2_oracle_trained_f16.npy: a d_model 256 x 3 layer predictor trained
by the FP64 oracle alone (oracle.grad: hand-written reverse mode and AdamW),
so that precision tests compare the GPU with the oracle on a model whose
predictions are sharp (about 5 bits/byte on the record streams) instead of
near uniform.  Nothing here runs the GPU library.

Recipe: seed-init weights (seed 4244), 60 AdamW steps (lr 3e-3, linear
warm-up over 10 steps, weight decay 0.01, global-norm clipping at 1.0) on
batches of 4 sequences of 512 bytes, alternating the 20-byte record stream
and the 64-byte structured record stream (fresh seeds every step).  The
weights are stored rounded to float16; the tests load them as float32, so
both sides read the same values.

    python tests/golden/make_trained_weights.py      (about 4 minutes on 8 cores)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from synth import ModelConfig, init_weights, records_f32_mix, records_structured64  # noqa: E402
from oracle import grad as og  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg2_oracle_trained_f16.npy")


def main():
    cfg = ModelConfig(256, 3)
    w = init_weights(cfg, 4244).astype(np.float64)
    opt = og.AdamW(w.size, lr=3e-3)
    B, T, steps = 4, 512, 60
    for s in range(steps):
        seqs = np.stack([records_f32_mix(T, 10000 + s * B + b) if b % 2 == 0 else
                         records_structured64(T, 20000 + s * B + b) for b in range(B)])
        loss, g = og.loss_and_grad(cfg, w, seqs)
        g, _ = og.clip_global_norm(g, 1.0)
        w = opt.step(w, g, opt.lr * min(1.0, (s + 1) / 10))
        print(f"step {s}: {loss / np.log(2):.3f} bits/byte", flush=True)
    np.save(OUT, w.astype(np.float16))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
