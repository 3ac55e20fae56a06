"""GPU training path against the FP64 oracle, through the C ABI.

* the hand-written selective-scan backward (behind torch.autograd.Function)
  matches the oracle's reverse recurrence element by element, with several
  chunk lengths;
* the whole-model loss and gradient match the oracle's hand-written FP64
  gradient (itself pinned by finite differences and autograd) element by
  element, with FP32 projections; with BF16 projection operands within the
  error that bf16 operand rounding allows;
* AdamW (clipping, decoupled decay, bias correction) applied to a seeded
  gradient matches the oracle's AdamW after several steps;
* training is deterministic (two runs give identical weights) and a training
  checkpoint resumes exactly;
* a trained network beats both the adaptive order-2 model and the untrained
  network on held-out bits/byte (learned gain; parity unpinned in absolute
  terms: the paper reports no synthetic-data numbers).
"""
import os

import numpy as np
import pytest
import torch

from synth import ModelConfig, init_weights, records_f32_mix, records_structured64
from synth.weights import param_layout
from oracle.grad import loss_and_grad as oracle_loss_grad, scan_forward, scan_backward, AdamW, clip_global_norm

pytestmark = pytest.mark.gpu


def boa():
    import paper_2511_11337_amd as b
    return b


def tr():
    import paper_2511_11337_amd.train as t
    return t


def assert_close(got, ref, rtol, atol_frac, what=""):
    """Element-wise |got - ref| <= atol + rtol |ref| with atol = atol_frac * max |ref|
    (the scale of the tensor: elements that cancel to near zero are held to the
    tensor's own magnitude, not to their own)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    atol = atol_frac * max(float(np.abs(ref).max()), 1e-30)
    err = np.abs(got - ref)
    bad = err > atol + rtol * np.abs(ref)
    assert not bad.any(), (what, int(bad.sum()), float(err.max()), atol)


@pytest.mark.parametrize("chunk_t", [1, 5, 64])
def test_scan_autograd_matches_oracle(chunk_t):
    print(f"[gpu] scan autograd chunk_t={chunk_t}", flush=True)
    rng = np.random.default_rng(chunk_t)
    Bt, T, Di, N = 2, 37, 300, 16          # Di spans two 256-channel workgroups with a ragged tail
    x = rng.normal(size=(Bt, T, Di))
    dt = np.exp(rng.normal(-1.5, 0.5, (Bt, T, Di)))
    A_log = rng.normal(0, 0.5, (Di, N))
    Bm, Cm = rng.normal(size=(Bt, T, N)), rng.normal(size=(Bt, T, N))
    Dv = rng.normal(size=Di)
    dy = rng.normal(size=(Bt, T, Di))
    A = -np.exp(A_log)
    y_ref, saved = scan_forward(x, dt, A, Bm, Cm, Dv, save_every=chunk_t)
    gx, gdt, gA, gB, gC, gD = scan_backward(dy, x, dt, A, Bm, Cm, Dv, saved, chunk_t)
    cu = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda", requires_grad=True)
    tx, tdt, tA, tB, tC, tD = (cu(v) for v in (x, dt, A_log, Bm, Cm, Dv))
    y = tr().selective_scan(tx, tdt, tA, tB, tC, tD, chunk_t=chunk_t)
    y.backward(torch.tensor(dy, dtype=torch.float32, device="cuda"))

    def close(a, b, what):
        assert_close(a.detach().cpu().numpy(), b, 1e-4, 1e-5, what)

    close(y, y_ref, "y")
    close(tx.grad, gx, "dx")
    close(tdt.grad, gdt, "ddt")
    close(tA.grad, gA * A, "dA_log")          # gradient with respect to A_log
    close(tB.grad, gB, "dB")
    close(tC.grad, gC, "dC")
    close(tD.grad, gD, "dD")


@pytest.mark.parametrize("d_model,n_layers,ffn_mult", [(64, 2, 0), (256, 1, 0), (64, 2, 4), (256, 1, 4)])
def test_model_gradient_matches_oracle(d_model, n_layers, ffn_mult):
    """FP32 projections: loss within 1e-5 relative and every gradient element
    within 2e-3 relative + 2e-4 of its tensor's largest magnitude (FP32
    arithmetic against FP64, rows summed in a different order); with and
    without Algorithm 1's feed-forward sub-layer (d_model 256, one layer and
    ffn_mult 4 is the paper's own model)."""
    print(f"[gpu] model gradient d_model={d_model} ffn_mult={ffn_mult}", flush=True)
    cfg = ModelConfig(d_model=d_model, n_layers=n_layers, ffn_mult=ffn_mult)
    flat = init_weights(cfg, 17)
    rng = np.random.default_rng(3)
    flat = (flat + rng.normal(0, 0.02, flat.size)).astype(np.float32)
    m = boa().Model(cfg, flat)
    # 3 x 40 rows: two 64-row GEMM tiles with a ragged tail, several row slices
    seqs = np.stack([records_f32_mix(41, 400 + b) for b in range(3)])
    loss, grad = tr().loss_and_grad(m, torch.from_numpy(seqs).cuda(), chunk_t=16)
    ref_loss, ref_grad = oracle_loss_grad(cfg, flat, seqs, Tc=16)
    print(f"[gpu] loss {loss:.8f} oracle {ref_loss:.8f}")
    assert abs(loss - ref_loss) <= 1e-5 * abs(ref_loss)
    g = grad.cpu().numpy().astype(np.float64)
    off = 0
    for name, shape in param_layout(cfg):
        n = int(np.prod(shape))
        assert_close(g[off:off + n], ref_grad[off:off + n], 2e-3, 2e-4, name)
        off += n
    # chunk length does not change the gradient beyond rounding
    _, grad2 = tr().loss_and_grad(m, torch.from_numpy(seqs).cuda(), chunk_t=3)
    assert torch.allclose(grad, grad2, rtol=1e-4, atol=1e-7)
    # fixed reduction order: the same call twice gives the same bits
    _, grad3 = tr().loss_and_grad(m, torch.from_numpy(seqs).cuda(), chunk_t=16)
    assert torch.equal(grad, grad3)


def test_model_gradient_bf16_matches_oracle():
    """BF16 projection operands (FP32 accumulation, FP32 master weights): the
    loss within 1e-3 relative and every gradient element within 3e-2 relative
    + 3e-2 of its tensor's largest magnitude.  bf16 keeps 8 significant bits
    (relative rounding 2^-9 per operand), and every gradient passes through up
    to three rounded products; the bound leaves room for that, not for a wrong
    term (a dropped or misplaced term shows at the scale of the tensor)."""
    print("[gpu] model gradient bf16", flush=True)
    cfg = ModelConfig(d_model=64, n_layers=2)
    flat = init_weights(cfg, 17)
    rng = np.random.default_rng(3)
    flat = (flat + rng.normal(0, 0.02, flat.size)).astype(np.float32)
    m = boa().Model(cfg, flat)
    seqs = np.stack([records_f32_mix(129, 700 + b) for b in range(4)])
    loss, grad = tr().loss_and_grad(m, torch.from_numpy(seqs).cuda(), chunk_t=32, dtype="bf16")
    ref_loss, ref_grad = oracle_loss_grad(cfg, flat, seqs, Tc=32)
    print(f"[gpu] bf16 loss {loss:.6f} oracle {ref_loss:.6f}")
    assert abs(loss - ref_loss) <= 1e-3 * abs(ref_loss)
    g = grad.cpu().numpy().astype(np.float64)
    off = 0
    for name, shape in param_layout(cfg):
        n = int(np.prod(shape))
        assert_close(g[off:off + n], ref_grad[off:off + n], 3e-2, 3e-2, name)
        off += n


def test_adamw_matches_oracle():
    """Three AdamW steps on seeded gradients (one above the clipping norm, one
    below, one with exact zeros) against the oracle's AdamW in FP64."""
    print("[gpu] adamw", flush=True)
    cfg = ModelConfig(d_model=64, n_layers=1)
    w0 = init_weights(cfg, 5).astype(np.float32)
    m = boa().Model(cfg, w0)
    o = tr().opts(lr=3e-3, warmup=2, weight_decay=0.05, grad_clip=1.0)
    ref = AdamW(w0.size, lr=3e-3, wd=0.05)
    w = w0.astype(np.float64)
    rng = np.random.default_rng(11)
    for step, scale in enumerate([1e-2, 1e-4, 3e-3]):
        g = (rng.normal(0, scale, w0.size)).astype(np.float32)
        if step == 2:
            g[::7] = 0.0
        tr().optimizer_step(m, torch.from_numpy(g).cuda(), o)
        gc, _ = clip_global_norm(g.astype(np.float64), 1.0)
        lr = 3e-3 * min(1.0, (step + 1) / 2)       # linear warm-up over 2 steps
        w = ref.step(w, gc, lr)
        assert_close(m.get_weights(), w, 2e-6, 1e-6, f"step {step}")


def test_training_is_deterministic_and_resumes(tmp_path):
    """Two runs from the same weights and data give identical weights; a
    checkpoint (weights, AdamW moments, step count) resumes exactly."""
    print("[gpu] training determinism", flush=True)
    cfg = ModelConfig(d_model=64, n_layers=2)
    w0 = init_weights(cfg, 23)
    data = torch.from_numpy(np.stack([records_f32_mix(513, 60 + b) for b in range(4)])).cuda()
    for dt in ("f32", "bf16"):
        o = tr().opts(lr=2e-3, warmup=2, chunk_t=64, dtype=dt)
        ma, mb = boa().Model(cfg, w0), boa().Model(cfg, w0)
        for _ in range(3):
            la = tr().train_step(ma, data, o)
            lb = tr().train_step(mb, data, o)
            assert la == lb
        assert np.array_equal(ma.get_weights(), mb.get_weights())
        path = str(tmp_path / f"ckpt_{dt}.boat")
        tr().save_state(ma, path)
        for _ in range(2):
            tr().train_step(ma, data, o)
        mc = boa().Model(cfg, init_weights(cfg, 99))
        tr().load_state(mc, path)
        for _ in range(2):
            tr().train_step(mc, data, o)
        assert np.array_equal(ma.get_weights(), mc.get_weights())
    with pytest.raises(boa().BoaError):
        tr().load_state(boa().Model(ModelConfig(d_model=128, n_layers=1), init_weights(ModelConfig(128, 1), 1)), path)
    # train(model, bytes) split into several calls equals one call: the window
    # order continues from the model's step count
    host = np.concatenate([records_f32_mix(4096, 90 + k) for k in range(8)])
    one, two = boa().Model(cfg, w0), boa().Model(cfg, w0)
    o6 = tr().opts(lr=2e-3, warmup=2, steps=6, batch=3, seq_len=1024, chunk_t=64, seed=9)
    l_one = tr().train(one, host, o6)
    o2 = tr().opts(lr=2e-3, warmup=2, steps=2, batch=3, seq_len=1024, chunk_t=64, seed=9)
    l_two = np.concatenate([tr().train(two, host, o2) for _ in range(3)])
    assert tr().steps_done(two) == 6
    assert np.array_equal(l_one, l_two)
    assert np.array_equal(one.get_weights(), two.get_weights())


def test_training_beats_order2_and_untrained():
    """Train the cfg2-shaped model on the record stream, then compare held-out
    coded bits/byte: trained < adaptive order-2 < untrained."""
    print("[gpu] training run", flush=True)
    cfg = ModelConfig(d_model=256, n_layers=3)
    w0 = init_weights(cfg, 4244)
    m = boa().Model(cfg, w0)
    # many independent record streams (each its own run-number range), as a
    # multi-run HEP sample: the model has to learn to carry the run number
    # forward instead of memorising one range
    train_data = np.concatenate([records_f32_mix(128 << 10, 1340 + k) for k in range(64)])
    o = tr().opts(lr=2e-3, warmup=30, steps=600, batch=8, seq_len=4096, chunk_t=256, seed=5)
    losses = tr().train(m, train_data, o)
    print(f"[gpu] loss first {losses[:5].mean():.3f} last {losses[-10:].mean():.3f} nats")
    assert np.all(np.isfinite(losses)) and losses[-10:].mean() < losses[:5].mean() - 0.5
    held = records_f32_mix(256 << 10, 7331)
    lens = [65536] * 4
    d = torch.from_numpy(held).cuda()

    def bpb(model):
        payload, poff, plen, ib = boa().encode_dev(model, d, lens)
        return float(ib.cpu().numpy()[:4].sum()) / (len(held) - 4)

    trained = bpb(m)
    d_in = torch.from_numpy(train_data[:256 << 10].copy()).cuda()
    pl_in = boa().encode_dev(m, d_in, lens)[3]
    print(f"[gpu] in-sample bits/byte {float(pl_in.cpu().numpy()[:4].sum()) / ((256 << 10) - 4):.3f}")
    untrained = bpb(boa().Model(cfg, w0))
    _, _, _, ib2 = boa().order2_encode(d, lens)
    o2 = float(ib2.cpu().numpy()[:4].sum()) / (len(held) - 4)
    print(f"[gpu] held-out bits/byte: trained {trained:.3f}, order-2 {o2:.3f}, untrained {untrained:.3f}")
    assert trained < o2 < untrained
    # the trained model still round-trips
    blob = boa().compress(m, held[:20000].tobytes(), chunk_len=5000)
    assert boa().decompress(m, blob) == held[:20000].tobytes()
