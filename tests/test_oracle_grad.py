"""Pins of the oracle's hand-written gradients, chunk recomputation and AdamW (CPU only).

Gradients are pinned by central finite differences in float64 and by PyTorch
autograd run over a library-op forward of the same network; chunked
recomputation of the scan must reproduce the unchunked gradient; one AdamW
step on f(theta) = theta^2 / 2 must match its closed form.
"""
import numpy as np
import pytest
import torch

from synth import ModelConfig, init_weights, records_f32_mix
from synth.weights import param_layout
from oracle.grad import loss_and_grad, AdamW, clip_global_norm, scan_forward, scan_backward

CFG = ModelConfig(d_model=8, n_layers=1)
CFG_FFN = ModelConfig(d_model=8, n_layers=1, ffn_mult=4)     # with Algorithm 1's feed-forward sub-layer


def small_case(seed=0, B=2, T=17, cfg=CFG):
    flat = init_weights(cfg, 21 + seed).astype(np.float64)
    rng = np.random.default_rng(seed)
    flat = flat + rng.normal(0, 0.05, flat.size)          # move off the symmetric init
    seqs = np.stack([records_f32_mix(T, 40 + seed + b) for b in range(B)])
    return flat, seqs


@pytest.mark.parametrize("cfg", [CFG, CFG_FFN], ids=["mamba", "mamba+ffn"])
def test_gradient_matches_central_differences(cfg):
    flat, seqs = small_case(cfg=cfg)
    _, g = loss_and_grad(cfg, flat, seqs)
    rng = np.random.default_rng(1)
    # every tensor gets probed
    offs, o = [], 0
    for name, shape in param_layout(cfg):
        n = int(np.prod(shape))
        offs += list(o + rng.choice(n, min(n, 6), replace=False))
        o += n
    h = 1e-6
    for i in offs:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        lp, _ = loss_and_grad(cfg, fp, seqs, need_grad=False)
        lm, _ = loss_and_grad(cfg, fm, seqs, need_grad=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 2e-9, (i, fd, g[i])


@pytest.mark.parametrize("ffn_mult", [0, 4])
def test_gradient_matches_torch_autograd(ffn_mult):
    cfg = ModelConfig(d_model=16, n_layers=2, ffn_mult=ffn_mult)
    flat = init_weights(cfg, 5).astype(np.float64)
    seqs = np.stack([records_f32_mix(24, 9), records_f32_mix(24, 10)])
    loss, g = loss_and_grad(cfg, flat, seqs)

    # autograd through a torch float64 forward assembled from library ops
    import torch.nn.functional as F
    from synth.weights import param_layout as pl
    tens, off = {}, 0
    for name, shape in pl(cfg):
        n = int(np.prod(shape))
        tens[name] = torch.tensor(flat[off:off + n].reshape(shape), requires_grad=True)
        off += n
    Di, R, N = cfg.d_inner, cfg.dt_rank, cfg.d_state
    y = torch.from_numpy(seqs[:, :-1].astype(np.int64))
    tgt = torch.from_numpy(seqs[:, 1:].astype(np.int64))
    r = F.embedding(y, tens["embed"])
    for l in range(cfg.n_layers):
        p = f"layers.{l}."
        a = F.layer_norm(r, (cfg.d_model,), tens[p + "norm_w"], tens[p + "norm_b"], eps=1e-5)
        xz = F.linear(a, tens[p + "in_proj_w"])
        x, z = xz[..., :Di], xz[..., Di:]
        T = x.shape[1]
        xc = F.conv1d(x.transpose(1, 2), tens[p + "conv_w"][:, None, :], tens[p + "conv_b"],
                      padding=cfg.d_conv - 1, groups=Di)[..., :T].transpose(1, 2)
        xs = F.silu(xc)
        dbc = F.linear(xs, tens[p + "x_proj_w"])
        dt = F.softplus(F.linear(dbc[..., :R], tens[p + "dt_proj_w"], tens[p + "dt_proj_b"]))
        Bm, Cm = dbc[..., R:R + N], dbc[..., R + N:]
        A = -torch.exp(tens[p + "A_log"])
        h = torch.zeros(x.shape[0], Di, N, dtype=torch.float64)
        ys = []
        for s in range(T):
            h = torch.exp(dt[:, s, :, None] * A) * h + (dt[:, s] * xs[:, s])[..., None] * Bm[:, s, None, :]
            ys.append((h * Cm[:, s, None, :]).sum(-1) + tens[p + "D"] * xs[:, s])
        r = r + F.linear(torch.stack(ys, 1) * F.silu(z), tens[p + "out_proj_w"])
        if cfg.ffn_mult:
            f = F.linear(F.gelu(F.linear(r, tens[p + "ffn_w1"], tens[p + "ffn_b1"])), tens[p + "ffn_w2"],
                         tens[p + "ffn_b2"])
            r = F.layer_norm(f, (cfg.d_model,), tens[p + "ffn_norm_w"], tens[p + "ffn_norm_b"], eps=1e-5)
    rf = F.layer_norm(r, (cfg.d_model,), tens["norm_f_w"], tens["norm_f_b"], eps=1e-5)
    logits = F.linear(rf, tens["head_w"], tens["head_b"])
    tl = F.cross_entropy(logits.reshape(-1, 256), tgt.reshape(-1))
    tl.backward()
    assert abs(tl.item() - loss) <= 1e-12 * abs(loss)
    tg = np.concatenate([tens[name].grad.numpy().ravel() for name, _ in pl(cfg)])
    assert np.allclose(g, tg, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("Tc", [1, 4, 16])
def test_chunk_recomputation_is_exact(Tc):
    flat, seqs = small_case(seed=3, T=30)
    _, g_full = loss_and_grad(CFG, flat, seqs, Tc=None)
    _, g_chunk = loss_and_grad(CFG, flat, seqs, Tc=Tc)
    assert np.allclose(g_full, g_chunk, rtol=1e-12, atol=1e-14)


def test_scan_backward_saved_states_are_sparse():
    rng = np.random.default_rng(2)
    B, T, Di, N = 2, 20, 3, 4
    x, dt = rng.normal(size=(B, T, Di)), np.exp(rng.normal(-1, 0.5, (B, T, Di)))
    A = -np.exp(rng.normal(size=(Di, N)))
    Bm, Cm = rng.normal(size=(B, T, N)), rng.normal(size=(B, T, N))
    _, saved = scan_forward(x, dt, A, Bm, Cm, np.ones(Di), save_every=8)
    assert len(saved) == 3                              # O(T / Tc) states kept
    out = scan_backward(rng.normal(size=(B, T, Di)), x, dt, A, Bm, Cm, np.ones(Di), saved, 8)
    assert all(np.all(np.isfinite(o)) for o in out)


def test_adamw_one_step_closed_form():
    """f = theta^2/2, g = theta.  Step 1: m = (1-b1) g, v = (1-b2) g^2, bias-corrected
    m_hat = g, v_hat = g^2, so theta' = theta (1 - lr wd) - lr g / (|g| + eps)."""
    th = np.array([0.5, -2.0, 3.0, 1e-3])
    opt = AdamW(4, lr=1e-2, wd=0.1, eps=1e-8)
    new = opt.step(th, th.copy())
    ref = th * (1 - 1e-2 * 0.1) - 1e-2 * th / (np.abs(th) + 1e-8)
    assert np.allclose(new, ref, rtol=1e-14, atol=1e-16)
    # a second step follows the recurrences for m, v
    new2 = opt.step(new, new.copy())
    m = 0.9 * (0.1 * th) + 0.1 * new
    v = 0.999 * (0.001 * th * th) + 0.001 * new * new
    ref2 = new * (1 - 1e-3) - 1e-2 * (m / (1 - 0.81)) / (np.sqrt(v / (1 - 0.999 ** 2)) + 1e-8)
    assert np.allclose(new2, ref2, rtol=1e-13, atol=1e-16)


def test_clip_global_norm():
    g = np.array([3.0, 4.0])
    c, n = clip_global_norm(g, 1.0)
    assert n == 5.0 and np.allclose(np.linalg.norm(c), 1.0, rtol=1e-6)
    c2, _ = clip_global_norm(g * 0.01, 1.0)
    assert np.array_equal(c2, g * 0.01)
