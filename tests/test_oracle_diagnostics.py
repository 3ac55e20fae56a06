"""Pins of the oracle's predictor diagnostics (confusion, Top-k, reliability /
ECE) against closed forms and brute force: a one-hot predictor is perfect and
calibrated, a uniform predictor's ranks are the byte values themselves, ranks
agree with a stable sort, Top-k is monotone and reaches 1 at k = 256, and ECE
agrees with a bin-by-bin float computation written independently."""
import numpy as np

from oracle import diagnostics as dg


def rng_probs(n, seed, temp=1.0):
    r = np.random.default_rng(seed)
    lg = r.normal(size=(n, 256)) / temp
    e = np.exp(lg - lg.max(axis=1, keepdims=True))
    return (e / e.sum(axis=1, keepdims=True)).astype(np.float32), r.integers(0, 256, n)


def test_one_hot_predictor_is_perfect_and_calibrated():
    y = np.random.default_rng(1).integers(0, 256, 500)
    p = np.zeros((500, 256), np.float32)
    p[np.arange(500), y] = 1.0
    d = dg.all_diagnostics(p, y, 10)
    assert d["top1"] == 1.0 and d["ece"] == 0.0
    assert np.array_equal(np.diag(d["confusion"]), np.bincount(y, minlength=256))
    assert d["confusion"].sum() == 500 and d["calibration"][9, 0] == 500


def test_uniform_predictor_ranks_are_the_byte_values():
    y = np.random.default_rng(2).integers(0, 256, 1000)
    p = np.full((1000, 256), 1.0 / 256, np.float32)
    assert np.array_equal(dg.ranks(p, y), y)                       # every tie broken by index
    d = dg.all_diagnostics(p, y, 10)
    assert np.array_equal(d["confusion"][:, 0], np.bincount(y, minlength=256))   # argmax = byte 0
    for k in (1, 5, 10, 100):
        assert dg.topk(d["rank_hist"], k) == np.mean(y < k)
    acc = np.mean(y == 0)
    assert abs(d["ece"] - abs(acc - 1.0 / 256)) < 1e-12
    assert d["calibration"][0, 0] == 1000 and d["calibration"][0, 2] == 1000 * 2 ** 24


def test_ranks_match_a_stable_sort():
    p, y = rng_probs(300, 3, temp=0.3)
    p[:, 7] = p[:, 9]                                              # planted ties
    for i in range(300):
        order = sorted(range(256), key=lambda a: (-float(p[i, a]), a))
        assert order.index(int(y[i])) == dg.ranks(p[i:i + 1], y[i:i + 1])[0]
        assert order[0] == dg.predicted(p[i:i + 1])[0]


def test_topk_is_monotone_and_complete():
    p, y = rng_probs(2000, 4)
    h = dg.rank_hist(p, y)
    tk = [dg.topk(h, k) for k in range(1, 257)]
    assert all(a <= b for a, b in zip(tk, tk[1:])) and tk[-1] == 1.0
    assert h.sum() == 2000


def test_ece_matches_a_direct_bin_computation():
    p, y = rng_probs(5000, 5, temp=0.05)                           # peaked: confidences spread over bins
    for nb in (1, 10, 15):
        cal = dg.calibration(p, y, nb)
        conf = p.max(axis=1).astype(np.float64)
        pred = p.argmax(axis=1)
        edges = np.linspace(0.0, 1.0, nb + 1)
        ref = 0.0
        for b in range(nb):
            hi = edges[b + 1] if b < nb - 1 else 1.0 + 1e-9
            m = (conf >= edges[b]) & (conf < hi)
            if m.any():
                ref += m.mean() * abs((pred[m] == y[m]).mean() - conf[m].mean())
        assert abs(dg.ece(cal) - ref) < 1e-6
        assert cal[:, 0].sum() == 5000
        assert cal[:, 1].sum() == int((pred == y).sum())
