"""Predictor diagnostics: confusion matrix, Top-k curve, reliability / ECE.

Test infrastructure (the oracle): plain NumPy, written from the definitions,
used only by tests, the smoke check and the bench's CPU baseline.

The paper (Results, the confusion-matrix, Top-k and reliability figures and
the ECE values per dataset) reports these for its trained predictors without
fixing the details; the readings here are:

* the predicted byte is the argmax of p, the lowest index on ties;
* the confidence is p[pred]; a position is correct when pred == y;
* the rank of the true byte y is the number of bytes ranked above it in the
  order (higher p first, lower index first on equal p): rank 0 is a Top-1
  hit, and Top-k = fraction of positions with rank < k;
* reliability bins are equal-width over [0, 1]: bin = min(floor(conf * B),
  B - 1) with the product taken in float32 (the precision of p); each bin
  keeps its count, its correct count and the sum of its confidences as the
  integers conf * 2^32 (the confidence is at least 1/256, and every float32
  in [2^-9, 1] times 2^32 is an integer, so the sums are exact);
* ECE = sum over bins of (n_b / N) * |acc_b - conf_b|, with acc_b the correct
  fraction and conf_b the mean confidence of bin b (empty bins add 0).

Every function takes probabilities p [N, 256] and true bytes y [N].
"""
from __future__ import annotations

import numpy as np

V = 256


def predicted(p: np.ndarray) -> np.ndarray:
    """argmax over the 256 bytes, lowest index on ties (numpy's argmax)."""
    return np.argmax(p, axis=1)


def ranks(p: np.ndarray, y: np.ndarray) -> np.ndarray:
    """rank of y: #{a : p[a] > p[y]} + #{a < y : p[a] == p[y]}."""
    py = p[np.arange(len(y)), y][:, None]
    idx = np.arange(V)[None, :]
    return ((p > py) | ((p == py) & (idx < y[:, None]))).sum(axis=1)


def confusion(p: np.ndarray, y: np.ndarray) -> np.ndarray:
    """[true byte, predicted byte] counts."""
    c = np.zeros((V, V), dtype=np.int64)
    np.add.at(c, (y, predicted(p)), 1)
    return c


def rank_hist(p: np.ndarray, y: np.ndarray) -> np.ndarray:
    h = np.zeros(V, dtype=np.int64)
    np.add.at(h, ranks(p, y), 1)
    return h


def topk(hist: np.ndarray, k: int) -> float:
    """Top-k accuracy from a rank histogram."""
    n = hist.sum()
    return float(hist[:k].sum() / n) if n else 0.0


def conf_bins(conf: np.ndarray, n_bins: int) -> np.ndarray:
    c32 = np.asarray(conf, dtype=np.float32)
    b = np.floor(c32 * np.float32(n_bins)).astype(np.int64)
    return np.minimum(b, n_bins - 1)


def calibration(p: np.ndarray, y: np.ndarray, n_bins: int) -> np.ndarray:
    """[n_bins, 3] integers: count, correct count, sum of conf * 2^32."""
    pred = predicted(p)
    conf = p[np.arange(len(y)), pred].astype(np.float32)
    b = conf_bins(conf, n_bins)
    out = np.zeros((n_bins, 3), dtype=np.int64)
    fixed = (conf.astype(np.float64) * 2.0 ** 32).astype(np.int64)
    np.add.at(out[:, 0], b, 1)
    np.add.at(out[:, 1], b, (pred == y).astype(np.int64))
    np.add.at(out[:, 2], b, fixed)
    return out


def ece(cal: np.ndarray) -> float:
    """Expected calibration error from calibration()'s bins."""
    n = cal[:, 0].sum()
    if n == 0:
        return 0.0
    tot = 0.0
    for cnt, cor, cs in cal:
        if cnt:
            tot += cnt / n * abs(cor / cnt - cs / 2.0 ** 32 / cnt)
    return float(tot)


def all_diagnostics(p: np.ndarray, y: np.ndarray, n_bins: int = 10) -> dict:
    h = rank_hist(p, y)
    cal = calibration(p, y, n_bins)
    return {"confusion": confusion(p, y), "rank_hist": h, "calibration": cal,
            "top1": topk(h, 1), "top5": topk(h, 5), "top10": topk(h, 10), "ece": ece(cal)}
