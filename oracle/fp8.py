"""FP8 (E4M3) projections of the predictor (test infrastructure only).

The precision modes run the projections (in_proj, out_proj, head) in a
narrower format with FP32 accumulation while the scan, softplus, exp and the
softmax normaliser stay FP32 and the CDF stays integer.  This module states
the FP8 mode exactly as the GPU path computes it, from the definition of the
OCP E4M3 format (1 sign, 4 exponent bits with bias 7, 3 mantissa bits;
subnormals; largest finite value 448; no infinities) and round to nearest
even:

* a weight matrix W is scaled by 2^-eW, eW = scale_exp(max |W|) (one exponent
  per tensor), and rounded to E4M3;
* each activation row a (the LayerNorm output feeding in_proj and the head,
  the gated row g feeding out_proj) is scaled by its own 2^-ea and rounded;
* the product is the exact dot product of the rounded values, rescaled by
  2^(ea + eW).

scale_exp(m) is the smallest integer e with m * 2^-e <= 448 (0 for m = 0), so
the scaled values never leave the finite range and every scale is a power of
two (exact to apply and to undo).  Everything here is float64.
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0
_MIN_NORMAL_EXP = -6          # 2^-6 is the smallest normal value
_SUB_STEP = 2.0 ** -9         # spacing of the subnormals


def e4m3(x):
    """Round to the nearest E4M3 value, ties to even; |x| must be <= 448."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    assert np.all(a <= E4M3_MAX), "value outside the E4M3 range"
    f, E = np.frexp(a)                        # a = f 2^E, f in [0.5, 1)
    e = E - 1                                 # a = (2f) 2^e, 2f in [1, 2)
    normal = e >= _MIN_NORMAL_EXP
    m = np.rint((2.0 * f - 1.0) * 8.0)        # 3 mantissa bits, half to even
    vn = np.ldexp(1.0 + m / 8.0, e)           # m == 8 carries into the exponent by itself
    vs = np.rint(a / _SUB_STEP) * _SUB_STEP   # subnormal grid (8 steps reach 2^-6 exactly)
    v = np.where(a == 0, 0.0, np.where(normal, vn, vs))
    return np.copysign(v, x)


def scale_exp(amax):
    """Smallest integer e with amax * 2^-e <= 448; 0 for amax = 0."""
    amax = float(amax)
    if not amax > 0.0:
        return 0
    f, E = np.frexp(amax)
    return int(E - 9 + (1 if 2.0 * f > 1.75 else 0))


def quantise_rows(a):
    """Per-row scaling and rounding: returns (q, e) with a ~ q 2^e row-wise."""
    a = np.atleast_2d(np.asarray(a, dtype=np.float64))
    e = np.array([scale_exp(np.abs(r).max()) for r in a], dtype=np.int64)
    q = e4m3(a * np.ldexp(1.0, -e)[:, None])
    return q, e


def quantise_tensor(w):
    """Per-tensor scaling and rounding: returns (q, e) with w ~ q 2^e."""
    w = np.asarray(w, dtype=np.float64)
    e = scale_exp(np.abs(w).max())
    return e4m3(w * 2.0 ** -e), e


def matmul_t(a, w):
    """a @ w.T in FP8 mode: a [B, K] rows scaled per row, w [N, K] per tensor."""
    qa, ea = quantise_rows(a)
    qw, ew = quantise_tensor(w)
    return (qa @ qw.T) * np.ldexp(1.0, ea + ew)[:, None]
