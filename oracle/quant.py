"""Post-training quantisation of a fitted frame's Gaussians and its bit
count (the compression pipeline, Sec. 3.3.A and 3.3.B, Eq. 3 and 4).

The paper applies distinct quantisation strategies to the three attributes
(mean, Cholesky vector, colour) following its predecessor image codec, and
codes I-frames with vanilla entropy coding and P-frames with bits-back
coding.  It gives no formulas for the quantisers or the coder; readings:

* mean: IEEE binary16 (round to nearest even), 16 bits per coordinate, not
  entropy coded;
* Cholesky vector and colour: per component, a uniform min-max scalar
  quantiser with b bits (b_chol, b_rgb; 1..12) over the frame's range of
  that component.  The code is an integer decision from floating point, so
  it is specified in FP32 with this order (no contraction):
      lo = min x, hi = max x;  L = 2^b - 1
      inv = L / (hi - lo)  (0 when hi == lo);  step = (hi - lo) / L
      code = clamp(rint((x - lo) * inv), 0, L)   (rint: nearest, ties to even)
      x_hat = lo + code * step
* vanilla entropy coding: an ideal static coder for the frame's own symbol
  statistics, N * H bits per quantised component with H = -sum p log2 p of
  the empirical code distribution (FP64), plus lo and hi of each component
  as side information (2 x 32 bits); positions at 16 bits each;
* bits-back saving of a P-frame that communicates n Gaussians (Eq. 3, logs
  in base 2): S_P = log2(n!) - log2(n), with n = N/20 in the paper; for F
  frames with an I-frame every K (Eq. 4): S_total = (F - F/K) S_P, and
  total bits = I-frame bits + P-frame bits - S_total.
"""
from __future__ import annotations

import math

import numpy as np

F32 = np.float32
MAX_BITS = 12
SIDE_BITS_PER_COMPONENT = 64        # lo and hi in FP32


def quantise_component(x, bits: int):
    """(codes int64 [N], x_hat float32 [N], lo, hi) for one component."""
    x = np.asarray(x, F32)
    L = F32(2 ** bits - 1)
    lo, hi = F32(x.min()), F32(x.max())
    rng = F32(hi - lo)
    if rng == F32(0):
        inv, step = F32(0), F32(0)
    else:
        inv, step = F32(L / rng), F32(rng / L)
    t = (x - lo) * inv
    codes = np.clip(np.rint(t), F32(0), L).astype(np.int64)
    xh = lo + codes.astype(F32) * step
    return codes, xh.astype(F32), lo, hi


def entropy_bits(codes, bits: int) -> float:
    """N * H of the empirical distribution of the codes (FP64)."""
    n = len(codes)
    cnt = np.bincount(np.asarray(codes, np.int64), minlength=2 ** bits).astype(np.float64)
    p = cnt[cnt > 0] / n
    return float(-(p * np.log2(p)).sum() * n)


def ptq(xy, chol, rgb, bits_chol: int = 6, bits_rgb: int = 6):
    """Quantise a frame's Gaussians.  Returns a dict with the dequantised
    parameters (float32), the codes, the ranges, the entropy-coded bits of
    every quantised component and the frame's total bits."""
    assert 1 <= bits_chol <= MAX_BITS and 1 <= bits_rgb <= MAX_BITS
    xy = np.asarray(xy, F32)
    chol = np.asarray(chol, F32)
    rgb = np.asarray(rgb, F32)
    N = xy.shape[0]
    q_xy = xy.astype(np.float16).astype(F32)
    q_chol = np.empty_like(chol)
    q_rgb = np.empty_like(rgb)
    codes = np.empty((N, 6), np.int64)
    ranges = np.empty((6, 2), F32)
    comp_bits = np.empty(6)
    for c in range(6):
        src, dst, b = (chol, q_chol, bits_chol) if c < 3 else (rgb, q_rgb, bits_rgb)
        k = c % 3
        codes[:, c], dst[:, k], ranges[c, 0], ranges[c, 1] = quantise_component(src[:, k], b)
        comp_bits[c] = entropy_bits(codes[:, c], b)
    total = 2 * 16 * N + comp_bits.sum() + 6 * SIDE_BITS_PER_COMPONENT
    return {"xy": q_xy, "chol": q_chol, "rgb": q_rgb, "codes": codes, "ranges": ranges,
            "component_bits": comp_bits, "bits": float(total)}


def bitsback_saving(n: float) -> float:
    """Eq. 3: S_P = log2(n!) - log2(n) bits for a P-frame of n Gaussians."""
    return (math.lgamma(n + 1.0) - math.log(n)) / math.log(2.0)


def sequence_bits(i_frame_bits, p_frame_bits, F: int, K: int, n_p: float):
    """Eq. 4 and the total: (total bits, S_total) for F frames with an
    I-frame every K, given the summed I-frame and P-frame bits."""
    s_total = (F - F / K) * bitsback_saving(n_p)
    return float(i_frame_bits + p_frame_bits - s_total), float(s_total)
