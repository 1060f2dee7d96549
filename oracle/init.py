"""Content-aware ROI initialisation (Sec. 3.2.A), synthetic-frame form.

The paper seeds one Gaussian per K-means superpixel of the ROI (person mask
from a matting model): mean at the segment centre, Cholesky factor from the
segment covariance, colour = the segment's mean colour.  Neither the matting
model nor the superpixel code is available, so the ROI is the frame's known
subject mask and the content awareness comes from sampling Gaussian centres
with probability rising with the local image gradient.  The rule, step by
step (integer decisions are exact; scales and colours are FP64 rounded to
FP32):

1. Y = (R + G) + B per pixel (FP32, left to right).
2. Gradient by central differences (Y[x+1] - Y[x-1]); at a border the
   one-sided difference times two; a dimension of size 1 has gradient 0.
   All in FP32.
3. mag = sqrt(gx*gx + gy*gy) in FP32 (no fused multiply-add, correctly
   rounded sqrt); q = floor(1024 * mag) as an integer.
4. Over the ROI pixels (raster order): Q = sum q, R = count, base
   b = Q // (10 R), weight w = q + b + 1, total Wt = Q + (b + 1) R.
   (a uniform floor of one tenth of the mean gradient, so flat parts of the
   subject still receive Gaussians)
5. ROI draw i: k = pick_i mod Wt; the pixel is the first ROI pixel whose
   running weight sum exceeds k.  mu = pixel centre + jitter.
   Scale s = clamp(0.5 sqrt(Wt / (n_roi w)), 0.5, 16): half the side of the
   area one Gaussian is expected to cover at that density.
6. Outside draw i: k = pick_i mod O over the O non-ROI pixels (raster order),
   s = clamp(0.5 sqrt(O / n_out), 0.5, 16).
7. l1 = l3 = s, l2 = 0; colour c' = T(pixel) * kappa with
   kappa = 1 / (2 pi (1/4) (1 - e^-4.5)), so that Gaussians spaced at density
   1/(4 s^2) over a flat region render that region's colour.
If the ROI is empty the whole frame is used as ROI; if it covers the whole
frame the outside draws are uniform over the whole frame.
"""
from __future__ import annotations

import math

import numpy as np

F32 = np.float32
KAPPA = 1.0 / (2.0 * math.pi * 0.25 * (1.0 - math.exp(-4.5)))


def gradient_levels(target) -> np.ndarray:
    """Steps 1-3: integer gradient level q [H,W] (int64)."""
    T = np.asarray(target, F32)
    Y = (T[0] + T[1]) + T[2]
    H, W = Y.shape
    gx = np.zeros((H, W), F32)
    gy = np.zeros((H, W), F32)
    if W > 1:
        gx[:, 1:-1] = Y[:, 2:] - Y[:, :-2]
        gx[:, 0] = (Y[:, 1] - Y[:, 0]) * F32(2.0)
        gx[:, -1] = (Y[:, -1] - Y[:, -2]) * F32(2.0)
    if H > 1:
        gy[1:-1, :] = Y[2:, :] - Y[:-2, :]
        gy[0, :] = (Y[1, :] - Y[0, :]) * F32(2.0)
        gy[-1, :] = (Y[-1, :] - Y[-2, :]) * F32(2.0)
    a = gx * gx
    b = gy * gy
    mag = np.sqrt(a + b)
    return np.floor(mag.astype(np.float64) * 1024.0).astype(np.int64)


def _clamp_scale(s: float) -> float:
    return min(max(s, 0.5), 16.0)


def init_from_frame(target, mask, draws):
    """Return (xy [N,2], chol [N,3], rgb [N,3]) float32 and a dict of the
    integer decisions (picked pixel indices) for exact comparison."""
    T = np.asarray(target, F32)
    H, W = T.shape[1:]
    m = np.asarray(mask, bool).reshape(-1)
    if not m.any():
        m = np.ones_like(m)
    out_region = ~m
    if not out_region.any():
        out_region = np.ones_like(m)
    q = gradient_levels(T).reshape(-1)
    roi_idx = np.nonzero(m)[0]
    out_idx = np.nonzero(out_region)[0]
    R = roi_idx.size
    Q = int(q[roi_idx].sum())
    b = Q // (10 * R)
    w = q[roi_idx] + b + 1
    cum = np.cumsum(w)
    Wt = int(cum[-1])
    n_roi = draws.pick_roi.shape[0]
    n_out = draws.pick_out.shape[0]
    N = n_roi + n_out
    xy = np.zeros((N, 2), F32)
    chol = np.zeros((N, 3), F32)
    rgb = np.zeros((N, 3), F32)
    picked = np.zeros(N, np.int64)
    for i in range(n_roi):
        k = int(draws.pick_roi[i]) % Wt
        r = int(np.searchsorted(cum, k, side="right"))
        p = int(roi_idx[r])
        picked[i] = p
        s = _clamp_scale(0.5 * math.sqrt(Wt / (n_roi * int(w[r]))))
        _place(i, p, W, draws.jit_roi[i], s, T, xy, chol, rgb)
    O = out_idx.size
    for i in range(n_out):
        k = int(draws.pick_out[i]) % O
        p = int(out_idx[k])
        picked[n_roi + i] = p
        s = _clamp_scale(0.5 * math.sqrt(O / n_out))
        _place(n_roi + i, p, W, draws.jit_out[i], s, T, xy, chol, rgb)
    return xy, chol, rgb, {"picked": picked, "Wt": Wt, "base": b}


def _place(i, p, W, jit, s, T, xy, chol, rgb):
    y, x = divmod(p, W)
    xy[i, 0] = (F32(x) + F32(0.5)) + F32(jit[0])
    xy[i, 1] = (F32(y) + F32(0.5)) + F32(jit[1])
    chol[i] = (s, 0.0, s)
    for k in range(3):
        rgb[i, k] = F32(float(T[k, y, x]) * KAPPA)
