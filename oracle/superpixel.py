"""Superpixel initialisation of an I-frame's Gaussians (Sec. 3.2.A, Fig. 2).

The paper segments the region of interest into superpixels with a K-means
clustering superpixel algorithm and initialises one Gaussian per segment:
mean at the segment centre, Cholesky factor from the segment covariance,
colour from the segment's average colour.  Readings (the paper gives no
parameters):

* K = the number of ROI Gaussians; the K seeds are the ROI pixels the
  content-aware sampler picks, so both initialisations share their seeds
  and their Gaussians outside the ROI; as there, an empty ROI mask stands
  for the whole frame;
* K-means in (x, y, colour) in the manner of SLIC: with S = max(1,
  round(sqrt(R / K))) (R ROI pixels) and compactness m, the distance of ROI
  pixel p to centre k is D = ((dr^2 + dg^2) + db^2) + w (dx^2 + dy^2),
  w = (m / S)^2, d = pixel value - centre value, pixel position = pixel
  centre; a pixel considers only the centres whose grid cell (floor of
  position / S per axis) is within one cell of its own, and joins the one
  with the smallest D, ties to the lowest index;
* centres are exact means: from integer sums of the pixel indices and of
  the colour in 1/65536 units (rounded to nearest), positions
  (sum x / n + 1/2) and colours (sum c / (n 65536)) evaluated in FP64 and
  rounded to FP32 once; a centre with no pixel stays where it is;
* after `iters` assignment + update rounds, segment k gives mean = its
  centre, covariance = the segment's pixel-position covariance + 1/12 on
  the diagonal (one pixel's own footprint), L = chol(covariance), and colour
  c' = mean colour * n / (2 pi l1 l3 (1 - e^-4.5)), so that the Gaussian's
  rendered mass (Eq. 2 with the q <= 9 cutoff) equals the segment's total
  colour.  In FP64 from the exact integer moments, in this order, then
  rounded to FP32 once:
      ex = Sx / n;  ey = Sy / n
      vxx = (Sxx / n - ex*ex) + 1/12;  vxy = Sxy / n - ex*ey;  vyy = (Syy / n - ey*ey) + 1/12
      l1 = sqrt(vxx);  l2 = vxy / l1;  l3 = sqrt(vyy - l2*l2)
      mu = (ex + 1/2, ey + 1/2);  c'_c = Sc_c / (((65536 * 2 pi * l1) * l3) * MASS)
  with MASS = 1 - e^-4.5 as the decimal constant below.  A segment with no
  pixel keeps the content-aware Gaussian of its seed.

Distances and cell indices decide integers, so they are specified in FP32
in exactly the order above, without fused multiply-adds.
"""
from __future__ import annotations

import math

import numpy as np

F32 = np.float32
COLOUR_SCALE = 65536
MASS = 0.98889100346175773           # 1 - exp(-4.5)
SCALE_2PI = 65536.0 * 2.0 * math.pi  # 65536 * 2 pi (exact product in FP64)


def grid_step(roi_pixels: int, K: int) -> int:
    return max(1, int(round(math.sqrt(roi_pixels / K))))


def compactness_weight(m: float, S: int):
    r = F32(F32(m) / F32(S))
    return F32(r * r)


def colour_codes(frame):
    """Pixel colours in 1/65536 units, rounded to nearest (int64 [3, H, W])."""
    return np.rint(np.asarray(frame, F32).astype(np.float64) * COLOUR_SCALE).astype(np.int64)


def assign(frame, roi, cx, cy, ccol, S: int, w, pixels=None):
    """The chosen centre of ROI pixels: with pixels None a label image
    [H, W] (-1 outside the ROI), else an int64 array for the (x, y) pixels."""
    img = np.asarray(frame, F32)
    w = F32(w)
    fS = F32(S)
    cellx = np.floor(cx / fS).astype(np.int64)          # FP32 division, then floor
    celly = np.floor(cy / fS).astype(np.int64)
    cells = {}
    for k in range(len(cx)):
        cells.setdefault((int(cellx[k]), int(celly[k])), []).append(k)
    if pixels is None:
        ys, xs = np.nonzero(np.asarray(roi, bool))
    else:
        xs, ys = np.asarray(pixels, np.int64).T
    out = np.empty(len(xs), np.int64)
    for i, (x, y) in enumerate(zip(xs, ys)):
        px, py = F32(x + 0.5), F32(y + 0.5)
        cand = []
        for oy in (-1, 0, 1):
            for ox in (-1, 0, 1):
                cand += cells.get((x // S + ox, y // S + oy), [])
        best, bk = None, -1
        for k in sorted(cand):
            dr = F32(img[0, y, x] - ccol[k, 0])
            dg = F32(img[1, y, x] - ccol[k, 1])
            db = F32(img[2, y, x] - ccol[k, 2])
            dx = F32(px - cx[k])
            dy = F32(py - cy[k])
            dcol = F32(F32(F32(dr * dr) + F32(dg * dg)) + F32(db * db))
            dpos = F32(F32(dx * dx) + F32(dy * dy))
            D = F32(dcol + F32(w * dpos))
            if best is None or D < best:
                best, bk = D, k
        out[i] = bk
    if pixels is not None:
        return out
    lab = np.full(np.asarray(roi).shape, -1, np.int64)
    lab[ys, xs] = out
    return lab


def segment_sums(lab, codes, K: int):
    """Exact integer moments per segment: n, Sx, Sy, Sxx, Sxy, Syy, Sc[3]."""
    ys, xs = np.nonzero(lab >= 0)
    k = lab[ys, xs]
    out = {"n": np.bincount(k, minlength=K).astype(np.int64)}
    for name, v in (("x", xs), ("y", ys), ("xx", xs * xs), ("xy", xs * ys), ("yy", ys * ys)):
        a = np.zeros(K, np.int64)
        np.add.at(a, k, v.astype(np.int64))
        out[name] = a
    sc = np.zeros((K, 3), np.int64)
    for c in range(3):
        np.add.at(sc[:, c], k, codes[c, ys, xs])
    out["c"] = sc
    return out


def update_centres(sums, cx, cy, ccol):
    """New FP32 centres from the sums; empty segments keep theirs."""
    cx, cy, ccol = cx.copy(), cy.copy(), ccol.copy()
    for k in np.nonzero(sums["n"] > 0)[0]:
        n = float(sums["n"][k])
        cx[k] = F32(sums["x"][k] / n + 0.5)
        cy[k] = F32(sums["y"][k] / n + 0.5)
        for c in range(3):
            ccol[k, c] = F32(sums["c"][k, c] / (n * COLOUR_SCALE))
    return cx, cy, ccol


def kmeans(frame, roi, seeds_xy, iters: int, m: float):
    """`iters` rounds of assignment + update from seed pixels (int [K, 2]
    x, y).  Returns (labels of the last assignment, centres before it,
    centres after it, S)."""
    roi = np.asarray(roi, bool)
    if not roi.any():
        roi = np.ones_like(roi)
    K = len(seeds_xy)
    S = grid_step(int(roi.sum()), K)
    w = compactness_weight(m, S)
    codes = colour_codes(frame)
    s = np.asarray(seeds_xy, np.int64)
    cx = (s[:, 0] + 0.5).astype(F32)
    cy = (s[:, 1] + 0.5).astype(F32)
    ccol = (codes[:, s[:, 1], s[:, 0]].T / COLOUR_SCALE).astype(F32)
    lab = None
    prev = (cx, cy, ccol)
    for _ in range(iters):
        prev = (cx, cy, ccol)
        lab = assign(frame, roi, cx, cy, ccol, S, w)
        cx, cy, ccol = update_centres(segment_sums(lab, codes, K), cx, cy, ccol)
    return lab, prev, (cx, cy, ccol), S


def segment_gaussians(sums, fallback):
    """FP32 (xy [K,2], chol [K,3], rgb [K,3]) of the segments, in the order
    of the module docstring; empty segments take their Gaussian from
    `fallback` = (xy, chol, rgb)."""
    xy, chol, rgb = (np.array(a, F32, copy=True) for a in fallback)
    for k in np.nonzero(sums["n"] > 0)[0]:
        n = float(sums["n"][k])
        ex = sums["x"][k] / n
        ey = sums["y"][k] / n
        vxx = (sums["xx"][k] / n - ex * ex) + 1.0 / 12.0
        vxy = sums["xy"][k] / n - ex * ey
        vyy = (sums["yy"][k] / n - ey * ey) + 1.0 / 12.0
        l1 = math.sqrt(vxx)
        l2 = vxy / l1
        l3 = math.sqrt(vyy - l2 * l2)
        den = ((SCALE_2PI * l1) * l3) * MASS
        xy[k] = [F32(ex + 0.5), F32(ey + 0.5)]
        chol[k] = [F32(l1), F32(l2), F32(l3)]
        rgb[k] = [F32(sums["c"][k, c] / den) for c in range(3)]
    return xy, chol, rgb
