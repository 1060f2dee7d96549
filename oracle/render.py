"""Forward rendering, Eq. 2 (Sec. 3.1), in FP64.

``render_bruteforce`` is the definition itself: every pixel sums every
non-culled Gaussian, with no tiling.  ``render_box`` evaluates the same sum
but visits, for each Gaussian, only the pixels inside its 3-sigma box (the
pixels the cutoff can admit); the two agree to FP64 rounding.

Both return, beside the image, the per-pixel absolute sum sum_n |c'_n| w_pn
and the part of it that comes from pairs within the ambiguity band
|q - 9| <= 1e-4 (evaluated whether or not the pair is admitted), which the
parity tests use to build their tolerance.
"""
from __future__ import annotations

import math

import numpy as np

from .gauss import AMBIGUOUS_BAND, CUTOFF_Q, box_halfwidths, culled, mahalanobis_sq


def _as64(xy, chol, rgb):
    return (np.asarray(xy, np.float64), np.asarray(chol, np.float64),
            np.asarray(rgb, np.float64))


def render_bruteforce(xy, chol, rgb, H: int, W: int):
    """Eq. 2 summed over all pixels x all Gaussians.  Cost O(H W N).

    Returns dict(img [3,H,W], abs [3,H,W], amb [3,H,W]).
    """
    xy, chol, rgb = _as64(xy, chol, rgb)
    dead = culled(xy, chol)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    cx, cy = xs + 0.5, ys + 0.5
    img = np.zeros((3, H, W))
    aab = np.zeros((3, H, W))
    amb = np.zeros((3, H, W))
    for n in range(xy.shape[0]):
        if dead[n]:
            continue
        l1, l2, l3 = chol[n]
        q = mahalanobis_sq(cx - xy[n, 0], cy - xy[n, 1], l1, l2, l3)
        e = np.exp(-0.5 * q)
        inside = q <= CUTOFF_Q
        band = np.abs(q - CUTOFF_Q) <= AMBIGUOUS_BAND
        w = np.where(inside, e, 0.0)
        for k in range(3):
            img[k] += rgb[n, k] * w
            aab[k] += abs(rgb[n, k]) * w
            amb[k] += np.where(band, abs(rgb[n, k]) * e, 0.0)
    return {"img": img, "abs": aab, "amb": amb}


def gaussian_window(xn, yn, l1, l2, l3, H: int, W: int):
    """Pixel index ranges [x0,x1) x [y0,y1) whose centres can satisfy q <= 9.

    Widened by one pixel on each side so that FP64 rounding of the box can
    never drop an admissible pixel; the cutoff test itself decides.
    """
    rx, ry = box_halfwidths(l1, l2, l3)
    if not (math.isfinite(rx) and math.isfinite(ry)):
        return 0, W, 0, H
    x0 = max(0, int(math.floor(xn - rx - 0.5)) - 1)
    x1 = min(W, int(math.floor(xn + rx - 0.5)) + 2)
    y0 = max(0, int(math.floor(yn - ry - 0.5)) - 1)
    y1 = min(H, int(math.floor(yn + ry - 0.5)) + 2)
    return x0, x1, y0, y1


def pair_terms(n, xy, chol, H, W):
    """For Gaussian n: window bounds and q, exp(-q/2) on the window."""
    l1, l2, l3 = chol[n]
    x0, x1, y0, y1 = gaussian_window(xy[n, 0], xy[n, 1], l1, l2, l3, H, W)
    if x1 <= x0 or y1 <= y0:
        return None
    ys, xs = np.mgrid[y0:y1, x0:x1].astype(np.float64)
    dx = xs + 0.5 - xy[n, 0]
    dy = ys + 0.5 - xy[n, 1]
    q = mahalanobis_sq(dx, dy, l1, l2, l3)
    return (x0, x1, y0, y1), dx, dy, q


def render_box(xy, chol, rgb, H: int, W: int, want_bounds: bool = True):
    """Eq. 2 evaluated per Gaussian over its 3-sigma box.

    Returns dict(img, abs, amb) like ``render_bruteforce``.
    """
    xy, chol, rgb = _as64(xy, chol, rgb)
    dead = culled(xy, chol)
    img = np.zeros((3, H, W))
    aab = np.zeros((3, H, W)) if want_bounds else None
    amb = np.zeros((3, H, W)) if want_bounds else None
    for n in range(xy.shape[0]):
        if dead[n]:
            continue
        t = pair_terms(n, xy, chol, H, W)
        if t is None:
            continue
        (x0, x1, y0, y1), _, _, q = t
        e = np.exp(-0.5 * q)
        w = np.where(q <= CUTOFF_Q, e, 0.0)
        for k in range(3):
            img[k, y0:y1, x0:x1] += rgb[n, k] * w
        if want_bounds:
            band = np.abs(q - CUTOFF_Q) <= AMBIGUOUS_BAND
            for k in range(3):
                aab[k, y0:y1, x0:x1] += abs(rgb[n, k]) * w
                amb[k, y0:y1, x0:x1] += np.where(band, abs(rgb[n, k]) * e, 0.0)
    return {"img": img, "abs": aab, "amb": amb}


def count_pairs_in_cutoff(xy, chol, H: int, W: int) -> int:
    """P_in: number of (pixel, Gaussian) pairs with q <= 9 in the frame."""
    xy = np.asarray(xy, np.float64)
    chol = np.asarray(chol, np.float64)
    dead = culled(xy, chol)
    total = 0
    for n in range(xy.shape[0]):
        if dead[n]:
            continue
        t = pair_terms(n, xy, chol, H, W)
        if t is None:
            continue
        total += int(np.count_nonzero(t[3] <= CUTOFF_Q))
    return total


def render_pixels(xy, chol, rgb, px, py):
    """Eq. 2 at selected pixels only: for pixel (px[i], py[i]) the sum over
    every non-culled Gaussian (brute force, vectorised over Gaussians).

    Returns dict(img [3,P], abs [3,P], amb [3,P]).
    """
    xy, chol, rgb = _as64(xy, chol, rgb)
    live = ~culled(xy, chol)
    xy, chol, rgb = xy[live], chol[live], rgb[live]
    l1, l2, l3 = chol[:, 0], chol[:, 1], chol[:, 2]
    P = len(px)
    img = np.zeros((3, P))
    aab = np.zeros((3, P))
    amb = np.zeros((3, P))
    for i in range(P):
        q = mahalanobis_sq(px[i] + 0.5 - xy[:, 0], py[i] + 0.5 - xy[:, 1], l1, l2, l3)
        e = np.exp(-0.5 * q)
        w = np.where(q <= CUTOFF_Q, e, 0.0)
        band = np.abs(q - CUTOFF_Q) <= AMBIGUOUS_BAND
        img[:, i] = rgb.T @ w
        aab[:, i] = np.abs(rgb).T @ w
        amb[:, i] = np.abs(rgb).T @ np.where(band, e, 0.0)
    return {"img": img, "abs": aab, "amb": amb}
