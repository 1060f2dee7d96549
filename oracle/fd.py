"""Central finite differences of the brute-force loss (FP64).

A parameter element is differentiated with step h = 1e-6 * max(1, |theta|).
The loss is piecewise smooth: the 3-sigma cutoff (q <= 9) switches pairs on
and off.  An FD estimate is accepted only if the set of admitted
(pixel, Gaussian) pairs is identical at theta + h and theta - h; otherwise h
is halved (up to five times) and, if the set still changes, the element is
reported as undefined (NaN) because the difference quotient straddles a
cutoff crossing.
"""
from __future__ import annotations

import numpy as np

from .gauss import CUTOFF_Q, culled, mahalanobis_sq
from .loss import mse


def _render_and_mask(xy, chol, rgb, H, W):
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    cx, cy = xs + 0.5, ys + 0.5
    img = np.zeros((3, H, W))
    dead = culled(xy, chol)
    masks = []
    for n in range(xy.shape[0]):
        if dead[n]:
            masks.append(None)
            continue
        q = mahalanobis_sq(cx - xy[n, 0], cy - xy[n, 1], *chol[n])
        inside = q <= CUTOFF_Q
        w = np.where(inside, np.exp(-0.5 * q), 0.0)
        for k in range(3):
            img[k] += rgb[n, k] * w
        masks.append(inside)
    return img, masks


def _same_masks(a, b):
    for x, y in zip(a, b):
        if (x is None) != (y is None):
            return False
        if x is not None and not np.array_equal(x, y):
            return False
    return True


def fd_gradients(xy, chol, rgb, target, H: int, W: int, which=None):
    """FD gradients of MSE(render(theta), target).

    ``which`` selects elements: a list of (group, n, j) with group in
    {'xy','chol','rgb'}; default all.  Returns dict group -> array with NaN
    where FD is undefined.
    """
    params = {"xy": np.array(xy, np.float64), "chol": np.array(chol, np.float64),
              "rgb": np.array(rgb, np.float64)}
    target = np.asarray(target, np.float64)
    out = {k: np.full(v.shape, np.nan) for k, v in params.items()}
    if which is None:
        which = [(g, n, j) for g, v in params.items()
                 for n in range(v.shape[0]) for j in range(v.shape[1])]
    for grp, n, j in which:
        base = params[grp][n, j]
        h = 1e-6 * max(1.0, abs(base))
        val = np.nan
        for _ in range(6):
            p_plus = {k: v.copy() for k, v in params.items()}
            p_minus = {k: v.copy() for k, v in params.items()}
            p_plus[grp][n, j] = base + h
            p_minus[grp][n, j] = base - h
            ip, mp = _render_and_mask(p_plus["xy"], p_plus["chol"], p_plus["rgb"], H, W)
            im, mm = _render_and_mask(p_minus["xy"], p_minus["chol"], p_minus["rgb"], H, W)
            if _same_masks(mp, mm):
                val = (mse(ip, target) - mse(im, target)) / (2.0 * h)
                break
            h *= 0.5
        out[grp][n, j] = val
    return out
