"""Which Gaussians a P-frame fine-tunes: selective optimisation, Sec. 3.2.C.

The paper forms the residual between the current frame and the reference
frame, keeps the pixels whose change exceeds a user-defined threshold, and
uses the reference frame's pixel-to-Gaussian mapping to find every Gaussian
that influences one of those pixels; only these Gaussians are optimised in
the P-frame, the rest keep the reference frame's parameters.

Readings (the paper gives no formula):

* the residual of pixel p is taken between the two source frames, channel by
  channel, and p has changed iff some channel's absolute difference is
  strictly above the threshold tau (for finite values: the largest one is; a
  channel whose difference is not a number never counts);
* a Gaussian influences p iff p lies inside its 3-sigma cutoff (q <= 9), the
  same rule that decides which terms Eq. 2 sums; a Gaussian that the
  degenerate-covariance rule culls influences nothing.

Both are integer decisions taken from floating-point values, so they are
specified in FP32 with a fixed operation order, round-to-nearest-even and no
fused multiply-add (numpy float32 scalars and arrays evaluate exactly that):

    d_k = I_t[k] - I_{t-1}[k];  changed = |d_0| > tau or |d_1| > tau or |d_2| > tau
    dx = (x + 1/2) - mx;  dy = (y + 1/2) - my
    u1 = dx / l1;  t = l2 * u1;  e = dy - t;  u2 = e / l3
    q = u1 * u1 + u2 * u2;  influences = q <= 9

(u = L^-1 d with L = [[l1, 0], [l2, l3]], Eq. 1, so q = d^T Sigma^-1 d.)  The
oracle evaluates every (changed pixel, Gaussian) pair by brute force.
"""
from __future__ import annotations

import numpy as np

from .gauss import culled

F32 = np.float32
CUTOFF = F32(9.0)


def changed_pixels(frame, prev, tau) -> np.ndarray:
    """Boolean [H, W]: pixels where some channel's absolute change between
    prev and frame ([3, H, W] each, FP32) is strictly above tau."""
    a = np.asarray(frame, F32)
    b = np.asarray(prev, F32)
    with np.errstate(invalid="ignore"):
        d = np.abs(a - b)
        return (d[0] > F32(tau)) | (d[1] > F32(tau)) | (d[2] > F32(tau))


def influence_q(xy, chol, px, py) -> np.ndarray:
    """FP32 q of every (pixel, Gaussian) pair: [P, N] for pixel columns px
    and rows py (integer arrays of length P), in the order specified above."""
    xy = np.asarray(xy, F32)
    chol = np.asarray(chol, F32)
    cx = (np.asarray(px, np.int64).astype(F32) + F32(0.5))[:, None]
    cy = (np.asarray(py, np.int64).astype(F32) + F32(0.5))[:, None]
    mx, my = xy[None, :, 0], xy[None, :, 1]
    l1, l2, l3 = chol[None, :, 0], chol[None, :, 1], chol[None, :, 2]
    with np.errstate(all="ignore"):
        dx = cx - mx
        dy = cy - my
        u1 = dx / l1
        t = l2 * u1
        e = dy - t
        u2 = e / l3
        return u1 * u1 + u2 * u2


def selected_gaussians(xy, chol, changed, chunk: int = 512) -> np.ndarray:
    """Boolean [N]: Gaussians with q <= 9 at some changed pixel (brute force
    over all changed pixels); culled Gaussians are never selected."""
    ys, xs = np.nonzero(np.asarray(changed, bool))
    N = np.asarray(xy).shape[0]
    sel = np.zeros(N, bool)
    for i in range(0, len(xs), chunk):
        q = influence_q(xy, chol, xs[i:i + chunk], ys[i:i + chunk])
        sel |= np.any(q <= CUTOFF, axis=0)
    return sel & ~culled(xy, chol)


def select(frame, prev, tau, xy, chol):
    """(changed [H, W], selected [N]) for a P-frame: the pixels that changed
    since the reference frame and the reference Gaussians influencing them."""
    ch = changed_pixels(frame, prev, tau)
    return ch, selected_gaussians(xy, chol, ch)
