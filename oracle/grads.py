"""Analytic gradients of the fitting loss w.r.t. every Gaussian parameter.

The image is Eq. 2 (Sec. 3.1), C_k(p) = sum_n c'_{n,k} w_pn with
w_pn = exp(-q_pn / 2) [q_pn <= 9] and q = d^T Sigma^{-1} d (Eq. 1,
Sigma = L L^T).  Given g(p) = dLoss/dC(p), the chain rule is taken through
the conic form:

    dL/dc'_k = sum_p g_k(p) w
    dL/dq    = -1/2 (g(p) . c') w
    dq/dmu   = -2 Sigma^{-1} d                       (v := Sigma^{-1} d)
    dq/dSigma^{-1} = d d^T,  dSigma^{-1} = -Sigma^{-1} dSigma Sigma^{-1}
      =>  dq = -v^T dSigma v,  with Sigma_11 = l1^2, Sigma_12 = l1 l2,
          Sigma_22 = l2^2 + l3^2.

The cutoff indicator is held fixed (no term from the discontinuity at
q = 9).  Beside each gradient element the function returns the sum of the
absolute values of its per-pixel terms (the scale of the sum, used for a
relative tolerance) and the part of that sum contributed by pairs inside the
ambiguity band |q - 9| <= 1e-4.
"""
from __future__ import annotations

import numpy as np

from .gauss import AMBIGUOUS_BAND, CUTOFF_Q, conic, culled
from .render import pair_terms


def gradients(xy, chol, rgb, dl_dimg, H: int, W: int):
    """Returns dict(g_xy [N,2], g_chol [N,3], g_rgb [N,3], and the matching
    'abs_*' and 'amb_*' arrays).  Culled Gaussians get exact zeros."""
    xy = np.asarray(xy, np.float64)
    chol = np.asarray(chol, np.float64)
    rgb = np.asarray(rgb, np.float64)
    g = np.asarray(dl_dimg, np.float64)
    N = xy.shape[0]
    out = {k: np.zeros((N, d)) for k, d in
           (("g_xy", 2), ("g_chol", 3), ("g_rgb", 3),
            ("abs_xy", 2), ("abs_chol", 3), ("abs_rgb", 3),
            ("amb_xy", 2), ("amb_chol", 3), ("amb_rgb", 3))}
    dead = culled(xy, chol)
    for n in range(N):
        if dead[n]:
            continue
        t = pair_terms(n, xy, chol, H, W)
        if t is None:
            continue
        (x0, x1, y0, y1), dx, dy, q = t
        l1, l2, l3 = chol[n]
        A, B, C = conic(l1, l2, l3)
        e = np.exp(-0.5 * q)
        inside = q <= CUTOFF_Q
        band = np.abs(q - CUTOFF_Q) <= AMBIGUOUS_BAND
        gw = g[:, y0:y1, x0:x1]
        v1 = A * dx + B * dy
        v2 = B * dx + C * dy
        dq_dl1 = -(2.0 * l1 * v1 * v1 + 2.0 * l2 * v1 * v2)
        dq_dl2 = -(2.0 * l1 * v1 * v2 + 2.0 * l2 * v2 * v2)
        dq_dl3 = -(2.0 * l3 * v2 * v2)
        gc = gw[0] * rgb[n, 0] + gw[1] * rgb[n, 1] + gw[2] * rgb[n, 2]
        dl_dq = -0.5 * gc * e          # before applying the indicator
        terms = {
            ("g_xy", 0): dl_dq * (-2.0 * v1),
            ("g_xy", 1): dl_dq * (-2.0 * v2),
            ("g_chol", 0): dl_dq * dq_dl1,
            ("g_chol", 1): dl_dq * dq_dl2,
            ("g_chol", 2): dl_dq * dq_dl3,
            ("g_rgb", 0): gw[0] * e,
            ("g_rgb", 1): gw[1] * e,
            ("g_rgb", 2): gw[2] * e,
        }
        for (name, j), term in terms.items():
            kept = np.where(inside, term, 0.0)
            out[name][n, j] = kept.sum()
            out["abs" + name[1:]][n, j] = np.abs(kept).sum()
            out["amb" + name[1:]][n, j] = np.abs(np.where(band, term, 0.0)).sum()
    return out


def loss_gradients(xy, chol, rgb, target, H: int, W: int):
    """Render, MSE loss and parameter gradients in one call (FP64)."""
    from .render import render_box
    from .loss import dloss_dimg, mse
    img = render_box(xy, chol, rgb, H, W, want_bounds=False)["img"]
    g = gradients(xy, chol, rgb, dloss_dimg(img, target), H, W)
    g["loss"] = mse(img, target)
    g["img"] = img
    return g
