"""The fitting loop: render (Eq. 2) -> MSE -> gradients -> Adam, in FP64.

This is the per-frame encoding loop of Sec. 3.2 ("optimization steps" that
fit the Gaussians to the frame), run for a fixed number of steps.  The loss
of step k is evaluated at the parameters before update k (so the first loss
is that of the initialisation).  With ``active`` only the Gaussians whose
flag is set are updated (P-frame selective optimisation, Sec. 3.2.C); the
loss and the rendering still use every Gaussian.  With ``quant_bits``
(bits of the Cholesky and colour quantisers) the loop is quantisation-aware
(Sec. 3.3.A): each step renders the parameters after ``quant.ptq`` (ranges
from the current parameters) and applies the gradients taken at that point
to the unquantised parameters (straight-through).
"""
from __future__ import annotations

import numpy as np

from .adam import adam_step
from .grads import gradients
from .loss import dloss_dimg, mse
from .quant import ptq
from .render import render_box


def fit(xy, chol, rgb, target, iters: int, lr, beta1=0.9, beta2=0.999, eps=1e-8, active=None,
        quant_bits=None):
    """Returns (theta dict FP64, list of per-step losses)."""
    target = np.asarray(target, np.float64)
    H, W = target.shape[1:]
    theta = {"xy": np.array(xy, np.float64), "chol": np.array(chol, np.float64),
             "rgb": np.array(rgb, np.float64)}
    m = {k: np.zeros_like(v) for k, v in theta.items()}
    v = {k: np.zeros_like(x) for k, x in theta.items()}
    if not isinstance(lr, dict):
        lr = {k: float(lr) for k in theta}
    t = 0
    losses = []
    for _ in range(iters):
        at = theta
        if quant_bits is not None:
            q = ptq(theta["xy"], theta["chol"], theta["rgb"], *quant_bits)
            at = {k: q[k].astype(np.float64) for k in ("xy", "chol", "rgb")}
        img = render_box(at["xy"], at["chol"], at["rgb"], H, W, want_bounds=False)["img"]
        losses.append(mse(img, target))
        g = gradients(at["xy"], at["chol"], at["rgb"], dloss_dimg(img, target), H, W)
        grad = {"xy": g["g_xy"], "chol": g["g_chol"], "rgb": g["g_rgb"]}
        theta, m, v, t = adam_step(theta, grad, m, v, t, lr, beta1, beta2, eps, active)
    return theta, losses
