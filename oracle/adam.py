"""One optimiser step of the fitting loop, in FP64.

The paper fits the Gaussians by iterative "encoding optimization steps"
(Sec. 3.2.A, Sec. 4.1) without naming the optimiser; it is taken as Adam
(Kingma & Ba, Algorithm 1) with bias correction and epsilon added to the
square root of the corrected second moment:

    t <- t + 1
    m <- b1 m + (1 - b1) g
    v <- b2 v + (1 - b2) g^2
    theta <- theta - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

The learning rate is per parameter group (mean, Cholesky vector, colour).
A Gaussian whose ``active`` flag is 0 keeps its parameters and moments
unchanged (the hook for optimising only a subset of Gaussians, Sec. 3.2.C).
"""
from __future__ import annotations

import numpy as np

GROUPS = ("xy", "chol", "rgb")


def adam_step(theta: dict, grad: dict, m: dict, v: dict, t_prev: int, lr: dict,
              beta1=0.9, beta2=0.999, eps=1e-8, active=None):
    """Return (theta', m', v', t) as new FP64 dicts; inputs are not modified."""
    t = t_prev + 1
    bc1 = 1.0 - beta1 ** t
    bc2 = 1.0 - beta2 ** t
    th2, m2, v2 = {}, {}, {}
    for k in GROUPS:
        th = np.array(theta[k], np.float64)
        g = np.asarray(grad[k], np.float64)
        mk = beta1 * np.asarray(m[k], np.float64) + (1.0 - beta1) * g
        vk = beta2 * np.asarray(v[k], np.float64) + (1.0 - beta2) * g * g
        step = lr[k] * (mk / bc1) / (np.sqrt(vk / bc2) + eps)
        new = th - step
        if active is not None:
            keep = ~np.asarray(active, bool)
            new[keep] = th[keep]
            mk[keep] = np.asarray(m[k], np.float64)[keep]
            vk[keep] = np.asarray(v[k], np.float64)[keep]
        th2[k], m2[k], v2[k] = new, mk, vk
    return th2, m2, v2, t


def adamw_step(p, g, m, v, t_prev: int, lr: float, weight_decay: float,
               beta1=0.9, beta2=0.999, eps=1e-8):
    """One step of Adam with decoupled weight decay (Loshchilov & Hutter) on
    a flat parameter vector, in FP64: the optimiser of the learned
    initialiser's weights (the paper trains its regressor, Sec. 3.2.B,
    without naming one).  The decay acts on the parameters directly, not
    through the moments:

        t <- t + 1
        m <- b1 m + (1 - b1) g;   v <- b2 v + (1 - b2) g^2
        p <- p - lr * ( (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps) + wd * p )

    Returns (p', m', v', t)."""
    t = t_prev + 1
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    mk = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    vk = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    upd = (mk / (1.0 - beta1 ** t)) / (np.sqrt(vk / (1.0 - beta2 ** t)) + eps)
    return p - lr * (upd + weight_decay * p), mk, vk, t
