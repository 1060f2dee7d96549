"""Per-Gaussian definitions shared by the oracle's render and gradient code.

Eq. 1 (Sec. 3.1): Sigma = L L^T with L = [[l1, 0], [l2, l3]] built from the
Cholesky vector l = (l1, l2, l3).  The oracle works with the *conic* form
Sigma^{-1} = adj(Sigma) / det(Sigma), which is a different computation from
the triangular solve the GPU kernels use.

Eq. 2 (Sec. 3.1): C_i = sum_n c'_n exp(-sigma_n).  The paper does not define
sigma_n; it is read as half the squared Mahalanobis distance of the pixel
centre from mu_n, sigma = q/2 with q = d^T Sigma^{-1} d, d = (x+1/2, y+1/2) - mu.
A pair contributes only if q <= 9 (the 3-sigma cutoff, inclusive).
"""
from __future__ import annotations

import numpy as np

CUTOFF_Q = 9.0            # 3-sigma cutoff on q = d^T Sigma^-1 d, inclusive
AMBIGUOUS_BAND = 1e-4     # |q - 9| <= band: either inclusion is accepted
MIN_DIAG = 2.0 ** -14     # |l1| or |l3| below this -> culled


def culled(xy: np.ndarray, chol: np.ndarray) -> np.ndarray:
    """Boolean [N]: Gaussians that take no part in rendering.

    A Gaussian is culled iff any of mu_x, mu_y, l1, l2, l3 is not finite or
    |l1| < 2^-14 or |l3| < 2^-14 (the covariance is then numerically
    singular).  Colour is not inspected.
    """
    xy = np.asarray(xy, dtype=np.float64)
    chol = np.asarray(chol, dtype=np.float64)
    bad = ~np.all(np.isfinite(xy), axis=1) | ~np.all(np.isfinite(chol), axis=1)
    with np.errstate(invalid="ignore"):
        bad |= np.abs(chol[:, 0]) < MIN_DIAG
        bad |= np.abs(chol[:, 2]) < MIN_DIAG
    return bad


def covariance(l1, l2, l3):
    """Sigma = L L^T entries (s11, s12, s22) for L = [[l1,0],[l2,l3]]."""
    return l1 * l1, l1 * l2, l2 * l2 + l3 * l3


def conic(l1, l2, l3):
    """Sigma^{-1} = adj(Sigma)/det(Sigma) entries (A, B, C) so that
    q = A dx^2 + 2 B dx dy + C dy^2.  det(L L^T) = (l1 l3)^2."""
    s11, s12, s22 = covariance(l1, l2, l3)
    det = (l1 * l3) ** 2
    return s22 / det, -s12 / det, s11 / det


def mahalanobis_sq(dx, dy, l1, l2, l3):
    A, B, C = conic(l1, l2, l3)
    return A * dx * dx + 2.0 * B * dx * dy + C * dy * dy


def box_halfwidths(l1, l2, l3):
    """Half-widths of the axis-aligned box around the q <= 9 ellipse:
    3 * sqrt(Sigma_11) and 3 * sqrt(Sigma_22)."""
    s11, _, s22 = covariance(l1, l2, l3)
    return 3.0 * np.sqrt(s11), 3.0 * np.sqrt(s22)
