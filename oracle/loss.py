"""Fitting loss, its image gradient and PSNR, in FP64.

The paper never names the fitting loss; the loop is read as minimising the
mean squared error over all 3*H*W values of the unclamped render, and
quality is reported as PSNR with peak value 1 over the full frame
(Sec. 4: PSNR is the quality axis of every result).
"""
from __future__ import annotations

import math

import numpy as np


def mse(img, target) -> float:
    r = np.asarray(img, np.float64) - np.asarray(target, np.float64)
    return float(np.sum(r * r) / r.size)


def dloss_dimg(img, target) -> np.ndarray:
    """d(MSE)/dC = 2 (C - T) / (3 H W)."""
    r = np.asarray(img, np.float64) - np.asarray(target, np.float64)
    return 2.0 * r / r.size


def psnr_from_mse(m: float) -> float:
    """10 log10(1 / MSE); +inf for a perfect fit."""
    if m <= 0.0:
        return math.inf
    return 10.0 * math.log10(1.0 / m)


def psnr(img, target) -> float:
    return psnr_from_mse(mse(img, target))


def psnr_clamped(img, target) -> float:
    return psnr(np.clip(np.asarray(img, np.float64), 0.0, 1.0), target)
