"""Tile binning of Gaussians, specified in FP32.

The method renders with the tile-based rasteriser it inherits (Sec. 3,
"differentiable tile-based rasterization"; no depth order is needed because
Eq. 2 is an order-free sum).  A tile list is an integer decision made from
floating-point geometry, so this part of the oracle is written in FP32 with a
fixed operation order, round-to-nearest-even and no fused multiply-add, the
same decision the GPU takes:

    a = l2*l2;  b = l3*l3;  s = a + b;  r = sqrt(s)        (correctly rounded)
    ry = 3*r;   rx = 3*|l1|
    xlo = mx - rx;  xhi = mx + rx;  ylo = my - ry;  yhi = my + ry
    fx0 = floor(xlo / T);  fx1 = floor(xhi / T)  (exact: T is a power of two)
    empty iff fx1 < 0 or fx0 > TX-1 or fy1 < 0 or fy0 > TY-1
    tx0 = max(fx0, 0);  tx1 = min(fx1, TX-1)   (same in y)

rx and ry are the exact half-widths of the box around the q <= 9 ellipse
(3 sqrt(Sigma_11) and 3 sqrt(Sigma_22) with Sigma = L L^T, Eq. 1).  Within a
tile the Gaussians are listed by ascending index.  The list is built here by
enumerating every (tile, index) pair and sorting with Python's ``sorted`` --
no radix sort, no scan.
"""
from __future__ import annotations

import math

import numpy as np

from .gauss import CUTOFF_Q, AMBIGUOUS_BAND, culled, mahalanobis_sq

F32 = np.float32


def tile_grid(W: int, H: int, T: int):
    return (W + T - 1) // T, (H + T - 1) // T


def _floor_div_f32(v: np.float32, T: int) -> float:
    q = F32(v) / F32(T)
    return math.floor(q) if math.isfinite(q) else float(q)


def tile_rect(mx, my, l1, l2, l3, W: int, H: int, T: int):
    """(tx0, tx1, ty0, ty1) inclusive, or None if the Gaussian hits no tile.

    Inputs are float32 scalars; every operation below is FP32.
    """
    TX, TY = tile_grid(W, H, T)
    mx, my, l1, l2, l3 = F32(mx), F32(my), F32(l1), F32(l2), F32(l3)
    with np.errstate(over="ignore", invalid="ignore"):
        a = l2 * l2
        b = l3 * l3
        s = a + b
        r = np.sqrt(s)
        ry = F32(3.0) * r
        rx = F32(3.0) * np.abs(l1)
        xlo = mx - rx
        xhi = mx + rx
        ylo = my - ry
        yhi = my + ry
    fx0 = _floor_div_f32(xlo, T)
    fx1 = _floor_div_f32(xhi, T)
    fy0 = _floor_div_f32(ylo, T)
    fy1 = _floor_div_f32(yhi, T)
    if fx1 < 0 or fx0 > TX - 1 or fy1 < 0 or fy0 > TY - 1:
        return None
    tx0 = int(max(fx0, 0))
    tx1 = int(min(fx1, TX - 1))
    ty0 = int(max(fy0, 0))
    ty1 = int(min(fy1, TY - 1))
    return tx0, tx1, ty0, ty1


def bin_gaussians(xy, chol, W: int, H: int, T: int):
    """Tile lists of all Gaussians.

    Returns dict with
      counts     [N]      int64   tiles touched by each Gaussian
      pair_ids   [P]      int64   Gaussian index of each pair, ordered by
                                  ascending (tile, index)
      pair_tiles [P]      int64   tile of each pair
      tile_start [TX*TY+1] int64  first pair index whose tile is >= t
      n_pairs    int
    """
    xy = np.asarray(xy, np.float32)
    chol = np.asarray(chol, np.float32)
    N = xy.shape[0]
    TX, TY = tile_grid(W, H, T)
    dead = culled(xy, chol)
    counts = np.zeros(N, np.int64)
    pairs = []
    for n in range(N):
        if dead[n]:
            continue
        rect = tile_rect(xy[n, 0], xy[n, 1], chol[n, 0], chol[n, 1], chol[n, 2], W, H, T)
        if rect is None:
            continue
        tx0, tx1, ty0, ty1 = rect
        counts[n] = (tx1 - tx0 + 1) * (ty1 - ty0 + 1)
        for ty in range(ty0, ty1 + 1):
            for tx in range(tx0, tx1 + 1):
                pairs.append((ty * TX + tx, n))
    pairs = sorted(pairs)
    n_pairs = len(pairs)
    pair_tiles = np.array([p[0] for p in pairs], np.int64)
    pair_ids = np.array([p[1] for p in pairs], np.int64)
    tile_start = np.searchsorted(pair_tiles, np.arange(TX * TY + 1), side="left")
    return {"counts": counts, "pair_ids": pair_ids, "pair_tiles": pair_tiles,
            "tile_start": tile_start.astype(np.int64), "n_pairs": n_pairs,
            "TX": TX, "TY": TY}


def tile_lists(bins) -> list:
    """List of per-tile Gaussian index arrays."""
    ts = bins["tile_start"]
    return [bins["pair_ids"][ts[t]:ts[t + 1]] for t in range(len(ts) - 1)]


def required_pairs(xy, chol, W: int, H: int, T: int):
    """Brute-force FP64 set of (tile, n) pairs that any correct binning must
    contain: some pixel centre of the tile has q <= 9 - 1e-4."""
    xy = np.asarray(xy, np.float64)
    chol = np.asarray(chol, np.float64)
    TX, TY = tile_grid(W, H, T)
    dead = culled(xy, chol)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    tile_of = (ys // T).astype(np.int64) * TX + (xs // T).astype(np.int64)
    need = set()
    for n in range(xy.shape[0]):
        if dead[n]:
            continue
        q = mahalanobis_sq(xs + 0.5 - xy[n, 0], ys + 0.5 - xy[n, 1], *chol[n])
        hit = q <= CUTOFF_Q - AMBIGUOUS_BAND
        for t in np.unique(tile_of[hit]):
            need.add((int(t), n))
    return need
