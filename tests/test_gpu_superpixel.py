"""GPU parity of the superpixel ROI initialisation (Sec. 3.2.A, Fig. 2).

Seeds and the Gaussians empty segments keep come from the oracle's
content-aware initialiser (inputs, not results).  Labels and centres are
integer or exactly specified decisions and the segment Gaussians are FP64
formulas of exact integer moments rounded once, so every comparison is
bit-exact.  At 1920x1080 the oracle cannot run the whole clustering, so one
round is compared on sampled pixels and on sampled segments (the oracle
assigns every pixel of their windows itself), and the ten-round
configuration is checked by the relations that define each round, on
sampled pixels and segments: every label is the argmin of the distance over
its candidates for the centres that round started from, and every new
centre and segment Gaussian is the one the labelled pixels define."""
import numpy as np
import pytest
import torch

from oracle.init import init_from_frame
from oracle.superpixel import (assign, colour_codes, compactness_weight, grid_step, kmeans,
                               segment_gaussians, segment_sums, update_centres)
from paper_2505_09324_amd import _lib, synth
from gpu_util import DEV, dev, host

pytestmark = pytest.mark.gpu

F32 = np.float32


def _inputs(W, H, N, seed, mask=None):
    frame, m = synth.make_frame(W, H, seed=seed)
    if mask is None:
        mask = m
    d = synth.init_draws(N, seed=seed + 1)
    ox, oc, orgb, info = init_from_frame(frame, mask, d)
    K = d.pick_roi.shape[0]
    return frame, mask, info["picked"][:K].astype(np.int32), (ox[:K], oc[:K], orgb[:K])


def _gpu(frame, mask, seeds, fb, iters, m):
    H, W = mask.shape
    K = len(seeds)
    xy, chol, rgb = (dev(np.ascontiguousarray(a, F32)) for a in fb)
    labels = torch.full((H, W), -7, dtype=torch.int32, device=DEV)
    centres = torch.zeros(2, 5, K, device=DEV)
    _lib.init_superpixel(dev(frame), dev(mask.astype(np.uint8)), dev(seeds), xy, chol, rgb,
                         iters=iters, compactness=m, labels=labels, centres=centres)
    torch.cuda.synchronize()
    return host(labels), host(centres), host(xy), host(chol), host(rgb)


def _compare_whole(frame, mask, seeds, fb, iters, m):
    lab, cen, gx, gc, gr = _gpu(frame, mask, seeds, fb, iters, m)
    xy_seeds = np.stack([seeds % frame.shape[2], seeds // frame.shape[2]], 1)
    olab, (px, py, pc), (cx, cy, cc), S = kmeans(frame, mask, xy_seeds, iters=iters, m=m)
    np.testing.assert_array_equal(lab, olab)
    np.testing.assert_array_equal(cen[0, 0], px)
    np.testing.assert_array_equal(cen[0, 1], py)
    np.testing.assert_array_equal(cen[0, 2:].T, pc)
    np.testing.assert_array_equal(cen[1, 0], cx)
    np.testing.assert_array_equal(cen[1, 1], cy)
    np.testing.assert_array_equal(cen[1, 2:].T, cc)
    ox, oc, orgb = segment_gaussians(segment_sums(olab, colour_codes(frame), len(seeds)), fb)
    np.testing.assert_array_equal(gx, ox)
    np.testing.assert_array_equal(gc, oc)
    np.testing.assert_array_equal(gr, orgb)
    return olab


@pytest.mark.parametrize("W,H,N,iters,m", [(96, 64, 300, 5, 0.1), (130, 77, 2000, 4, 0.05),
                                           (200, 120, 800, 6, 0.3)])
def test_superpixel_small_frames(W, H, N, iters, m):
    print(f"superpixel {W}x{H} N={N} iters={iters} m={m}", flush=True)
    frame, mask, seeds, fb = _inputs(W, H, N, seed=9)
    lab = _compare_whole(frame, mask, seeds, fb, iters, m)
    assert np.all(lab[~mask] == -1)


def test_superpixel_edge_cases():
    print("superpixel edge cases", flush=True)
    frame, mask, seeds, fb = _inputs(50, 40, 120, seed=3)
    # empty ROI mask: the whole frame
    _compare_whole(frame, np.zeros((40, 50), bool), seeds, fb, 3, 0.1)
    # full ROI, one round
    _compare_whole(frame, np.ones((40, 50), bool), seeds, fb, 1, 0.1)
    # duplicated seeds: the later copy is empty after one round and keeps its Gaussian
    dup = seeds.copy()
    dup[1] = dup[0]
    lab = _compare_whole(frame, mask, dup, fb, 1, 0.1)
    assert not np.any(lab == 1)
    # one seed: the window is the whole frame
    _compare_whole(frame, mask, seeds[:1], tuple(a[:1] for a in fb), 3, 0.1)
    # one-pixel ROI and a single-row frame
    one = np.zeros((40, 50), bool)
    one[17, 23] = True
    _compare_whole(frame, one, np.array([17 * 50 + 23], np.int32), tuple(a[:1] for a in fb), 2, 0.1)
    f1, m1, s1, fb1 = _inputs(64, 1, 20, seed=5, mask=np.ones((1, 64), bool))
    _compare_whole(f1, m1, s1, fb1, 3, 0.2)


def _window_labels(frame, roi, cx, cy, cc, S, w, k):
    """The oracle's labels of every pixel of centre k's 3S x 3S window."""
    H, W = roi.shape
    gx, gy = int(np.floor(cx[k] / F32(S))), int(np.floor(cy[k] / F32(S)))
    xs = np.arange(max((gx - 1) * S, 0), min((gx + 2) * S, W))
    ys = np.arange(max((gy - 1) * S, 0), min((gy + 2) * S, H))
    X, Y = np.meshgrid(xs, ys)
    X, Y = X.ravel(), Y.ravel()
    inside = roi[Y, X]
    lab = np.full((H, W), -1, np.int64)
    pix = np.stack([X[inside], Y[inside]], 1)
    lab[pix[:, 1], pix[:, 0]] = assign(frame, roi, cx, cy, cc, S, w, pixels=pix)
    return lab


def _segment_from(lab, frame, k, K, fb):
    one = np.where(lab == k, k, -1)
    return segment_gaussians(segment_sums(one, colour_codes(frame), K), fb)


def test_superpixel_full_hd():
    """1920x1080, 30,000 draws with 70 % in the ROI (21,000 segments): the
    configuration the 1080p initialisation uses (10 rounds, m = 0.1)."""
    print("superpixel 1080p", flush=True)
    W, H = 1920, 1080
    frame, mask, seeds, fb = _inputs(W, H, 30000, seed=201)
    K = len(seeds)
    S = grid_step(int(mask.sum()), K)
    w = compactness_weight(0.1, S)
    rng = np.random.default_rng(7)
    ys, xs = np.nonzero(mask)
    pick = rng.choice(len(xs), 20000, replace=False)
    pix = np.stack([xs[pick], ys[pick]], 1)
    seg = rng.choice(K, 40, replace=False)

    # one round: oracle parity from the seeds
    lab, cen, gx, gc, gr = _gpu(frame, mask, seeds, fb, 1, 0.1)
    sx = (seeds % W + 0.5).astype(F32)
    sy = (seeds // W + 0.5).astype(F32)
    codes = colour_codes(frame)
    sc = (codes[:, seeds // W, seeds % W].T / 65536).astype(F32)
    np.testing.assert_array_equal(cen[0, 0], sx)
    np.testing.assert_array_equal(cen[0, 2:].T, sc)
    np.testing.assert_array_equal(lab[pix[:, 1], pix[:, 0]],
                                  assign(frame, mask, sx, sy, sc, S, w, pixels=pix))
    assert np.all(lab[~mask] == -1)
    for k in seg:
        ox, oc, orgb = _segment_from(_window_labels(frame, mask, sx, sy, sc, S, w, k), frame, k, K,
                                     fb)
        np.testing.assert_array_equal(gx[k], ox[k])
        np.testing.assert_array_equal(gc[k], oc[k])
        np.testing.assert_array_equal(gr[k], orgb[k])

    # ten rounds: the relations that define the last round
    lab, cen, gx, gc, gr = _gpu(frame, mask, seeds, fb, 10, 0.1)
    px_, py_, pc_ = cen[0, 0], cen[0, 1], np.ascontiguousarray(cen[0, 2:].T)
    np.testing.assert_array_equal(lab[pix[:, 1], pix[:, 0]],
                                  assign(frame, mask, px_, py_, pc_, S, w, pixels=pix))
    sums = segment_sums(lab, codes, K)
    assert sums["n"].sum() == (lab >= 0).sum()
    nx, ny, nc = update_centres(sums, px_, py_, pc_)
    np.testing.assert_array_equal(cen[1, 0], nx)
    np.testing.assert_array_equal(cen[1, 1], ny)
    np.testing.assert_array_equal(cen[1, 2:].T, nc)
    ox, oc, orgb = segment_gaussians(sums, fb)
    np.testing.assert_array_equal(gx, ox)
    np.testing.assert_array_equal(gc, oc)
    np.testing.assert_array_equal(gr, orgb)
