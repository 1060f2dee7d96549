"""Pins of the superpixel-initialisation oracle (Sec. 3.2.A, Fig. 2)."""
import math

import numpy as np

from oracle.render import render_bruteforce
from oracle.superpixel import (MASS, assign, compactness_weight, grid_step, kmeans,
                               segment_gaussians, segment_sums, colour_codes)

F32 = np.float32


def _flat(H, W, colour):
    return np.broadcast_to(np.asarray(colour, F32)[:, None, None], (3, H, W)).copy()


def test_one_segment_is_the_uniform_rectangle():
    """A w x h rectangle of one colour as the ROI with one seed: the segment
    is the rectangle, its covariance that of the continuous uniform
    rectangle (w^2/12, 0, h^2/12) and its colour c 6 / (pi MASS); the render
    of that Gaussian carries the rectangle's total colour (to the 1 % the
    pixel grid allows)."""
    H, W, x0, y0, w, h = 40, 50, 10, 8, 24, 16
    roi = np.zeros((H, W), bool)
    roi[y0:y0 + h, x0:x0 + w] = True
    c = [0.25, 0.5, 0.75]
    frame = _flat(H, W, c)
    lab, _, _, S = kmeans(frame, roi, [[20, 15]], iters=3, m=0.1)
    assert np.all(lab[roi] == 0) and np.all(lab[~roi] == -1)
    sums = segment_sums(lab, colour_codes(frame), 1)
    fb = (np.zeros((1, 2)), np.ones((1, 3)), np.zeros((1, 3)))
    xy, chol, rgb = segment_gaussians(sums, fb)
    np.testing.assert_allclose(xy[0], [x0 + w / 2, y0 + h / 2], rtol=0, atol=0)
    np.testing.assert_allclose(chol[0], [w / math.sqrt(12), 0, h / math.sqrt(12)], rtol=1e-6)
    np.testing.assert_allclose(rgb[0], np.array(c) * 6 / (math.pi * MASS), rtol=1e-6)
    img = render_bruteforce(xy.astype(np.float64), chol.astype(np.float64),
                            rgb.astype(np.float64), H, W)["img"]
    np.testing.assert_allclose(img.sum(axis=(1, 2)), np.array(c) * w * h, rtol=1e-2)


def test_two_colours_split_into_their_halves():
    H, W = 20, 32
    roi = np.zeros((H, W), bool)
    roi[2:18, 4:28] = True
    frame = _flat(H, W, [0.1, 0.1, 0.1])
    frame[:, :, 16:] = 0.9
    lab, _, (cx, cy, col), S = kmeans(frame, roi, [[10, 9], [20, 9]], iters=4, m=0.01)
    assert np.all(lab[2:18, 4:16] == 0) and np.all(lab[2:18, 16:28] == 1)
    np.testing.assert_array_equal(cx, F32([10.0, 22.0]))      # (4..15) and (16..27) centres
    np.testing.assert_array_equal(cy, F32([10.0, 10.0]))
    np.testing.assert_allclose(col[:, 0], [0.1, 0.9], atol=1e-5)


def test_ties_go_to_the_lower_index_and_far_cells_are_never_candidates():
    frame = _flat(4, 60, [0.5, 0.5, 0.5])
    roi = np.ones((4, 60), bool)
    S = 4
    w = compactness_weight(0.5, S)
    # pixel (10, 1) at (10.5, 1.5): centres at (8.5, 1.5) and (12.5, 1.5) tie
    cx = F32([12.5, 8.5, 40.5])
    cy = F32([1.5, 1.5, 1.5])
    col = np.full((3, 3), 0.5, F32)
    assert assign(frame, roi, cx, cy, col, S, w, pixels=[[10, 1]])[0] == 0
    cx2 = F32([8.5, 12.5, 40.5])
    assert assign(frame, roi, cx2, cy, col, S, w, pixels=[[10, 1]])[0] == 0
    # only centre 2 matches the pixel's colour, but it is many cells away
    f2 = frame.copy()
    f2[:, 1, 10] = 0.0
    col2 = col.copy()
    col2[2] = 0.0
    assert assign(f2, roi, cx, cy, col2, S, w, pixels=[[10, 1]])[0] in (0, 1)
    assert assign(f2, roi, F32([12.5, 8.5, 14.5]), cy, col2, S, w, pixels=[[10, 1]])[0] == 2


def test_empty_segment_keeps_its_fallback_and_moments_match_numpy():
    rng = np.random.default_rng(2)
    H, W = 30, 36
    roi = np.zeros((H, W), bool)
    yy, xx = np.mgrid[0:H, 0:W]
    roi[((xx - 18) / 14.0) ** 2 + ((yy - 15) / 12.0) ** 2 <= 1] = True
    frame = rng.uniform(0, 1, (3, H, W)).astype(F32)
    seeds = [[18, 15], [18, 15], [10, 12], [26, 18], [18, 6]]   # seed 1 duplicates seed 0
    # one round: every pixel that ties between seeds 0 and 1 joins 0
    lab, _, _, S = kmeans(frame, roi, seeds, iters=1, m=0.2)
    K = len(seeds)
    sums = segment_sums(lab, colour_codes(frame), K)
    assert sums["n"][1] == 0 and sums["n"].sum() == roi.sum()
    fb = (np.full((K, 2), 7.0), np.full((K, 3), 2.0), np.full((K, 3), 0.3))
    xy, chol, rgb = segment_gaussians(sums, fb)
    np.testing.assert_array_equal(xy[1], [7, 7])
    np.testing.assert_array_equal(chol[1], [2, 2, 2])
    for k in (0, 2, 3, 4):
        ys, xs = np.nonzero(lab == k)
        cov = np.cov(np.stack([xs, ys]).astype(np.float64), bias=True) + np.eye(2) / 12
        L = np.linalg.cholesky(cov)
        np.testing.assert_allclose(chol[k], [L[0, 0], L[1, 0], L[1, 1]], rtol=1e-5)
        np.testing.assert_allclose(xy[k], [xs.mean() + 0.5, ys.mean() + 0.5], rtol=1e-6)
        mean = frame[:, ys, xs].astype(np.float64).mean(axis=1)
        np.testing.assert_allclose(rgb[k], mean * len(xs) / (2 * math.pi * L[0, 0] * L[1, 1] * MASS),
                                   rtol=1e-4)
    assert grid_step(int(roi.sum()), K) == S


def test_assignment_is_the_argmin_of_the_slic_distance():
    """With a grid step that puts every centre in the window, the choice is
    the argmin over all centres of |colour - c_k|^2 + (m/S)^2 |p - xy_k|^2
    (brute force in FP64; near-ties skipped)."""
    rng = np.random.default_rng(5)
    H, W, K, S, m = 12, 14, 9, 16, 0.7
    frame = rng.uniform(0, 1, (3, H, W)).astype(F32)
    roi = np.ones((H, W), bool)
    cx = rng.uniform(0, W, K).astype(F32)
    cy = rng.uniform(0, H, K).astype(F32)
    col = rng.uniform(0, 1, (K, 3)).astype(F32)
    lab = assign(frame, roi, cx, cy, col, S, compactness_weight(m, S))
    checked = 0
    for y in range(H):
        for x in range(W):
            d = ((frame[:, y, x].astype(np.float64)[None] - col) ** 2).sum(1) \
                + (m * m / (S * S)) * ((x + 0.5 - cx) ** 2 + (y + 0.5 - cy) ** 2)
            o = np.sort(d)
            if o[1] - o[0] > 1e-5 * o[1]:
                assert lab[y, x] == np.argmin(d)
                checked += 1
    assert checked > 0.9 * H * W
    assert grid_step(1000, 10) == 10 and grid_step(5, 10) == 1 and grid_step(1000, 7) == 12


def test_empty_roi_is_the_whole_frame():
    frame = np.random.default_rng(3).uniform(0, 1, (3, 10, 12)).astype(F32)
    a = kmeans(frame, np.zeros((10, 12), bool), [[2, 2], [9, 7]], iters=2, m=0.3)
    b = kmeans(frame, np.ones((10, 12), bool), [[2, 2], [9, 7]], iters=2, m=0.3)
    np.testing.assert_array_equal(a[0], b[0])
    assert np.all(a[0] >= 0) and a[3] == b[3] == 8
