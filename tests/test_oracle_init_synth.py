"""Pins for the synthetic inputs and the oracle's content-aware init."""
import hashlib
import math

import numpy as np
import pytest
from scipy.stats import chisquare

from oracle.init import KAPPA, gradient_levels, init_from_frame
from oracle.render import render_box
from paper_2505_09324_amd import synth


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


def test_frame_deterministic_and_in_range():
    a, ma = synth.make_frame(96, 64, seed=101)
    b, mb = synth.make_frame(96, 64, seed=101)
    c, _ = synth.make_frame(96, 64, seed=102)
    assert _digest(a) == _digest(b) and np.array_equal(ma, mb)
    assert _digest(a) != _digest(c)
    assert a.dtype == np.float32 and a.shape == (3, 64, 96)
    assert a.min() >= 0.0 and a.max() <= 1.0


@pytest.mark.slow
def test_roi_fraction_1080p():
    """P14: the elliptical subject covers pi*0.19*0.42 = 25.07 % of the frame."""
    _, m = synth.make_frame(1920, 1080, seed=201)
    assert abs(m.mean() - math.pi * 0.19 * 0.42) < 0.002


def test_background_is_planar_away_from_subject():
    f, m = synth.make_frame(200, 120, seed=5)
    bg = f[:, :, :20].astype(np.float64)     # left strip, outside the subject
    d2x = bg[:, :, 2:] - 2 * bg[:, :, 1:-1] + bg[:, :, :-2]
    d2y = bg[:, 2:, :] - 2 * bg[:, 1:-1, :] + bg[:, :-2, :]
    assert np.abs(d2x).max() < 1e-6 and np.abs(d2y).max() < 1e-6
    assert not m[:, :20].any()


def test_sequence_motion():
    frames, masks = synth.make_sequence(160, 90, seed=301, n_frames=3)
    assert not np.array_equal(masks[0], masks[1])
    # background pixels far from the subject never change
    np.testing.assert_array_equal(frames[0][:, :, :5], frames[2][:, :, :5])


def test_batch_counts_affine_in_area():
    assert [synth.batch_gaussian_count(w, h) for w, h in synth.BATCH_SIZES] == [3000, 8423, 22885, 50000]


def test_gradient_levels_flat_and_ramp():
    flat = np.full((3, 8, 9), 0.25, np.float32)
    assert not gradient_levels(flat).any()
    ramp = np.zeros((3, 6, 10), np.float32)
    ramp[0] = np.arange(10, dtype=np.float32)[None, :] * np.float32(0.125)
    q = gradient_levels(ramp)
    # central difference of a ramp of slope 1/8 is 1/4 everywhere (borders
    # use twice the one-sided difference): floor(1024 * 0.25) = 256
    assert np.all(q == 256)


def test_sampler_follows_pmf_chi_square():
    """P13: 1e5 draws vs the stated pmf on a 32x32 frame (p > 1e-3)."""
    rng = np.random.default_rng(0)
    f = rng.uniform(size=(3, 32, 32)).astype(np.float32)
    mask = np.zeros((32, 32), bool)
    mask[8:24, 6:26] = True
    draws = synth.init_draws(100000, seed=77, roi_fraction=1.0)
    _, _, _, info = init_from_frame(f, mask, draws)
    q = gradient_levels(f).reshape(-1)[mask.reshape(-1)]
    w = q + info["base"] + 1
    roi_idx = np.nonzero(mask.reshape(-1))[0]
    pos = {p: i for i, p in enumerate(roi_idx)}
    counts = np.bincount([pos[p] for p in info["picked"]], minlength=roi_idx.size)
    expect = w / w.sum() * counts.sum()
    assert chisquare(counts, expect).pvalue > 1e-3


def test_init_deterministic_and_split():
    f, m = synth.make_frame(80, 60, seed=9)
    d = synth.init_draws(300, seed=10)
    a = init_from_frame(f, m, d)
    b = init_from_frame(f, m, d)
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)
    picked = a[3]["picked"]
    flat = m.reshape(-1)
    assert flat[picked[:210]].all() and not flat[picked[210:]].any()
    xy = a[0]
    assert np.all(np.abs(xy[:, 0] - (picked % 80 + 0.5)) <= 0.5)
    assert np.all(np.abs(xy[:, 1] - (picked // 80 + 0.5)) <= 0.5)


def test_flat_frame_renders_its_colour():
    """kappa: Gaussians at the sampling density over a flat region render the
    region's colour on average (interior mean within 5 %)."""
    H = W = 96
    col = np.array([0.2, 0.5, 0.8], np.float32)
    f = np.broadcast_to(col[:, None, None], (3, H, W)).copy()
    mask = np.zeros((H, W), bool)
    mask[:, : W // 2] = True
    # equal counts in equal halves: one density over the whole frame; the
    # interior mean then has ~1/sqrt(#Gaussians) = 2.5 % sampling noise
    d = synth.init_draws(4000, seed=3, roi_fraction=0.5)
    xy, chol, rgb, _ = init_from_frame(f, mask, d)
    img = render_box(xy, chol, rgb, H, W, want_bounds=False)["img"]
    inner = img[:, 8:-8, 8:-8].mean(axis=(1, 2))
    np.testing.assert_allclose(inner, col, rtol=0.05)
    assert KAPPA == pytest.approx(0.6437, abs=1e-4)
