"""Pins for the oracle's forward render (Eq. 1, Eq. 2; Sec. 3.1).

Each test checks the oracle against something other than itself: a library
density (scipy), a closed-form integral, an exact boundary value, or the
second oracle implementation.
"""
import math

import numpy as np
import pytest
from scipy.stats import multivariate_normal

from oracle.render import render_box, render_bruteforce, count_pairs_in_cutoff
from paper_2505_09324_amd import synth


def _sigma(l):
    L = np.array([[l[0], 0.0], [l[1], l[2]]])
    return L @ L.T


@pytest.mark.parametrize("l", [(2.0, 0.0, 1.5), (1.3, 0.9, 0.7), (3.0, -2.0, 1.0)])
def test_single_gaussian_matches_scipy_density(l):
    """P1: w = pdf(x) * 2 pi sqrt(det Sigma) at pixel centres, cut at q <= 9."""
    H, W = 24, 28
    mu = np.array([13.3, 11.7])
    c = np.array([0.7, -0.2, 1.5])
    S = _sigma(l)
    rv = multivariate_normal(mean=mu, cov=S)
    ys, xs = np.mgrid[0:H, 0:W]
    pts = np.stack([xs + 0.5, ys + 0.5], -1).reshape(-1, 2)
    dens = rv.pdf(pts) * 2 * math.pi * math.sqrt(np.linalg.det(S))
    Si = np.linalg.inv(S)
    d = pts - mu
    q = np.einsum("pi,ij,pj->p", d, Si, d)
    w = np.where(q <= 9.0, dens, 0.0).reshape(H, W)
    out = render_bruteforce(mu[None], np.array([l]), c[None], H, W)["img"]
    for k in range(3):
        np.testing.assert_allclose(out[k], c[k] * w, rtol=1e-12, atol=1e-14)


def test_transposed_cholesky_differs():
    """Sigma = L L^T, not L^T L: with l2 != 0 the two give different images."""
    l = (1.3, 0.9, 0.7)
    a = render_bruteforce(np.array([[10.0, 10.0]]), np.array([l]), np.ones((1, 3)), 20, 20)["img"]
    L = np.array([[l[0], 0.0], [l[1], l[2]]])
    S_wrong = L.T @ L
    # the Cholesky factor of the wrong covariance, as an l vector
    Lw = np.linalg.cholesky(S_wrong)
    b = render_bruteforce(np.array([[10.0, 10.0]]), np.array([[Lw[0, 0], Lw[1, 0], Lw[1, 1]]]),
                          np.ones((1, 3)), 20, 20)["img"]
    assert np.abs(a - b).max() > 1e-2


@pytest.mark.parametrize("l", [(2.0, 0.5, 1.5), (3.0, -1.0, 2.5), (1.6, 0.0, 1.6)])
def test_mass_closed_form(l):
    """P3: sum over pixels ~ c' 2 pi |l1 l3| (1 - e^-4.5) (chi-square, 2 dof)."""
    H = W = 64
    c = 0.8
    img = render_bruteforce(np.array([[32.2, 31.9]]), np.array([l]),
                            np.array([[c, c, c]]), H, W)["img"]
    expect = c * 2 * math.pi * abs(l[0] * l[2]) * (1 - math.exp(-4.5))
    assert abs(img[0].sum() - expect) / expect < 0.01


def test_cutoff_boundary_is_inclusive():
    """P4: q = 9 exactly is admitted with weight e^-4.5; just beyond is not."""
    W = H = 16
    c = np.array([[1.0, 2.0, 3.0]])
    l = np.array([[2.0, 0.0, 2.0]])
    on = render_bruteforce(np.array([[2.5, 8.5]]), l, c, H, W)["img"]
    assert on[0, 8, 8] == pytest.approx(math.exp(-4.5), rel=1e-15)
    assert on[2, 8, 8] == pytest.approx(3 * math.exp(-4.5), rel=1e-15)
    off = render_bruteforce(np.array([[2.5 - 2.0 ** -10, 8.5]]), l, c, H, W)["img"]
    assert off[0, 8, 8] == 0.0


def test_additive_and_permutation_invariant():
    """P2: render(S1 u S2) = render(S1) + render(S2); order does not matter."""
    xy, chol, rgb = synth.random_gaussians(40, 48, 40, seed=7)
    chol[:, 1] = np.linspace(-1, 1, 40)
    full = render_bruteforce(xy, chol, rgb, 40, 48)["img"]
    a = render_bruteforce(xy[:17], chol[:17], rgb[:17], 40, 48)["img"]
    b = render_bruteforce(xy[17:], chol[17:], rgb[17:], 40, 48)["img"]
    np.testing.assert_allclose(full, a + b, rtol=1e-13, atol=1e-14)
    p = np.random.default_rng(3).permutation(40)
    perm = render_bruteforce(xy[p], chol[p], rgb[p], 40, 48)["img"]
    np.testing.assert_allclose(full, perm, rtol=1e-13, atol=1e-14)


def test_box_render_equals_bruteforce():
    """O-2 (per-Gaussian box) == O-1 (all pixels x all Gaussians)."""
    xy, chol, rgb = synth.random_gaussians(120, 64, 48, seed=11, scale_lo=0.4, scale_hi=6.0)
    chol[:, 1] = np.random.default_rng(5).uniform(-3, 3, size=120)
    xy[:5] = [[-3.0, 5.0], [70.0, 10.0], [30.0, -6.0], [30.0, 52.0], [0.0, 0.0]]
    a = render_bruteforce(xy, chol, rgb, 48, 64)
    b = render_box(xy, chol, rgb, 48, 64)
    for k in ("img", "abs", "amb"):
        np.testing.assert_allclose(a[k], b[k], rtol=1e-12, atol=1e-13)


def test_culled_gaussians_contribute_nothing():
    xy = np.array([[5.0, 5.0], [np.nan, 5.0], [5.0, 5.0], [5.0, 5.0]])
    chol = np.array([[1.0, 0, 1.0], [1.0, 0, 1.0], [0.0, 0, 1.0], [1.0, np.inf, 1.0]])
    rgb = np.ones((4, 3))
    img = render_bruteforce(xy, chol, rgb, 10, 10)["img"]
    one = render_bruteforce(xy[:1], chol[:1], rgb[:1], 10, 10)["img"]
    np.testing.assert_array_equal(img, one)


def test_empty_set_renders_black():
    img = render_bruteforce(np.zeros((0, 2)), np.zeros((0, 3)), np.zeros((0, 3)), 5, 7)["img"]
    assert img.shape == (3, 5, 7) and not img.any()


def test_pairs_in_cutoff_matches_ellipse_area():
    """Number of admitted pixels ~ area of the q<=9 ellipse, 9 pi |l1 l3|."""
    l = (4.0, 1.0, 3.0)
    n = count_pairs_in_cutoff(np.array([[50.3, 50.1]]), np.array([l]), 100, 100)
    assert abs(n - 9 * math.pi * 12.0) / (9 * math.pi * 12.0) < 0.02


def test_render_pixels_equals_bruteforce_at_sampled_pixels():
    """The per-pixel evaluator that checks large frames: at sampled pixels
    (corners and edges included) it must give the brute-force image, the
    absolute sum and the ambiguity-band mass, with culled Gaussians (NaN,
    inf, |l1| or |l3| below 2^-14), off-frame means and huge, sheared and
    negative-diagonal Gaussians in the set."""
    from oracle.render import render_pixels
    W, H, N = 57, 43, 160
    xy, chol, rgb = synth.random_gaussians(N, W, H, seed=21, scale_lo=0.3, scale_hi=7.0)
    rng = np.random.default_rng(22)
    chol[:, 1] = rng.uniform(-4, 4, N)
    chol[::9, 0] *= -1
    chol[::11, 2] *= -1
    xy[:12] = rng.uniform(-25, 80, size=(12, 2))
    xy[12] = [np.nan, 3.0]
    chol[13] = [np.inf, 0.0, 1.0]
    chol[14] = [0.5 * 2.0 ** -14, 0.0, 2.0]
    chol[15] = [2.0, 0.0, 0.0]
    chol[16] = [60.0, -20.0, 45.0]
    rgb[:] = rng.uniform(-1.0, 1.0, (N, 3))
    full = render_bruteforce(xy, chol, rgb, H, W)
    px = np.concatenate([rng.integers(0, W, 200), [0, W - 1, 0, W - 1]])
    py = np.concatenate([rng.integers(0, H, 200), [0, 0, H - 1, H - 1]])
    got = render_pixels(xy, chol, rgb, px, py)
    for k in ("img", "abs", "amb"):
        np.testing.assert_allclose(got[k], full[k][:, py, px], rtol=1e-12, atol=1e-14)
    assert np.any(full["img"][:, py, px] != 0.0)


def test_render_pixels_single_gaussian_matches_scipy_density():
    """P1 at arbitrary pixels: one Gaussian's value is c' times the scipy
    normal density scaled by 2 pi sqrt(det Sigma), cut at q <= 9 computed
    from numpy's inverse of L L^T."""
    from oracle.render import render_pixels
    l = (2.3, -1.1, 1.4)
    mu = np.array([31.7, 18.2])
    c = np.array([0.6, -0.4, 1.2])
    S = _sigma(l)
    rv = multivariate_normal(mean=mu, cov=S)
    rng = np.random.default_rng(23)
    px = rng.integers(20, 44, 400)
    py = rng.integers(10, 27, 400)
    pts = np.stack([px + 0.5, py + 0.5], -1)
    d = pts - mu
    q = np.einsum("pi,ij,pj->p", d, np.linalg.inv(S), d)
    w = np.where(q <= 9.0, rv.pdf(pts) * 2 * math.pi * math.sqrt(np.linalg.det(S)), 0.0)
    got = render_pixels(mu[None], np.array([l]), c[None], px, py)["img"]
    assert np.count_nonzero(w) > 50 and np.count_nonzero(w == 0.0) > 50
    for k in range(3):
        np.testing.assert_allclose(got[k], c[k] * w, rtol=1e-12, atol=1e-15)
