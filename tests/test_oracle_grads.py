"""Pins for the oracle's analytic gradients: finite differences (an
independent route through the loss), exactness for the quadratic colour
dependence, and the zero gradient at an exact fit."""
import numpy as np
import pytest

from oracle.fd import fd_gradients
from oracle.grads import gradients, loss_gradients
from oracle.loss import dloss_dimg, mse
from oracle.render import render_bruteforce
from paper_2505_09324_amd import synth


def _problem(seed, N=10, H=30, W=34):
    xy, chol, rgb = synth.random_gaussians(N, W, H, seed=seed, scale_lo=1.5, scale_hi=5.0)
    chol = chol.astype(np.float64)
    chol[:, 1] = np.random.default_rng(seed + 1).uniform(-2, 2, size=N)
    chol[1, 0] = -chol[1, 0]           # a negative diagonal entry is legal
    target = np.random.default_rng(seed + 2).uniform(0, 1, size=(3, H, W))
    return xy.astype(np.float64), chol, rgb.astype(np.float64) - 0.3, target, H, W


@pytest.mark.parametrize("seed", [1, 2])
def test_analytic_matches_finite_differences(seed):
    """P7: O-5 vs O-6 to 1e-6 relative on every FD-defined element."""
    xy, chol, rgb, target, H, W = _problem(seed)
    g = loss_gradients(xy, chol, rgb, target, H, W)
    fd = fd_gradients(xy, chol, rgb, target, H, W)
    n_checked = 0
    top = max(np.abs(g[k]).max() for k in ("g_xy", "g_chol", "g_rgb"))
    for grp, key in (("xy", "g_xy"), ("chol", "g_chol"), ("rgb", "g_rgb")):
        f = fd[grp]
        ok = np.isfinite(f)
        # FD round-off floor: eps * loss / h ~ 1e-11 absolute, far below
        # 2e-8 of the largest gradient in the problem
        err = np.abs(f[ok] - g[key][ok])
        assert np.all(err <= 1e-6 * np.abs(g[key][ok]) + 2e-8 * top), (grp, err.max())
        n_checked += ok.sum()
    assert n_checked >= 0.9 * 8 * xy.shape[0]


def test_colour_gradient_exact_for_quadratic():
    """The loss is quadratic in the colours, so a central difference with a
    large step is exact: no FD truncation, no cutoff change."""
    xy, chol, rgb, target, H, W = _problem(3)
    g = loss_gradients(xy, chol, rgb, target, H, W)
    h = 0.25
    for n in (0, 4, 9):
        for k in range(3):
            p, m = rgb.copy(), rgb.copy()
            p[n, k] += h
            m[n, k] -= h
            lp = mse(render_bruteforce(xy, chol, p, H, W)["img"], target)
            lm = mse(render_bruteforce(xy, chol, m, H, W)["img"], target)
            assert (lp - lm) / (2 * h) == pytest.approx(g["g_rgb"][n, k], rel=1e-9, abs=1e-15)


def test_zero_gradient_at_exact_fit():
    """P6: target = render(theta) gives all gradients 0."""
    xy, chol, rgb, _, H, W = _problem(4)
    target = render_bruteforce(xy, chol, rgb, H, W)["img"]
    g = loss_gradients(xy, chol, rgb, target, H, W)
    for k in ("g_xy", "g_chol", "g_rgb"):
        assert np.abs(g[k]).max() <= 1e-12


def test_bounds_dominate_gradients():
    xy, chol, rgb, target, H, W = _problem(5)
    img = render_bruteforce(xy, chol, rgb, H, W)["img"]
    g = gradients(xy, chol, rgb, dloss_dimg(img, target), H, W)
    for k in ("xy", "chol", "rgb"):
        assert np.all(np.abs(g["g_" + k]) <= g["abs_" + k] * (1 + 1e-12))
