"""Pin for the oracle's fitting loop: recovery of a known parameter set."""
import numpy as np

from oracle.fit import fit
from oracle.loss import psnr_from_mse
from oracle.render import render_box
from paper_2505_09324_amd import synth


def test_recovers_known_gaussians():
    """P10: target = render(theta*) (N=40 on 48x48); starting from theta*
    plus noise the loop drives the PSNR far above the start."""
    H = W = 48
    xy, chol, rgb = synth.random_gaussians(40, W, H, seed=31, scale_lo=2.0, scale_hi=4.0)
    target = render_box(xy, chol, rgb, H, W, want_bounds=False)["img"]
    rng = np.random.default_rng(32)
    xy0 = xy + rng.normal(scale=0.3, size=xy.shape)
    chol0 = chol + rng.normal(scale=0.05, size=chol.shape) * np.array([1, 0, 1])
    rgb0 = rgb + rng.normal(scale=0.03, size=rgb.shape)
    _, losses = fit(xy0, chol0, rgb0, target, iters=300, lr={"xy": 2e-3, "chol": 1e-3, "rgb": 1e-3})
    start, end = psnr_from_mse(losses[0]), psnr_from_mse(losses[-1])
    assert end > start + 15.0 and end > 40.0
