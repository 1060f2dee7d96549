"""The autograd.Function around the HIP rasteriser: gradients through a torch
loss vs FP64 finite differences and the oracle's analytic gradient, on a
64x64 crop of a moving-subject frame."""
import numpy as np
import pytest
import torch

from oracle.fd import fd_gradients
from oracle.grads import loss_gradients
from paper_2505_09324_amd import synth
from paper_2505_09324_amd.autograd import render
from gpu_util import DEV, assert_grads_close, dev, host

pytestmark = pytest.mark.gpu


def _crop():
    """64x64 window of frame 1 whose left edge is at the subject's right
    boundary, with 40 Gaussians scattered over it."""
    W, H = 320, 180
    frame, mask = synth.make_frame(W, H, seed=301, t=1)
    row = H // 2
    right = int(np.nonzero(mask[row])[0].max())
    x0 = min(right, W - 64)
    y0 = row - 32
    crop = np.ascontiguousarray(frame[:, y0:y0 + 64, x0:x0 + 64])
    xy, chol, rgb = synth.random_gaussians(40, 64, 64, seed=302, scale_lo=2.0, scale_hi=7.0)
    chol[:, 1] = np.random.default_rng(303).uniform(-2, 2, 40).astype(np.float32)
    return crop, xy, chol, rgb


@pytest.mark.parametrize("tile", [8, 16])
def test_autograd_matches_fd_and_oracle(tile):
    print(f"autograd tile={tile}", flush=True)
    crop, xy, chol, rgb = _crop()
    P = [dev(a).requires_grad_(True) for a in (xy, chol, rgb)]
    T = dev(crop)
    img = render(*P, 64, 64, tile=tile)
    loss = ((img - T) ** 2).mean()
    loss.backward()
    got = {"xy": host(P[0].grad), "chol": host(P[1].grad), "rgb": host(P[2].grad)}
    ref = loss_gradients(xy, chol, rgb, crop, 64, 64)
    assert float(loss) == pytest.approx(ref["loss"], rel=1e-4)
    assert_grads_close(got, ref)
    fd = fd_gradients(xy, chol, rgb, crop, 64, 64)
    top = max(np.abs(ref[k]).max() for k in ("g_xy", "g_chol", "g_rgb"))
    n_ok = 0
    for k in ("xy", "chol", "rgb"):
        ok = np.isfinite(fd[k])
        err = np.abs(got[k][ok] - fd[k][ok])
        assert np.all(err <= 1e-3 * np.abs(fd[k][ok]) + 1e-5 * top), (k, err.max())
        n_ok += ok.sum()
    assert n_ok >= 0.9 * 8 * 40


def test_autograd_composes_with_other_terms():
    """Gradients add up with other terms of a torch graph (a weighted sum of
    two renders and a parameter penalty)."""
    print("autograd compose", flush=True)
    crop, xy, chol, rgb = _crop()
    P = [dev(a).requires_grad_(True) for a in (xy, chol, rgb)]
    T = dev(crop)
    a = ((render(*P, 64, 64) - T) ** 2).mean()
    b = ((render(*P, 64, 64, tile=8) - T) ** 2).mean()
    (0.25 * a + 0.75 * b + 1e-3 * (P[2] ** 2).sum()).backward()
    ref = loss_gradients(xy, chol, rgb, crop, 64, 64)
    got = {"xy": host(P[0].grad), "chol": host(P[1].grad),
           "rgb": host(P[2].grad) - 2e-3 * rgb}
    assert_grads_close(got, ref)
