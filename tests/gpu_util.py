"""Shared helpers for the GPU parity tests (not collected: no test_ prefix)."""
from __future__ import annotations

import numpy as np
import torch

from paper_2505_09324_amd import _lib, synth

DEV = "cuda"


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def host(t):
    return t.detach().cpu().numpy()


class GpuFrame:
    """Shape + workspace for one frame on the GPU."""

    def __init__(self, W, H, N, tile=16, max_pairs=None, ppl=1):
        self.shape = _lib.make_shape(W, H, N, tile, max_pairs, ppl)
        self.ws = _lib.alloc_workspace(self.shape)
        self.W, self.H, self.N = W, H, N

    def bin(self, xy, chol):
        _lib.project_bin(self.shape, xy, chol, self.ws)
        torch.cuda.synchronize()
        return _lib.read_bins(self.shape, self.ws)

    def forward(self, xy, chol, rgb, target=None):
        _lib.project_bin(self.shape, xy, chol, self.ws)
        img = torch.empty(3, self.H, self.W, device=DEV)
        dl = loss = None
        if target is not None:
            dl = torch.empty_like(img)
            loss = torch.empty((), device=DEV)
        _lib.render_fwd(self.shape, self.ws, rgb, target, img, dl, loss)
        torch.cuda.synchronize()
        return img, dl, loss

    def backward(self, rgb, dl):
        N = self.N
        g = (torch.empty(N, 2, device=DEV), torch.empty(N, 3, device=DEV), torch.empty(N, 3, device=DEV))
        _lib.render_bwd(self.shape, self.ws, rgb, dl, *g)
        torch.cuda.synchronize()
        return g


def assert_pixels_close(gpu_img, ref, rel=1e-4, what="image"):
    """|C_gpu - C_ref| <= rel * A_p + Amb_p; pixels with A_p == 0 exactly 0."""
    g = np.asarray(gpu_img, np.float64)
    err = np.abs(g - ref["img"])
    bound = rel * ref["abs"] + ref["amb"] + 1e-30
    bad = err > bound
    assert not bad.any(), (f"{what}: {bad.sum()} of {bad.size} values out of tolerance; worst "
                           f"err {err[bad].max():.3e} bound {bound[bad][np.argmax(err[bad])]:.3e}")
    empty = ref["abs"] == 0
    assert np.all(g[empty] == 0.0), f"{what}: pixels with no contributing pair are not 0"


def assert_grads_close(gpu, ref, rel=1e-3):
    """|g_gpu - g_ref| <= rel * B_e + Amb_e, element by element."""
    for k in ("xy", "chol", "rgb"):
        g = np.asarray(gpu[k], np.float64)
        err = np.abs(g - ref["g_" + k])
        bound = rel * ref["abs_" + k] + ref["amb_" + k] + 1e-30
        bad = err > bound
        assert not bad.any(), (f"g_{k}: {bad.sum()} elements out of tolerance; worst err "
                               f"{err[bad].max():.3e}")


# every compiled raster variant: (tile, pixels per lane)
VARIANTS = [(8, 1), (16, 1), (16, 2), (32, 1), (32, 2), (32, 4)]


def dense_long_lists():
    """A dense 90x70 frame of 3000 large, sheared, zero-mean-colour
    Gaussians: tile lists reach 806 (tile 8), 1119 (16) and 1657 (32)
    entries, i.e. up to seven LDS chunks of 256."""
    W, H, N = 90, 70, 3000
    xy, chol, rgb = synth.random_gaussians(N, W, H, seed=31, scale_lo=1.5, scale_hi=9.0)
    chol[:, 1] = np.random.default_rng(32).uniform(-3, 3, N).astype(np.float32)
    rgb -= 0.5
    frame, _ = synth.make_frame(W, H, seed=33)
    return W, H, N, frame, xy, chol, rgb


def loss_bound(ref, frame):
    """Largest |loss_gpu - loss_ref| that pixels within their own bar
    (|dC| <= 1e-4 A + Amb) allow, plus FP32 summation slack."""
    b = 1e-4 * ref["abs"] + ref["amb"]
    r = np.abs(ref["img"] - frame)
    lo = float(((ref["img"] - frame) ** 2).mean())
    return float((2 * r * b + b * b).sum() / r.size) + 1e-6 * lo

