"""Learned initialiser kernels (BF16 MFMA convolutions, head loss, Adam,
targets, decode) against the FP64 oracle on small frames."""
import numpy as np
import pytest
import torch

from oracle import cnn as ocnn
from paper_2505_09324_amd import _lib, synth
from gpu_util import DEV, dev, host

pytestmark = pytest.mark.gpu

H, W = 96, 128          # 6 x 8 tiles of 16 px


def _frames(seed):
    f0, _ = synth.make_frame(W, H, seed=seed, t=0)
    f1, _ = synth.make_frame(W, H, seed=seed, t=3)
    return f0, f1


def _x(f1, f0):
    return np.concatenate([f1, f1 - f0]).astype(np.float64)


def test_forward_matches_oracle():
    print("cnn forward", flush=True)
    f0, f1 = _frames(41)
    net = _lib.CNNInit(H, W, seed=5)
    head = torch.empty(73, net.TY, net.TX, device=DEV)
    net.forward(dev(f1), dev(f0), head_out=head)
    torch.cuda.synchronize()
    ref, _ = ocnn.forward(_x(f1, f0), net.oracle_params(), bf16=True)
    got = host(head)
    assert got.shape == ref.shape == (73, 6, 8)
    scale = np.abs(ref).mean()
    assert np.abs(got - ref).max() <= 2e-2 * scale, np.abs(got - ref).max() / scale


def test_targets_match_oracle():
    print("cnn targets", flush=True)
    xy, chol, rgb = synth.random_gaussians(900, W, H, seed=6, scale_lo=0.6, scale_hi=3.0)
    chol[:, 1] = np.random.default_rng(1).uniform(-1, 1, 900).astype(np.float32)
    xy[:5] = [[-1.0, 3.0], [W + 1.0, 4.0], [5.0, H + 2.0], [15.999, 15.999], [16.0, 16.0]]
    net = _lib.CNNInit(H, W, seed=5)
    net.set_targets(dev(xy), dev(chol), dev(rgb))
    counts, vec = net.read_targets()
    torch.cuda.synchronize()
    ref = ocnn.tile_targets(xy, chol, rgb, W, H, 16)
    counts, vec = host(counts), host(vec)
    n_tiles = net.TY * net.TX
    for t in range(n_tiles):
        r = ref.get(t, np.zeros((0, 8)))
        assert counts[t] == len(r), t
        np.testing.assert_allclose(vec[t, :len(r)], r, rtol=1e-5, atol=1e-5)
        assert not vec[t, len(r):].any()
    assert counts.max() == 8 and counts.sum() > 300


def test_backward_matches_oracle():
    print("cnn backward", flush=True)
    f0, f1 = _frames(43)
    xy, chol, rgb = synth.random_gaussians(700, W, H, seed=7, scale_lo=0.6, scale_hi=3.0)
    net = _lib.CNNInit(H, W, seed=8)
    net.set_targets(dev(xy), dev(chol), dev(rgb))
    head = torch.empty(73, net.TY, net.TX, device=DEV)
    net.forward(dev(f1), dev(f0), head_out=head)
    loss = net.backward()
    torch.cuda.synchronize()
    params = net.oracle_params()
    x = _x(f1, f0)
    ref_head, _ = ocnn.forward(x, params, bf16=True)
    targets = ocnn.tile_targets(xy, chol, rgb, W, H, 16)
    # loss of the GPU's own head output against the oracle's targets
    l_gpu_head, hg = ocnn.head_loss(host(head).astype(np.float64), targets)
    assert float(loss[0]) == pytest.approx(l_gpu_head, rel=2e-3)
    grads = ocnn.backward(x, params, hg, bf16=True)
    got = net.oracle_grads()
    for i in range(5):
        for j in range(2):
            g, r = got[i][j].astype(np.float64), grads[i][j]
            rel = np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-30)
            assert rel < 3e-2, (i, j, rel)


def test_training_reduces_loss_and_decode_matches_oracle():
    print("cnn train + decode", flush=True)
    f0, f1 = _frames(45)
    xy, chol, rgb = synth.random_gaussians(600, W, H, seed=9, scale_lo=0.8, scale_hi=3.0)
    net = _lib.CNNInit(H, W, seed=10)
    net.set_targets(dev(xy), dev(chol), dev(rgb))
    losses = []
    for it in range(60):
        net.forward(dev(f1), dev(f0))
        losses.append(float(net.backward()[0]))
        net.step(lr=3e-3)
    assert losses[-1] < 0.7 * losses[0], losses[::10]
    # decode vs the oracle's decode of the same head output
    head = torch.empty(73, net.TY, net.TX, device=DEV)
    net.forward(dev(f1), dev(f0), head_out=head)
    pxy, pch, prgb = synth.random_gaussians(600, W, H, seed=11)
    gx, gc, gr, npred = net.decode(600, dev(pxy), dev(pch), dev(prgb))
    torch.cuda.synchronize()
    rx, rc, rr, rn = ocnn.decode(host(head).astype(np.float64), 600, (pxy, pch, prgb))
    assert int(npred[0]) == rn
    np.testing.assert_allclose(host(gx), rx, rtol=1e-5, atol=1e-4)
    np.testing.assert_allclose(host(gc), rc, rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(host(gr), rr, rtol=1e-5, atol=1e-6)
