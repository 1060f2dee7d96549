"""GPU parity of the learned re-initialisation of warm-started P-frames
(Sec. 3.2.B at P-frames, Sec. 3.2.C): the selected tiles, the freed
Gaussians and every count are integer decisions and must be identical to
the oracle's; the Gaussians not replaced are bit for bit unchanged, and the
replaced ones equal the oracle's decoding of the same slot within the slot
decoder's bar (GPU sigmoid and exp against the FP64 ones).  The head is a
seeded synthetic input shared by both sides."""
import numpy as np
import pytest
import torch

from oracle.cnn import pframe_replace
from paper_2505_09324_amd import _lib, synth
from gpu_util import DEV, dev, host

pytestmark = pytest.mark.gpu

F32 = np.float32


def _head(TY, TX, seed, nan_unused=False):
    rng = np.random.default_rng(seed)
    h = rng.normal(0, 1.5, (73, TY, TX)).astype(F32)
    if nan_unused:                        # NaN in slot 7 of every tile whose count is < 8
        k = np.argmax(h[:9], axis=0)
        h[9 + 7 * 8 + 2][k < 8] = np.nan
    return h


def _gaussians(N, W, H, seed):
    xy, chol, rgb = synth.random_gaussians(N, W, H, seed=seed)
    xy[:4] = [[-3, 5], [W + 2, 1], [np.nan, 4], [16.0, 16.0]]   # off-frame, not finite, a corner
    return xy, chol, rgb


def _compare(frame, prev, head, xy, chol, rgb, tau, net=None):
    H, W = frame.shape[1:]
    N = len(xy)
    if net is None:
        net = _lib.CNNInit(H, W, seed=3)
    gx, gc, gr = dev(xy), dev(chol), dev(rgb)
    sel = torch.zeros(net.TY, net.TX, dtype=torch.uint8, device=DEV)
    stats = net.pframe_replace(dev(frame), dev(prev), tau, gx, gc, gr, head=dev(head), tile_sel=sel)
    torch.cuda.synchronize()
    ox, oc, orgb, info = pframe_replace(frame, prev, head, xy, chol, rgb, tau)
    np.testing.assert_array_equal(host(sel).astype(bool), info["selected"])
    np.testing.assert_array_equal(host(stats), [info["selected"].sum(), len(info["freed"]),
                                                info["n_predicted"], info["replaced"]])
    gx, gc, gr = host(gx), host(gc), host(gr)
    done = info["freed"][:info["replaced"]]
    keep = np.setdiff1d(np.arange(N), done)
    np.testing.assert_array_equal(gx[keep], xy[keep])
    np.testing.assert_array_equal(gc[keep], chol[keep])
    np.testing.assert_array_equal(gr[keep], rgb[keep])
    np.testing.assert_allclose(gx[done], ox[done], rtol=1e-5, atol=1e-4)
    np.testing.assert_allclose(gc[done], oc[done], rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(gr[done], orgb[done], rtol=1e-5, atol=1e-6)
    return info


@pytest.mark.parametrize("W,H,N,tau", [(96, 64, 300, 1e-3), (117, 70, 500, 0.03),
                                       (117, 70, 40, 1e-3)])
def test_pframe_replace_small(W, H, N, tau):
    print(f"pframe replace {W}x{H} N={N} tau={tau}", flush=True)
    prev, _ = synth.make_frame(W, H, seed=5999, t=3)
    frame, _ = synth.make_frame(W, H, seed=5999, t=4)
    TY, TX = (H + 15) // 16, (W + 15) // 16
    info = _compare(frame, prev, _head(TY, TX, 7, nan_unused=True), *_gaussians(N, W, H, 8), tau)
    assert info["replaced"] > 0 and info["selected"].any() and not info["selected"].all()


def test_pframe_replace_guards():
    print("pframe replace guards", flush=True)
    W, H = 96, 64
    prev, _ = synth.make_frame(W, H, seed=5999, t=3)
    frame, _ = synth.make_frame(W, H, seed=5999, t=4)
    g = _gaussians(300, W, H, 8)
    head = _head(4, 6, 7)
    # nothing changed
    info = _compare(prev, prev, head, *g, 0.0)
    assert info["replaced"] == 0 and not info["selected"].any()
    # every tile selected
    info = _compare(frame + F32(0.5), prev, head, *g, 0.0)
    assert info["selected"].all()
    # a non-finite raw parameter of a used slot: nothing replaced
    bad = head.copy()
    k = np.argmax(bad[:9], axis=0)
    ty, tx = np.argwhere(k > 0)[0]
    bad[9 + 4, ty, tx] = np.inf
    info = _compare(frame + F32(0.5), prev, bad, *g, 0.0)
    assert info["replaced"] == 0 and info["n_predicted"] > 0


def test_pframe_replace_uses_the_last_forward_head():
    print("pframe replace, head from the forward pass", flush=True)
    W, H = 96, 64
    prev, _ = synth.make_frame(W, H, seed=5999, t=3)
    frame, _ = synth.make_frame(W, H, seed=5999, t=4)
    xy, chol, rgb = _gaussians(300, W, H, 8)
    net = _lib.CNNInit(H, W, seed=3)
    head = torch.empty(73, net.TY, net.TX, device=DEV)
    net.forward(dev(frame), dev(prev), head_out=head)
    a = [dev(xy), dev(chol), dev(rgb)]
    b = [dev(xy), dev(chol), dev(rgb)]
    sa = net.pframe_replace(dev(frame), dev(prev), 1e-3, *a)
    sb = net.pframe_replace(dev(frame), dev(prev), 1e-3, *b, head=head)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(sa), host(sb))
    for u, v in zip(a, b):
        np.testing.assert_array_equal(host(u), host(v))


def test_pframe_replace_full_hd():
    """1920x1080, 30,000 warm-started Gaussians from the content-aware
    initialisation of the previous frame, the whole decision compared."""
    print("pframe replace 1080p", flush=True)
    from oracle.init import init_from_frame
    W, H = 1920, 1080
    prev, mask = synth.make_frame(W, H, seed=5999, t=3)
    frame, _ = synth.make_frame(W, H, seed=5999, t=4)
    xy, chol, rgb, _ = init_from_frame(prev, mask, synth.init_draws(30000, seed=12))
    info = _compare(frame, prev, _head(68, 120, 9, nan_unused=True), xy, chol, rgb, 1e-3)
    assert info["replaced"] > 1000
