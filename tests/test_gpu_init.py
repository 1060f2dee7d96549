"""GPU parity of the content-aware ROI initialiser: the drawn pixel of every
Gaussian is identical to the oracle's (an integer decision), the parameters
agree to FP32 rounding."""
import numpy as np
import pytest
import torch

from oracle.init import init_from_frame
from paper_2505_09324_amd import _lib, synth
from gpu_util import DEV, dev, host

pytestmark = pytest.mark.gpu


def _run(frame, mask, draws):
    N = draws.pick_roi.shape[0] + draws.pick_out.shape[0]
    picked = torch.full((N,), -1, dtype=torch.int32, device=DEV)
    xy, chol, rgb = _lib.init_plain(dev(frame), dev(mask.astype(np.uint8)), dev(draws.pick_roi),
                                    dev(draws.jit_roi), dev(draws.pick_out), dev(draws.jit_out),
                                    picked=picked)
    torch.cuda.synchronize()
    return host(xy), host(chol), host(rgb), host(picked)


def _compare(frame, mask, draws):
    gx, gc, gr, gp = _run(frame, mask, draws)
    ox, oc, orgb, info = init_from_frame(frame, mask, draws)
    np.testing.assert_array_equal(gp, info["picked"])
    np.testing.assert_array_equal(gx, ox)
    np.testing.assert_allclose(gc, oc, rtol=1e-6)
    np.testing.assert_allclose(gr, orgb, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("W,H,N", [(96, 64, 300), (130, 77, 2000)])
def test_init_small_frames(W, H, N):
    print(f"init {W}x{H} N={N}", flush=True)
    frame, mask = synth.make_frame(W, H, seed=9)
    _compare(frame, mask, synth.init_draws(N, seed=10))


def test_init_empty_and_full_roi():
    print("init empty/full roi", flush=True)
    frame, _ = synth.make_frame(50, 40, seed=3)
    d = synth.init_draws(120, seed=4)
    _compare(frame, np.zeros((40, 50), bool), d)
    _compare(frame, np.ones((40, 50), bool), d)


def test_init_full_hd():
    """1920x1080 with 30k Gaussians, 70 % in the ROI: the initialisation used
    by the 1080p fitting workload."""
    print("init 1080p", flush=True)
    frame, mask = synth.make_frame(1920, 1080, seed=201)
    _compare(frame, mask, synth.init_draws(30000, seed=202))
