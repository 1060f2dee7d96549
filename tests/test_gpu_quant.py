"""Post-training quantisation and quantisation-aware fitting on the GPU
(Sec. 3.3) against the oracle: codes, dequantised parameters and ranges bit
for bit, entropy-coded bits to FP64 rounding, and the quantisation-aware
loop's loss against the oracle's."""
import numpy as np
import pytest
import torch

from oracle.fit import fit as oracle_fit
from oracle.quant import ptq as oracle_ptq
from paper_2505_09324_amd import _lib, synth
from gpu_util import DEV, GpuFrame, dev, host

pytestmark = pytest.mark.gpu


def _gaussians(N, seed):
    rng = np.random.default_rng(seed)
    xy = np.stack([rng.uniform(-20, 1940, N), rng.uniform(-20, 1100, N)], 1).astype(np.float32)
    chol = np.stack([rng.lognormal(0.5, 0.6, N), rng.normal(0, 1.5, N), rng.lognormal(0.4, 0.7, N)],
                    1).astype(np.float32)
    rgb = rng.normal(0.5, 0.3, (N, 3)).astype(np.float32)
    rgb[:, 1] = np.round(rgb[:, 1] * 8) / 8        # values on a grid: ties and repeats
    return xy, chol, rgb


@pytest.mark.parametrize("bits", [(6, 6), (4, 8), (12, 5), (1, 1)])
def test_ptq_matches_oracle_bit_for_bit(bits):
    print(f"ptq {bits}", flush=True)
    N = 5001
    xy, chol, rgb = _gaussians(N, sum(bits))
    ref = oracle_ptq(xy, chol, rgb, *bits)
    got = _lib.ptq(dev(xy), dev(chol), dev(rgb), *bits, want_codes=True)
    torch.cuda.synchronize()
    for k in ("xy", "chol", "rgb"):
        np.testing.assert_array_equal(host(got[k]), ref[k])
    np.testing.assert_array_equal(host(got["ranges"]), ref["ranges"])
    codes = host(got["codes"])
    np.testing.assert_array_equal(codes[:, 2:], ref["codes"])
    np.testing.assert_array_equal(codes[:, :2].astype(np.uint16),
                                  xy.astype(np.float16).view(np.uint16))
    b = host(got["bits"])
    np.testing.assert_allclose(b[:6], ref["component_bits"], rtol=1e-12, atol=1e-9)
    assert abs(b[6] - ref["bits"]) <= 1e-12 * ref["bits"]


def test_ptq_constant_component_and_fitted_frame():
    print("ptq constant + init", flush=True)
    N = 3000
    xy, chol, rgb = _gaussians(N, 77)
    chol[:, 1] = 0.0                                # l2 = 0 everywhere (plain init): one symbol
    ref = oracle_ptq(xy, chol, rgb, 6, 6)
    got = _lib.ptq(dev(xy), dev(chol), dev(rgb), 6, 6)
    np.testing.assert_array_equal(host(got["chol"]), ref["chol"])
    assert host(got["bits"])[1] == 0.0 and ref["component_bits"][1] == 0.0
    # the content-aware initialisation of a 1080p frame
    from paper_2505_09324_amd import workloads
    f, m = synth.make_frame_torch(1920, 1080, 201, None, DEV)
    p = [q.contiguous() for q in workloads.plain_init_dev(f, m, 30000, 202)]
    ref = oracle_ptq(*[host(q) for q in p], 6, 6)
    got = _lib.ptq(*p, 6, 6, want_codes=True)
    np.testing.assert_array_equal(host(got["codes"])[:, 2:], ref["codes"])
    np.testing.assert_array_equal(host(got["rgb"]), ref["rgb"])


@pytest.mark.parametrize("use_graph,skin", [(True, 1.0), (False, 1.0), (True, 0.0)])
def test_quantisation_aware_fit_follows_the_oracle(use_graph, skin):
    """128x128 / 500 Gaussians, 5-bit Cholesky and colour: the first
    iteration's loss is the oracle's loss at the quantised point (1e-5
    relative), and 10 steps follow the oracle's quantisation-aware loop
    (1e-3 relative; codes of the two trajectories may part at rounding
    boundaries); with lazy tile lists of the quantised Gaussians (skin 1)
    and with the lists rebuilt every iteration (skin 0)."""
    print(f"qat graph={use_graph} skin={skin}", flush=True)
    frame, _ = synth.make_frame(128, 128, seed=101)
    xy, chol, rgb = synth.random_gaussians(500, 128, 128, seed=102)
    N = 500
    f = GpuFrame(128, 128, N, 16)
    P = [dev(xy), dev(chol), dev(rgb)]
    M, V = torch.zeros(8 * N, device=DEV), torch.zeros(8 * N, device=DEV)
    step = torch.zeros(1, dtype=torch.int32, device=DEV)
    trace = torch.zeros(32, device=DEV)
    st = _lib.fit_frame(f.shape, dev(frame), *P, M, V, step, trace, f.ws,
                        _lib.fit_opts(10, 4, use_graph=use_graph, cfg=_lib.adam_cfg(1e-2),
                                      qat=(5, 5), bin_skin=skin))
    assert st.iters_run == 10
    _, ref = oracle_fit(xy, chol, rgb, frame, 10, lr=1e-2, quant_bits=(5, 5))
    tr = host(trace)[:10]
    assert abs(tr[0] - ref[0]) <= 1e-5 * ref[0]
    np.testing.assert_allclose(tr, ref, rtol=1e-3)
    _, plain = oracle_fit(xy, chol, rgb, frame, 1, lr=1e-2)
    assert abs(tr[0] - plain[0]) > 1e-4 * plain[0]   # the quantised point is not the plain one
