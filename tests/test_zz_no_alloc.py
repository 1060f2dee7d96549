"""gs2d_fit_frame_static (the fitting loop on the library's device-resident
workspace, for callers that cannot allocate) against gs2d_fit_frame with a
caller workspace: two calls in a row, the second on a smaller frame with
fewer Gaussians, so that whatever the first call left in the shared array
must not leak into the second."""
import numpy as np
import pytest
import torch

from paper_2505_09324_amd import _lib, synth
from gpu_util import DEV, dev, host

pytestmark = pytest.mark.gpu


def _fit_both(W, H, N, tile, ppl, iters, chunk, frame, params, lr):
    shape = _lib.make_shape(W, H, N, tile, px_per_lane=ppl)
    cfg = _lib.adam_cfg(lr)
    out = []
    for which in ("workspace", "static"):
        p = [q.clone() for q in params]
        m, v = torch.zeros(8 * N, device=DEV), torch.zeros(8 * N, device=DEV)
        step = torch.zeros(1, dtype=torch.int32, device=DEV)
        trace = torch.full((iters + 4,), -1.0, device=DEV)
        opts = _lib.fit_opts(iters, chunk, use_graph=False, cfg=cfg)
        if which == "workspace":
            st = _lib.fit_frame(shape, frame, *p, m, v, step, trace, _lib.alloc_workspace(shape),
                                opts, ctx=False)
        else:
            st = _lib.fit_frame_static(shape, frame, *p, m, v, step, trace, opts)
        torch.cuda.synchronize()
        assert st.iters_run == iters and st.status == 0 and int(step.item()) == iters
        out.append((host(trace), [host(q) for q in p], host(m), host(v)))
    (ta, pa, ma, va), (tb, pb, mb, vb) = out
    # identical arithmetic; only the order of the float atomics that sum
    # the gradients differs between runs
    np.testing.assert_allclose(tb[:iters], ta[:iters], rtol=1e-5)
    assert np.all(tb[iters:] == -1.0)
    for a, b, step in zip(pa, pb, lr):
        assert np.all(np.abs(a - b) <= 1e-3 * step + 1e-6 * np.abs(a)), np.abs(a - b).max()
    for a, b in ((ma, mb), (va, vb)):
        assert np.abs(a - b).max() <= 1e-4 * np.abs(a).max() + 1e-12


def test_static_workspace_fit_matches_caller_workspace_twice():
    print("static fit 1920x1080/30k, then 128x128/500", flush=True)
    from paper_2505_09324_amd import workloads
    f, m = synth.make_frame_torch(1920, 1080, 71, 0, DEV)
    p0 = [q.contiguous() for q in workloads.plain_init_dev(f, m, 30000, 72)]
    _fit_both(1920, 1080, 30000, 32, 2, 6, 3, f, p0, (2e-2, 5e-3, 5e-3))
    frame, _ = synth.make_frame(128, 128, seed=101)
    xy, chol, rgb = synth.random_gaussians(500, 128, 128, seed=102)
    _fit_both(128, 128, 500, 16, 1, 10, 4, dev(frame), [dev(xy), dev(chol), dev(rgb)],
              (1e-2, 1e-2, 1e-2))


def test_static_workspace_rejects_shapes_beyond_its_size():
    shape = _lib.make_shape(4096, 4096, 65536, 16)
    assert _lib.workspace_bytes(shape) > _lib.GS2D_STATIC_WORKSPACE_BYTES
    N = 65536
    z = lambda *s: torch.zeros(*s, device=DEV)
    st = _lib.fit_frame_static(shape, z(3, 4096, 4096), z(N, 2), z(N, 3), z(N, 3), z(8 * N),
                               z(8 * N), torch.zeros(1, dtype=torch.int32, device=DEV), z(16),
                               _lib.fit_opts(1, 1), check=False)
    assert st.code == _lib.GS2D_ENOSPACE
