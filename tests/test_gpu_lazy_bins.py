"""Lazy tile binning in the fitting loop (gs2d_fit_opts.bin_skin > 0).

Between rebuilds the loop renders with the lists of an earlier iteration,
built from 3-sigma boxes grown by the skin.  That is exact only if those
lists hold every (tile, Gaussian) pair whose current box meets the tile, in
(tile, index) order.  After a fit the workspace holds the lists and the
geometry of the last iteration (centre and box half-widths), so the tests
rebuild each Gaussian's exact tile rectangle on the host, with the FP32
operations the binning specifies, and check that every such pair is in the
lists; they also check that rebuilds were skipped, that motion fast enough
to force rebuilds and Gaussians crossing the cull threshold keep the
property, and that a lazy fit follows the exactly binned one."""
import numpy as np
import pytest
import torch

from paper_2505_09324_amd import _lib, synth
from gpu_util import DEV, dev, host

pytestmark = pytest.mark.gpu

F32 = np.float32


def _exact_rects(geom, W, H, T):
    """Exact tile rectangles of the last projection (FP32, as specified)."""
    mx, my, rx, ry = (geom[:, i].astype(F32) for i in (0, 1, 5, 6))
    inv = F32(1.0 / T)
    TX, TY = (W + T - 1) // T, (H + T - 1) // T
    fx0, fx1 = np.floor((mx - rx) * inv), np.floor((mx + rx) * inv)
    fy0, fy1 = np.floor((my - ry) * inv), np.floor((my + ry) * inv)
    culled = np.all(geom == 0, axis=1)
    off = (fx1 < 0) | (fx0 > TX - 1) | (fy1 < 0) | (fy0 > TY - 1) | culled
    rc = np.stack([np.maximum(fx0, 0), np.maximum(fy0, 0), np.minimum(fx1, TX - 1),
                   np.minimum(fy1, TY - 1)], 1).astype(np.int64)
    return rc, off


def _check_lists(shape, ws, W, H, T):
    b = _lib.read_bins(shape, ws)
    view = _lib.bins_view(shape, ws)
    geom = _lib._slice(ws, view.geom, 8 * shape.N, torch.float32).cpu().numpy().reshape(-1, 8)
    keys = b["keys"].astype(np.int64)
    assert np.all(np.diff(keys) > 0), "keys are not strictly ascending (tile, index)"
    ts = b["tile_start"]
    tiles = keys >> 16
    np.testing.assert_array_equal(ts, np.searchsorted(tiles, np.arange(b["n_tiles"] + 1)))
    rc, off = _exact_rects(geom, W, H, T)
    TX = b["TX"]
    need = []
    for n in np.nonzero(~off)[0]:
        x0, y0, x1, y1 = rc[n]
        for ty in range(y0, y1 + 1):
            for tx in range(x0, x1 + 1):
                need.append(((ty * TX + tx) << 16) | n)
    need = np.array(need, np.int64)
    missing = np.setdiff1d(need, keys)
    assert missing.size == 0, f"{missing.size} exact pairs missing from the lists"
    return len(need), len(keys)


def _fit(W, H, N, iters, seed, skin, lr=(2e-2, 5e-3, 5e-3), init=None, chunk=None):
    frame, mask = synth.make_frame(W, H, seed=seed)
    d = synth.init_draws(N, seed=seed + 1)
    T = torch.from_numpy(frame).to(DEV)
    if init is None:
        xy, chol, rgb = _lib.init_plain(T, dev(mask.astype(np.uint8)), dev(d.pick_roi),
                                        dev(d.jit_roi), dev(d.pick_out), dev(d.jit_out))
    else:
        xy, chol, rgb = (dev(a) for a in init)
    shape = _lib.make_shape(W, H, N, 32, px_per_lane=2)
    ws = _lib.alloc_workspace(shape)
    # a recycled block could hold complete lists of this shape from an
    # earlier test, which the first call would keep (valid, but the rebuild
    # counts asserted below assume a fresh workspace)
    ws.zero_()
    m = torch.zeros(8 * N, device=DEV)
    v = torch.zeros(8 * N, device=DEV)
    step = torch.zeros(1, dtype=torch.int32, device=DEV)
    trace = torch.zeros(iters + 8, device=DEV)
    st = _lib.fit_frame(shape, T, xy, chol, rgb, m, v, step, trace, ws,
                        _lib.fit_opts(iters, chunk or iters, cfg=_lib.adam_cfg(lr), bin_skin=skin))
    torch.cuda.synchronize()
    return shape, ws, st, host(trace[:iters]), (host(xy), host(chol), host(rgb))


def test_lazy_lists_cover_every_pair_full_hd():
    """Three chunks of 20 iterations: the lists of one chunk carry over to
    the next (only the call's first iteration forces a rebuild), the Adam
    step between chunks included."""
    print("lazy binning 1080p", flush=True)
    shape, ws, st, tr, _ = _fit(1920, 1080, 30000, 60, 201, 1.0, chunk=20)
    assert 1 <= st.rebins < 60, st.rebins
    need, have = _check_lists(shape, ws, 1920, 1080, 32)
    assert have >= need


def test_lazy_lists_under_fast_motion():
    """Means moving up to ~0.5 px per step: rebuilds most iterations."""
    print("lazy binning, fast motion", flush=True)
    shape, ws, st, tr, _ = _fit(320, 240, 2000, 40, 17, 1.0, lr=(0.5, 0.05, 5e-3))
    assert st.rebins >= 5, st.rebins
    _check_lists(shape, ws, 320, 240, 32)


def test_lazy_lists_across_the_cull_threshold():
    """Gaussians whose Cholesky diagonal starts below or near the cull
    threshold (|l| < 2^-14): crossing it either way must rebuild."""
    print("lazy binning, culling", flush=True)
    W, H, N = 256, 192, 600
    xy, chol, rgb = synth.random_gaussians(N, W, H, seed=5)
    chol[:40, 0] = np.linspace(-3e-4, 3e-4, 40)
    chol[40:80, 2] = np.linspace(-3e-4, 3e-4, 40)
    shape, ws, st, tr, (fx, fc, fr) = _fit(W, H, N, 30, 31, 1.0, lr=(2e-2, 2e-4, 5e-3),
                                           init=(xy, chol, rgb), chunk=30)
    assert st.rebins >= 1
    _check_lists(shape, ws, W, H, 32)
    assert np.all(np.isfinite(tr))


@pytest.mark.parametrize("skin", [1.0, 0.02])
def test_lazy_fit_follows_the_exact_fit(skin):
    """A 0.02-px skin rebuilds the lists every few iterations (66 of 200
    measured), running the rebuild path of the combined emission/scatter
    launch (ticketed roles, the handoff between them) many times."""
    print(f"lazy vs exact fit, skin {skin}", flush=True)
    a = _fit(320, 240, 1500, 200, 23, skin, chunk=50)
    b = _fit(320, 240, 1500, 200, 23, 0.0, chunk=50)
    print(f"rebuilds {a[2].rebins}", flush=True)
    assert b[2].rebins == 0 and a[2].rebins >= (1 if skin >= 1.0 else 20), a[2].rebins
    # the render at the first iteration uses the same parameters: bit-equal
    assert a[3][0] == b[3][0]
    np.testing.assert_allclose(a[3], b[3], rtol=1e-4)
    for u, w in zip(a[4], b[4]):
        np.testing.assert_allclose(u, w, rtol=1e-3, atol=1e-4)


def test_bin_skin_is_validated():
    print("bin_skin validation", flush=True)
    W, H, N = 64, 48, 50
    for skin in (-1.0, 65.0, float("nan")):
        with pytest.raises(_lib.GS2DError):
            _fit(W, H, N, 2, 3, skin)


def _state(W, H, N, seed):
    frame, mask = synth.make_frame(W, H, seed=seed)
    d = synth.init_draws(N, seed=seed + 1)
    T = torch.from_numpy(frame).to(DEV)
    xy, chol, rgb = _lib.init_plain(T, dev(mask.astype(np.uint8)), dev(d.pick_roi),
                                    dev(d.jit_roi), dev(d.pick_out), dev(d.jit_out))
    m = torch.zeros(8 * N, device=DEV)
    v = torch.zeros(8 * N, device=DEV)
    step = torch.zeros(1, dtype=torch.int32, device=DEV)
    return T, xy, chol, rgb, m, v, step


def _call(shape, ws, T, xy, chol, rgb, m, v, step, trace, iters, lr, chunk=None):
    st = _lib.fit_frame(shape, T, xy, chol, rgb, m, v, step, trace, ws,
                        _lib.fit_opts(iters, chunk or iters, cfg=_lib.adam_cfg(lr), bin_skin=1.0))
    torch.cuda.synchronize()
    return st


def test_lazy_lists_carry_over_between_calls():
    """A call on a workspace that holds complete lazy lists of the same shape
    starts from them: with the Gaussians all but still, the first call
    rebuilds once and the second not at all.  Exact binning into the
    workspace, or another shape over the same memory, makes the next call
    rebuild.  The lists cover every exact pair after each call."""
    print("lazy lists across calls", flush=True)
    W, H, N = 320, 240, 1500
    T, xy, chol, rgb, m, v, step = _state(W, H, N, 61)
    shape = _lib.make_shape(W, H, N, 32, px_per_lane=2)
    ws = _lib.alloc_workspace(shape)
    ws.zero_()  # no stamp left by an earlier user of this memory
    trace = torch.zeros(200, device=DEV)
    still = (1e-7, 1e-7, 1e-7)
    args = (T, xy, chol, rgb, m, v, step, trace)
    assert _call(shape, ws, *args, 10, still).rebins == 1
    assert _call(shape, ws, *args, 10, still).rebins == 0
    _check_lists(shape, ws, W, H, 32)
    _lib.project_bin(shape, xy, chol, ws)  # exact lists replace the lazy ones
    assert _call(shape, ws, *args, 10, still).rebins == 1
    _check_lists(shape, ws, W, H, 32)
    n2 = N - 100  # a smaller shape over the same memory
    shape2 = _lib.make_shape(W, H, n2, 32, px_per_lane=2)
    a2 = (T, xy[:n2], chol[:n2], rgb[:n2], m[:8 * n2], v[:8 * n2], step, trace)
    assert _call(shape2, ws, *a2, 10, still).rebins == 1
    assert _call(shape2, ws, *a2, 10, still).rebins == 0
    _check_lists(shape2, ws, W, H, 32)
    assert _call(shape, ws, *args, 10, still).rebins == 1
    _check_lists(shape, ws, W, H, 32)


def test_two_calls_follow_one_call():
    """40 iterations as two calls on one workspace (the second starting from
    the first's lists) against one call of 40 on a fresh workspace: the
    same lists in use at every iteration, so the same loss trace up to the
    order of the gradients' float atomics."""
    print("two calls vs one", flush=True)
    W, H, N = 320, 240, 1500
    lr = (2e-2, 5e-3, 5e-3)
    runs = []
    for split in (True, False):
        T, xy, chol, rgb, m, v, step = _state(W, H, N, 67)
        shape = _lib.make_shape(W, H, N, 32, px_per_lane=2)
        ws = _lib.alloc_workspace(shape)
        ws.zero_()
        trace = torch.zeros(48, device=DEV)
        args = (T, xy, chol, rgb, m, v, step, trace)
        if split:
            r = _call(shape, ws, *args, 20, lr).rebins + _call(shape, ws, *args, 20, lr).rebins
        else:
            r = _call(shape, ws, *args, 40, lr, chunk=20).rebins
        _check_lists(shape, ws, W, H, 32)
        runs.append((host(trace[:40]), r))
    print(f"rebuilds {runs[0][1]} (two calls), {runs[1][1]} (one call)", flush=True)
    assert runs[0][0][0] == runs[1][0][0]
    np.testing.assert_allclose(runs[0][0], runs[1][0], rtol=1e-4)


def test_overflowed_lists_are_not_kept():
    """Lists truncated at the pair capacity are never carried into the next
    call: with the Gaussians all but still, each call rebuilds exactly once
    (at its first iteration) and reports the overflow."""
    print("overflowed lists across calls", flush=True)
    W, H, N = 128, 128, 500
    T, xy, chol, rgb, m, v, step = _state(W, H, N, 71)
    shape = _lib.make_shape(W, H, N, 32, max_pairs=100, px_per_lane=2)
    ws = _lib.alloc_workspace(shape)
    ws.zero_()
    trace = torch.zeros(64, device=DEV)
    opts = _lib.fit_opts(5, 5, cfg=_lib.adam_cfg((1e-7, 1e-7, 1e-7)), bin_skin=1.0)
    for _ in range(2):
        st = _lib.fit_frame(shape, T, xy, chol, rgb, m, v, step, trace, ws, opts, check=False)
        torch.cuda.synchronize()
        assert st.code == _lib.GS2D_EOVERFLOW and st.status & _lib.STATUS_OVERFLOW
        assert st.rebins == 1, st.rebins
