"""P-frame selective optimisation on the GPU (Sec. 3.2.C): the selection
against the FP32-specified oracle (bit-exact), and the fitting loop with an
active mask (inactive Gaussians untouched, trajectory against the oracle's
masked loop)."""
import numpy as np
import pytest
import torch

from oracle.fit import fit as oracle_fit
from oracle.select import changed_pixels, influence_q, select
from paper_2505_09324_amd import _lib, synth
from gpu_util import DEV, VARIANTS, GpuFrame, dev, host

pytestmark = pytest.mark.gpu


def _moving_pair(W, H, seed, t):
    a, _ = synth.make_frame(W, H, seed=seed, t=t)
    b, _ = synth.make_frame(W, H, seed=seed, t=t + 1)
    return b, a  # current, reference


@pytest.mark.parametrize("tile,ppl", VARIANTS)
def test_selection_matches_oracle_on_a_ragged_frame(tile, ppl):
    print(f"select {tile}/{ppl}", flush=True)
    W, H, N = 123, 90, 700
    cur, prev = _moving_pair(W, H, 11, 3)
    xy, chol, rgb = synth.random_gaussians(N, W, H, seed=12)
    chol[:, 1] = np.random.default_rng(13).uniform(-1.5, 1.5, N).astype(np.float32)
    xy[5] = [np.nan, 3.0]       # culled
    xy[6] = [-30.0, -30.0]      # off-frame
    ch_ref, sel_ref = select(cur, prev, 0.03, xy, chol)
    assert 0 < ch_ref.sum() < W * H and 0 < sel_ref.sum() < N
    f = GpuFrame(W, H, N, tile, ppl=ppl)
    X, Cc = dev(xy), dev(chol)
    _lib.project_bin(f.shape, X, Cc, f.ws)
    counts = torch.full((2,), -1, dtype=torch.int32, device=DEV)
    act = _lib.select_changed(f.shape, f.ws, X, Cc, dev(cur), dev(prev), 0.03, counts=counts)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(act).astype(bool), sel_ref)
    assert host(act).max() <= 1
    np.testing.assert_array_equal(host(counts), [int(ch_ref.sum()), int(sel_ref.sum())])


def test_selection_edge_cases():
    print("select edges", flush=True)
    W, H, N = 40, 24, 60
    cur, prev = _moving_pair(W, H, 21, 0)
    xy, chol, _ = synth.random_gaussians(N, W, H, seed=22)
    f = GpuFrame(W, H, N, 16)
    X, Cc = dev(xy), dev(chol)
    _lib.project_bin(f.shape, X, Cc, f.ws)
    counts = torch.zeros(2, dtype=torch.int32, device=DEV)
    same = dev(prev)
    act = _lib.select_changed(f.shape, f.ws, X, Cc, same, same, 0.0, counts=counts)
    torch.cuda.synchronize()
    assert host(act).sum() == 0 and host(counts).tolist() == [0, 0]   # nothing changed
    act = _lib.select_changed(f.shape, f.ws, X, Cc, same, same, -1.0, counts=counts)
    _, sel_all = select(prev, prev, -1.0, xy, chol)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(act).astype(bool), sel_all)   # every pixel changed
    assert host(counts).tolist() == [W * H, int(sel_all.sum())]


def test_selection_full_hd_sampled_gaussians():
    """1920x1080, 30k Gaussians from the content-aware init on frame t,
    selection for frame t+1 at tile 32 / 2 px per lane: the change mask is
    compared whole, the selection for 3000 sampled Gaussians (each against
    the changed pixels in a window around its 3-sigma box, which holds every
    pixel it can influence), and the selected count against the oracle's
    count over the whole frame."""
    print("select 1080p", flush=True)
    from paper_2505_09324_amd import workloads
    W, H, N = 1920, 1080, 30000
    f0, m0 = synth.make_frame_torch(W, H, 301, 4, DEV)
    f1, _ = synth.make_frame_torch(W, H, 301, 5, DEV)
    xy_d, chol_d, _ = [p.contiguous() for p in workloads.plain_init_dev(f0, m0, N, 302)]
    shape = _lib.make_shape(W, H, N, 32, px_per_lane=2)
    ws = _lib.alloc_workspace(shape)
    _lib.project_bin(shape, xy_d, chol_d, ws)
    counts = torch.zeros(2, dtype=torch.int32, device=DEV)
    act = host(_lib.select_changed(shape, ws, xy_d, chol_d, f1, f0, 0.02, counts=counts)).astype(bool)
    cur, prev, xy, chol = host(f1), host(f0), host(xy_d), host(chol_d)
    ch = changed_pixels(cur, prev, 0.02)
    assert host(counts)[0] == ch.sum() and host(counts)[1] == act.sum()
    idx = np.random.default_rng(0).choice(N, 3000, replace=False)
    for n in idx:
        l1, l2, l3 = (float(c) for c in chol[n])
        rx, ry = 3 * abs(l1) + 2, 3 * np.hypot(l2, l3) + 2
        x0, x1 = max(int(xy[n, 0] - rx), 0), min(int(xy[n, 0] + rx) + 1, W)
        y0, y1 = max(int(xy[n, 1] - ry), 0), min(int(xy[n, 1] + ry) + 1, H)
        ys, xs = np.nonzero(ch[y0:y1, x0:x1]) if x0 < x1 and y0 < y1 else ((), ())
        want = bool(len(xs)) and bool(np.any(influence_q(xy[n:n + 1], chol[n:n + 1],
                                                         np.asarray(xs) + x0,
                                                         np.asarray(ys) + y0) <= 9))
        assert act[n] == want, n
    print(f"changed {ch.sum()} px, selected {act.sum()} of {N}", flush=True)


@pytest.mark.parametrize("use_graph", [True, False])
def test_masked_fit_matches_oracle_and_keeps_inactive(use_graph):
    """128x128 / 500 Gaussians, 10 Adam steps at lr 1e-2 with a third of the
    Gaussians active: inactive parameters and moments stay bit for bit, the
    loss trajectory follows the oracle's masked loop (1e-3 relative)."""
    print(f"masked fit graph={use_graph}", flush=True)
    frame, _ = synth.make_frame(128, 128, seed=101)
    xy, chol, rgb = synth.random_gaussians(500, 128, 128, seed=102)
    act = np.zeros(500, bool)
    act[np.random.default_rng(5).choice(500, 170, replace=False)] = True
    N = 500
    f = GpuFrame(128, 128, N, 16)
    P = {"xy": dev(xy), "chol": dev(chol), "rgb": dev(rgb)}
    M = torch.full((8 * N,), 0.5, device=DEV)   # non-zero moments must survive too
    V = torch.full((8 * N,), 0.25, device=DEV)
    M0, V0 = host(M).copy(), host(V).copy()
    step = torch.zeros(1, dtype=torch.int32, device=DEV)
    trace = torch.zeros(32, device=DEV)
    A = dev(act.astype(np.uint8))
    opts = _lib.fit_opts(10, 4, use_graph=use_graph, cfg=_lib.adam_cfg(1e-2), active=A)
    st = _lib.fit_frame(f.shape, dev(frame), P["xy"], P["chol"], P["rgb"], M, V, step, trace,
                        f.ws, opts)
    assert st.iters_run == 10
    for k, a in (("xy", xy), ("chol", chol), ("rgb", rgb)):
        got = host(P[k])
        np.testing.assert_array_equal(got[~act], a[~act])
        assert np.all(np.any(got[act] != a[act], axis=1))
    lay = np.concatenate([np.repeat(act, 2), np.repeat(act, 3), np.repeat(act, 3)])
    np.testing.assert_array_equal(host(M)[~lay], M0[~lay])
    np.testing.assert_array_equal(host(V)[~lay], V0[~lay])
    # the oracle starts from zero moments: rerun the GPU from zero moments
    P = {"xy": dev(xy), "chol": dev(chol), "rgb": dev(rgb)}
    M.zero_(), V.zero_(), step.zero_()
    _lib.fit_frame(f.shape, dev(frame), P["xy"], P["chol"], P["rgb"], M, V, step, trace, f.ws,
                   opts)
    _, ref = oracle_fit(xy, chol, rgb, frame, 10, lr=1e-2, active=act)
    np.testing.assert_allclose(host(trace)[:10], ref, rtol=1e-3)
