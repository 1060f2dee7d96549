"""Batched fitting: the persistent (frame, tile) raster and the segmented
per-frame binning against the oracle, frame by frame, and the autotuner."""
import numpy as np
import pytest
import torch

from oracle.binning import bin_gaussians
from oracle.fit import fit as oracle_fit
from oracle.grads import gradients
from oracle.loss import dloss_dimg, mse
from oracle.render import render_box
from paper_2505_09324_amd import _lib, synth
from gpu_util import DEV, VARIANTS, assert_grads_close, dense_long_lists, dev, host, loss_bound

pytestmark = pytest.mark.gpu

SMALL = [(96, 64, 300), (130, 77, 700), (64, 64, 200), (200, 120, 1500), (50, 40, 100)]


def _batch_inputs(sizes, seed):
    frames, params = [], []
    for i, (w, h, n) in enumerate(sizes):
        f, _ = synth.make_frame(w, h, seed=seed + i)
        xy, chol, rgb = synth.random_gaussians(n, w, h, seed=seed + 100 + i, scale_lo=0.8,
                                               scale_hi=5.0)
        chol[:, 1] = np.random.default_rng(seed + 200 + i).uniform(-1.5, 1.5, n).astype(np.float32)
        frames.append(f)
        params.append((xy, chol, rgb))
    targets = np.concatenate([f.ravel() for f in frames])
    cat = [np.concatenate([p[k] for p in params]) for k in range(3)]
    return frames, params, targets, cat


def _split(a, sizes, per):
    out, o = [], 0
    for _, _, n in sizes:
        out.append(a[o:o + n * per].reshape(n, per) if per > 1 else a[o:o + n])
        o += n * per
    return out


@pytest.mark.parametrize("T,ppl", VARIANTS)
def test_batch_render_matches_oracle_per_frame(T, ppl):
    print(f"batch render T={T} ppl={ppl}", flush=True)
    frames, params, targets, cat = _batch_inputs(SMALL, 500)
    Nt = sum(n for _, _, n in SMALL)
    ws = torch.empty(_lib.batch_workspace_bytes(SMALL, T, ppl), dtype=torch.uint8, device=DEV)
    g = [torch.zeros(Nt, d, device=DEV) for d in (2, 3, 3)]
    loss = torch.zeros(len(SMALL), device=DEV)
    _lib.batch_render_grads(SMALL, T, ppl, dev(targets), dev(cat[0]), dev(cat[1]), dev(cat[2]),
                            *g, ws, loss_per_frame=loss)
    torch.cuda.synchronize()
    gx = _split(host(g[0]).ravel(), SMALL, 2)
    gc = _split(host(g[1]).ravel(), SMALL, 3)
    gr = _split(host(g[2]).ravel(), SMALL, 3)
    for f, ((w, h, n), frame, (xy, chol, rgb)) in enumerate(zip(SMALL, frames, params)):
        b = _lib.read_batch_bins(SMALL, T, ppl, f, ws)
        ob = bin_gaussians(xy, chol, w, h, T)
        np.testing.assert_array_equal(b["keys"].astype(np.int64),
                                      ob["pair_tiles"] * 65536 + ob["pair_ids"])
        np.testing.assert_array_equal(b["tile_start"], ob["tile_start"])
        img = render_box(xy, chol, rgb, h, w, want_bounds=False)["img"]
        assert float(loss[f]) == pytest.approx(mse(img, frame), rel=1e-4)
        ref = gradients(xy, chol, rgb, dloss_dimg(img, frame), h, w)
        assert_grads_close({"xy": gx[f], "chol": gc[f], "rgb": gr[f]}, ref)


def test_batch_two_pass_sort_when_a_frame_has_many_tiles():
    """A batch mixing small frames with one of more than 2048 tiles (400 x
    330 at T = 8: 50 x 42, 12-bit tile ids, so both 8-bit radix passes
    carry keys across the whole tile range): lists, loss and gradients of
    every frame against the oracle."""
    print("batch two-pass sort", flush=True)
    sizes = SMALL[:2] + [(400, 330, 1200)]
    frames, params, targets, cat = _batch_inputs(sizes, 700)
    Nt = sum(n for _, _, n in sizes)
    ws = torch.empty(_lib.batch_workspace_bytes(sizes, 8, 1), dtype=torch.uint8, device=DEV)
    g = [torch.zeros(Nt, d, device=DEV) for d in (2, 3, 3)]
    loss = torch.zeros(len(sizes), device=DEV)
    _lib.batch_render_grads(sizes, 8, 1, dev(targets), dev(cat[0]), dev(cat[1]), dev(cat[2]),
                            *g, ws, loss_per_frame=loss)
    torch.cuda.synchronize()
    gx = _split(host(g[0]).ravel(), sizes, 2)
    gc = _split(host(g[1]).ravel(), sizes, 3)
    gr = _split(host(g[2]).ravel(), sizes, 3)
    for f, ((w, h, n), frame, (xy, chol, rgb)) in enumerate(zip(sizes, frames, params)):
        b = _lib.read_batch_bins(sizes, 8, 1, f, ws)
        ob = bin_gaussians(xy, chol, w, h, 8)
        np.testing.assert_array_equal(b["keys"].astype(np.int64),
                                      ob["pair_tiles"] * 65536 + ob["pair_ids"])
        np.testing.assert_array_equal(b["tile_start"], ob["tile_start"])
        img = render_box(xy, chol, rgb, h, w, want_bounds=False)["img"]
        assert float(loss[f]) == pytest.approx(mse(img, frame), rel=1e-4)
        ref = gradients(xy, chol, rgb, dloss_dimg(img, frame), h, w)
        assert_grads_close({"xy": gx[f], "chol": gc[f], "rgb": gr[f]}, ref)


def test_fit_batch_trajectories_match_oracle():
    """10 lockstep Adam steps: every frame's loss trace vs the oracle loop
    run on that frame alone (1e-3 relative)."""
    print("fit batch trajectory", flush=True)
    sizes = SMALL[:3]
    frames, params, targets, cat = _batch_inputs(sizes, 600)
    Nt = sum(n for _, _, n in sizes)
    ws = torch.empty(_lib.batch_workspace_bytes(sizes, 16, 1), dtype=torch.uint8, device=DEV)
    P = [dev(c) for c in cat]
    m = torch.zeros(8 * Nt, device=DEV)
    v = torch.zeros(8 * Nt, device=DEV)
    step = torch.zeros(1, dtype=torch.int32, device=DEV)
    trace = torch.full((32, len(sizes)), -1.0, device=DEV)
    st = _lib.fit_batch(sizes, 16, 1, dev(targets), *P, m, v, step, trace, ws,
                        _lib.fit_opts(10, 5, cfg=_lib.adam_cfg(1e-2)))
    assert st.iters_run == 10 and int(step[0]) == 10
    tr = host(trace)
    for f, (frame, (xy, chol, rgb)) in enumerate(zip(frames, params)):
        _, losses = oracle_fit(xy, chol, rgb, frame, 10, lr=1e-2)
        np.testing.assert_allclose(tr[:10, f], losses, rtol=1e-3)
    assert np.all(tr[10:] == -1.0)


def test_autotuner_and_full_batch_workload():
    """The 48-frame batched workload (sizes drawn from 320x240 .. 1920x1080,
    3k-50k Gaussians from the content-aware init): the autotuner times every
    variant; 3 lockstep iterations run without overflow; one small frame's
    bins and loss match the oracle."""
    print("full batch", flush=True)
    from paper_2505_09324_amd import workloads
    sizes, targets, xy, chol, rgb, frames_np = workloads.batch_inputs(48, seed=400, device=DEV)
    cands = [(8, 1), (16, 1), (16, 2), (32, 2)]
    best, ms = _lib.autotune_batch(sizes, targets, xy, chol, rgb, cands, reps=2)
    assert 0 <= best < len(cands) and all(x > 0 for x in ms)
    T, ppl = cands[best]
    Nt = sum(n for _, _, n in sizes)
    ws = torch.empty(_lib.batch_workspace_bytes(sizes, T, ppl), dtype=torch.uint8, device=DEV)
    x0, c0, r0 = xy.clone(), chol.clone(), rgb.clone()
    m = torch.zeros(8 * Nt, device=DEV)
    v = torch.zeros(8 * Nt, device=DEV)
    step = torch.zeros(1, dtype=torch.int32, device=DEV)
    trace = torch.zeros((8, len(sizes)), device=DEV)
    st = _lib.fit_batch(sizes, T, ppl, targets, xy, chol, rgb, m, v, step, trace, ws,
                        _lib.fit_opts(3, 3, cfg=_lib.adam_cfg((2e-2, 5e-3, 5e-3))))
    assert st.code == 0 and st.iters_run == 3
    f = min(range(len(sizes)), key=lambda i: sizes[i][0] * sizes[i][1])
    w, h, n = sizes[f]
    off = sum(s[2] for s in sizes[:f])
    pxy, pch, prgb = (host(t)[off:off + n] for t in (x0, c0, r0))
    img = render_box(pxy, pch, prgb, h, w, want_bounds=False)["img"]
    assert float(trace[0, f]) == pytest.approx(mse(img, frames_np[f]), rel=1e-4)
    # bins of the final state of that frame
    g = [torch.zeros(Nt, d, device=DEV) for d in (2, 3, 3)]
    _lib.batch_render_grads(sizes, T, ppl, targets, xy, chol, rgb, *g, ws)
    b = _lib.read_batch_bins(sizes, T, ppl, f, ws)
    ob = bin_gaussians(host(xy)[off:off + n], host(chol)[off:off + n], w, h, T)
    np.testing.assert_array_equal(b["keys"].astype(np.int64), ob["pair_tiles"] * 65536 + ob["pair_ids"])


def test_autotune_cache_on_device(tmp_path):
    """The first call times the candidates on the GPU and stores the choice;
    the second call with the same batch returns it from the JSON file."""
    print("autotune cache", flush=True)
    from paper_2505_09324_amd import autotune
    frames, params, targets, cat = _batch_inputs(SMALL, 900)
    path = str(tmp_path / "autotune.json")
    args = (SMALL, dev(targets), dev(cat[0]), dev(cat[1]), dev(cat[2]))
    cands = [(16, 1), (32, 2)]
    cfg, ms, cached = autotune.tuned_batch_config(*args, candidates=cands, reps=2, cache_path=path)
    assert not cached and cfg in cands and all(v > 0 for v in ms.values())
    cfg2, ms2, cached2 = autotune.tuned_batch_config(*args, candidates=cands, reps=2,
                                                     cache_path=path)
    assert cached2 and cfg2 == cfg and ms2 == {}



def test_batch_long_lists_every_variant():
    """The persistent batched kernel on a frame whose tile lists exceed 256
    and 512 entries (up to seven LDS chunks), beside a sparse frame: lists
    bit-exact, loss and every gradient element of both frames against the
    oracle, for every (tile, pixels per lane) variant."""
    W, H, N, frame, xy, chol, rgb = dense_long_lists()
    f2, _ = synth.make_frame(64, 48, seed=34)
    xy2, chol2, rgb2 = synth.random_gaussians(150, 64, 48, seed=35, scale_lo=0.8, scale_hi=4.0)
    sizes = [(W, H, N), (64, 48, 150)]
    frames = [frame, f2]
    params = [(xy, chol, rgb), (xy2, chol2, rgb2)]
    targets = np.concatenate([a.ravel() for a in frames])
    cat = [np.concatenate([p[k] for p in params]) for k in range(3)]
    refs = []
    for (w, h, n), fr, (a, b, c) in zip(sizes, frames, params):
        r = render_box(a, b, c, h, w)
        refs.append((r, gradients(a, b, c, dloss_dimg(r["img"], fr), h, w)))
    Nt = N + 150
    for T, ppl in VARIANTS:
        print(f"batch long lists T={T} ppl={ppl}", flush=True)
        ws = torch.empty(_lib.batch_workspace_bytes(sizes, T, ppl), dtype=torch.uint8, device=DEV)
        g = [torch.zeros(Nt, d, device=DEV) for d in (2, 3, 3)]
        loss = torch.zeros(2, device=DEV)
        _lib.batch_render_grads(sizes, T, ppl, dev(targets), dev(cat[0]), dev(cat[1]),
                                dev(cat[2]), *g, ws, loss_per_frame=loss)
        torch.cuda.synchronize()
        gx = _split(host(g[0]).ravel(), sizes, 2)
        gc = _split(host(g[1]).ravel(), sizes, 3)
        gr = _split(host(g[2]).ravel(), sizes, 3)
        for fi, ((w, h, n), fr, (a, b, c)) in enumerate(zip(sizes, frames, params)):
            bb = _lib.read_batch_bins(sizes, T, ppl, fi, ws)
            ob = bin_gaussians(a, b, w, h, T)
            np.testing.assert_array_equal(bb["keys"].astype(np.int64),
                                          ob["pair_tiles"] * 65536 + ob["pair_ids"])
            np.testing.assert_array_equal(bb["tile_start"], ob["tile_start"])
            if fi == 0:
                assert np.diff(ob["tile_start"]).max() > 512
            r, want = refs[fi]
            assert abs(float(loss[fi]) - mse(r["img"], fr)) <= loss_bound(r, fr)
            assert_grads_close({"xy": gx[fi], "chol": gc[fi], "rgb": gr[fi]}, want)


def test_lazy_batch_fit_follows_the_exact_fit():
    """Lazy binning frame by frame (a 1-px skin): each frame keeps its tile
    lists until one of its Gaussians leaves its recorded rectangle.  Against
    the same fit with the lists rebuilt every iteration the loss traces
    agree (the first bit for bit), some rebuilds are skipped, and after the
    fit every frame's lists still hold every exact (tile, Gaussian) pair of
    its last projection, in (tile, index) order."""
    print("lazy batch fit", flush=True)
    from test_gpu_lazy_bins import _exact_rects
    sizes = SMALL
    frames, params, targets, cat = _batch_inputs(sizes, 650)
    Nt = sum(n for _, _, n in sizes)
    T, ppl, iters = 16, 1, 40
    runs = []
    for skin in (1.0, 0.0):
        ws = torch.empty(_lib.batch_workspace_bytes(sizes, T, ppl), dtype=torch.uint8, device=DEV)
        P = [dev(c) for c in cat]
        m = torch.zeros(8 * Nt, device=DEV)
        v = torch.zeros(8 * Nt, device=DEV)
        step = torch.zeros(1, dtype=torch.int32, device=DEV)
        trace = torch.zeros((iters + 4, len(sizes)), device=DEV)
        st = _lib.fit_batch(sizes, T, ppl, dev(targets), *P, m, v, step, trace, ws,
                            _lib.fit_opts(iters, 20, cfg=_lib.adam_cfg((2e-2, 5e-3, 5e-3)),
                                          bin_skin=skin))
        assert st.code == 0 and st.iters_run == iters
        runs.append((host(trace[:iters]), st.rebins, ws))
    (ta, ra, ws), (tb, rb, _) = runs
    print(f"rebuilds {ra} of {iters * len(sizes)} frame-iterations", flush=True)
    assert rb == 0 and len(sizes) <= ra < iters * len(sizes)
    np.testing.assert_array_equal(ta[0], tb[0])
    np.testing.assert_allclose(ta, tb, rtol=1e-4)
    for f, (w, h, n) in enumerate(sizes):
        b = _lib.read_batch_bins(sizes, T, ppl, f, ws)
        keys = b["keys"].astype(np.int64)
        assert np.all(np.diff(keys) > 0)
        np.testing.assert_array_equal(
            b["tile_start"], np.searchsorted(keys >> 16, np.arange(len(b["tile_start"]))))
        rc, off = _exact_rects(b["geom"], w, h, T)
        TX = (w + T - 1) // T
        need = [((ty * TX + tx) << 16) | i for i in np.nonzero(~off)[0]
                for ty in range(rc[i, 1], rc[i, 3] + 1) for tx in range(rc[i, 0], rc[i, 2] + 1)]
        assert np.setdiff1d(np.array(need, np.int64), keys).size == 0, f"frame {f}"


def test_persistent_and_grid_batch_rasters_agree():
    """The batched fit's two raster launches, one workgroup per (frame, tile)
    item (exact block masks) and the persistent work-queue grid (box
    masks): the same loss traces (the first row bit for bit, both summing
    the same pairs in the same order) and the oracle's first loss."""
    print("persistent vs grid batch raster", flush=True)
    sizes = SMALL
    frames, params, targets, cat = _batch_inputs(sizes, 700)
    Nt = sum(n for _, _, n in sizes)
    T, ppl, iters = 32, 2, 12
    traces = []
    for persistent in (False, True):
        ws = torch.empty(_lib.batch_workspace_bytes(sizes, T, ppl), dtype=torch.uint8, device=DEV)
        P = [dev(c) for c in cat]
        m = torch.zeros(8 * Nt, device=DEV)
        v = torch.zeros(8 * Nt, device=DEV)
        step = torch.zeros(1, dtype=torch.int32, device=DEV)
        trace = torch.zeros((iters + 4, len(sizes)), device=DEV)
        st = _lib.fit_batch(sizes, T, ppl, dev(targets), *P, m, v, step, trace, ws,
                            _lib.fit_opts(iters, 6, cfg=_lib.adam_cfg((2e-2, 5e-3, 5e-3)),
                                          batch_persistent=persistent))
        assert st.code == 0 and st.iters_run == iters
        traces.append(host(trace[:iters]))
    np.testing.assert_array_equal(traces[0][0], traces[1][0])
    np.testing.assert_allclose(traces[0], traces[1], rtol=1e-4)
    for f, (frame, (xy, chol, rgb)) in enumerate(zip(frames, params)):
        h, w = frame.shape[1:]
        img = render_box(xy, chol, rgb, h, w, want_bounds=False)["img"]
        assert float(traces[0][0, f]) == pytest.approx(mse(img, frame), rel=1e-4)
