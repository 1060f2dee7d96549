"""GPU parity of the Adam step and of the fitting loop (per-step teacher
forcing and free-running trajectory) against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle.adam import adam_step as oracle_adam
from oracle.binning import bin_gaussians
from oracle.fit import fit as oracle_fit
from oracle.grads import gradients
from oracle.loss import dloss_dimg, mse
from oracle.render import render_box
from paper_2505_09324_amd import _lib, synth
from gpu_util import DEV, GpuFrame, assert_grads_close, assert_pixels_close, dev, host

pytestmark = pytest.mark.gpu

LR = (1e-2, 1e-2, 1e-2)
# the hyper-parameters the GPU receives are FP32 numbers; the oracle takes
# their exact values
B1, B2, EPS = (float(np.float32(x)) for x in (0.9, 0.999, 1e-8))


def _f32(d):
    return {k: float(np.float32(x)) for k, x in d.items()}


def _rand_state(N, seed):
    rng = np.random.default_rng(seed)
    th = {"xy": rng.uniform(0, 50, (N, 2)), "chol": rng.uniform(0.5, 3, (N, 3)),
          "rgb": rng.uniform(0, 1, (N, 3))}
    g = {k: rng.normal(scale=1e-3, size=v.shape) for k, v in th.items()}
    m = {k: rng.normal(scale=1e-4, size=v.shape) for k, v in th.items()}
    v = {k: rng.uniform(0, 1e-6, size=x.shape) for k, x in th.items()}
    f32 = lambda d: {k: x.astype(np.float32) for k, x in d.items()}
    return f32(th), f32(g), f32(m), f32(v)


def _flat(d):
    return np.concatenate([d["xy"].ravel(), d["chol"].ravel(), d["rgb"].ravel()])


def _unflat(a, N):
    return {"xy": a[:2 * N].reshape(N, 2), "chol": a[2 * N:5 * N].reshape(N, 3),
            "rgb": a[5 * N:].reshape(N, 3)}


@pytest.mark.parametrize("t0", [0, 7])
def test_adam_step_matches_oracle(t0):
    print(f"adam t0={t0}", flush=True)
    N = 1000
    th, g, m, v = _rand_state(N, 1 + t0)
    P = {k: dev(x) for k, x in th.items()}
    G = {k: dev(x) for k, x in g.items()}
    M, V = dev(_flat(m)), dev(_flat(v))
    step = torch.tensor([t0], dtype=torch.int32, device=DEV)
    cfg = _lib.adam_cfg((1e-2, 2e-3, 5e-3))
    _lib.adam_step(P["xy"], P["chol"], P["rgb"], G["xy"], G["chol"], G["rgb"], M, V, step, cfg,
                   zero_grads=True)
    torch.cuda.synchronize()
    lr = _f32({"xy": 1e-2, "chol": 2e-3, "rgb": 5e-3})
    th2, m2, v2, t = oracle_adam(th, g, m, v, t0, lr, B1, B2, EPS)
    assert host(step).tolist() == [t0 + 1]
    for k in th:
        # relative to theta, plus FP32 rounding of the step itself
        err = np.abs(host(P[k]) - th2[k])
        assert np.all(err <= 1e-6 * np.abs(th2[k]) + 1e-6 * lr[k]), k
        assert not host(G[k]).any()
    # moments: relative to the magnitude of the two summed terms (the sum
    # itself may cancel)
    gf, mf, vf = _flat(g).astype(np.float64), _flat(m).astype(np.float64), _flat(v).astype(np.float64)
    m_scale = B1 * np.abs(mf) + (1 - B1) * np.abs(gf)
    v_scale = B2 * vf + (1 - B2) * gf * gf
    assert np.all(np.abs(host(M) - _flat(m2)) <= 1e-6 * m_scale)
    assert np.all(np.abs(host(V) - _flat(v2)) <= 1e-5 * v_scale)


def test_adam_inactive_bitwise_unchanged():
    print("adam active", flush=True)
    N = 777
    th, g, m, v = _rand_state(N, 3)
    P = {k: dev(x) for k, x in th.items()}
    G = {k: dev(x) for k, x in g.items()}
    M, V = dev(_flat(m)), dev(_flat(v))
    active = (np.arange(N) % 3 == 0).astype(np.uint8)
    step = torch.zeros(1, dtype=torch.int32, device=DEV)
    _lib.adam_step(P["xy"], P["chol"], P["rgb"], G["xy"], G["chol"], G["rgb"], M, V, step,
                   _lib.adam_cfg(LR), active=dev(active))
    torch.cuda.synchronize()
    off = active == 0
    for k in th:
        np.testing.assert_array_equal(host(P[k])[off], th[k][off])
        assert np.all(host(P[k])[~off] != th[k][~off])
    mm = _unflat(host(M), N)
    for k in th:
        np.testing.assert_array_equal(mm[k][off], m[k][off])


def test_step_parity_teacher_forced_tiny_frame():
    """Each of 10 steps on the tiny frame: the oracle takes the GPU's
    parameters theta_k and checks bins, image, loss, gradients and theta_{k+1}."""
    print("teacher forced", flush=True)
    frame, _ = synth.make_frame(128, 128, seed=101)
    xy, chol, rgb = synth.random_gaussians(500, 128, 128, seed=102)
    N = 500
    f = GpuFrame(128, 128, N, 16)
    P = {"xy": dev(xy), "chol": dev(chol), "rgb": dev(rgb)}
    M = torch.zeros(8 * N, device=DEV)
    V = torch.zeros(8 * N, device=DEV)
    step = torch.zeros(1, dtype=torch.int32, device=DEV)
    T = dev(frame)
    cfg = _lib.adam_cfg(LR)
    for k in range(10):
        th = {kk: host(x).copy() for kk, x in P.items()}
        m_k, v_k = _unflat(host(M).copy(), N), _unflat(host(V).copy(), N)
        bins = f.bin(P["xy"], P["chol"])
        ob = bin_gaussians(th["xy"], th["chol"], 128, 128, 16)
        np.testing.assert_array_equal(bins["keys"].astype(np.int64),
                                      ob["pair_tiles"] * 65536 + ob["pair_ids"])
        img, dl, loss = f.forward(P["xy"], P["chol"], P["rgb"], T)
        ref = render_box(th["xy"], th["chol"], th["rgb"], 128, 128)
        assert_pixels_close(host(img), ref, what=f"step {k}")
        assert float(loss) == pytest.approx(mse(ref["img"], frame), rel=1e-4)
        gx, gc, gr = f.backward(P["rgb"], dl)
        oref = gradients(th["xy"], th["chol"], th["rgb"], dloss_dimg(ref["img"], frame), 128, 128)
        got = {"xy": host(gx), "chol": host(gc), "rgb": host(gr)}
        assert_grads_close(got, oref)
        _lib.adam_step(P["xy"], P["chol"], P["rgb"], gx, gc, gr, M, V, step, cfg)
        torch.cuda.synchronize()
        lr = _f32({"xy": LR[0], "chol": LR[1], "rgb": LR[2]})
        th2, _, _, _ = oracle_adam(th, got, m_k, v_k, k, lr, B1, B2, EPS)
        for kk in th:
            err = np.abs(host(P[kk]) - th2[kk])
            assert np.all(err <= 1e-6 * np.abs(th2[kk]) + 1e-5 * lr[kk]), (k, kk, err.max())


@pytest.mark.parametrize("use_graph", [True, False])
def test_fit_frame_trajectory_tiny_frame(use_graph):
    """GPU fit loop alone vs oracle loop alone: 10 Adam steps at lr 1e-2,
    losses within 1e-3 relative at every step."""
    print(f"fit trajectory graph={use_graph}", flush=True)
    frame, _ = synth.make_frame(128, 128, seed=101)
    xy, chol, rgb = synth.random_gaussians(500, 128, 128, seed=102)
    N = 500
    f = GpuFrame(128, 128, N, 16)
    P = {"xy": dev(xy), "chol": dev(chol), "rgb": dev(rgb)}
    M = torch.zeros(8 * N, device=DEV)
    V = torch.zeros(8 * N, device=DEV)
    step = torch.zeros(1, dtype=torch.int32, device=DEV)
    trace = torch.full((64,), -1.0, device=DEV)
    opts = _lib.fit_opts(10, check_every=4, use_graph=use_graph, cfg=_lib.adam_cfg(LR))
    st = _lib.fit_frame(f.shape, dev(frame), P["xy"], P["chol"], P["rgb"], M, V, step, trace,
                        f.ws, opts)
    assert st.iters_run == 10 and host(step)[0] == 10
    _, losses = oracle_fit(xy, chol, rgb, frame, 10, lr=LR[0])
    np.testing.assert_allclose(host(trace)[:10], losses, rtol=1e-3)
    assert np.all(host(trace)[10:] == -1.0)


def test_fit_frame_stops_at_psnr_and_flags_overflow():
    print("fit stop/overflow", flush=True)
    frame, _ = synth.make_frame(128, 128, seed=101)
    xy, chol, rgb = synth.random_gaussians(500, 128, 128, seed=102)
    N = 500
    f = GpuFrame(128, 128, N, 16)
    M = torch.zeros(8 * N, device=DEV)
    V = torch.zeros(8 * N, device=DEV)
    step = torch.zeros(1, dtype=torch.int32, device=DEV)
    trace = torch.zeros(400, device=DEV)
    P = {"xy": dev(xy), "chol": dev(chol), "rgb": dev(rgb)}
    # PSNR of the initial state is low; a target just above it is met early
    opts = _lib.fit_opts(300, check_every=10, psnr_target=12.0, cfg=_lib.adam_cfg(LR))
    st = _lib.fit_frame(f.shape, dev(frame), P["xy"], P["chol"], P["rgb"], M, V, step, trace,
                        f.ws, opts)
    tr = host(trace)[:st.iters_run]
    psnr = 10 * np.log10(1.0 / tr)
    assert st.iter_hit_target >= 0 and st.iters_run < 300
    assert psnr[st.iter_hit_target] >= 12.0 and np.all(psnr[:st.iter_hit_target] < 12.0)
    assert st.iters_run % 10 == 0
    small = GpuFrame(128, 128, N, 16, max_pairs=100)
    st2 = _lib.fit_frame(small.shape, dev(frame), P["xy"], P["chol"], P["rgb"], M, V, step, trace,
                         small.ws, _lib.fit_opts(20, 5, cfg=_lib.adam_cfg(LR)), check=False)
    assert st2.code == _lib.GS2D_EOVERFLOW and st2.status & _lib.STATUS_OVERFLOW
    assert st2.iters_run == 20  # no target: the chunks run back to back, all of them


def test_fit_frame_rejects_a_short_trace():
    """trace_len <= step[0] + iters: with a PSNR target the call returns
    GS2D_EINVAL before any work; without one it learns step[0] only when the
    work has run, returns GS2D_EINVAL then, and writes no entry past
    trace_len (the kernels bound the index)."""
    print("fit short trace", flush=True)
    frame, _ = synth.make_frame(96, 64, seed=101)
    xy, chol, rgb = synth.random_gaussians(200, 96, 64, seed=102)
    N = 200
    f = GpuFrame(96, 64, N, 16)
    buf = torch.full((64,), -7.0, device=DEV)
    trace = buf[:8]
    for target in (12.0, 0.0):
        P = [dev(xy), dev(chol), dev(rgb)]
        M = torch.zeros(8 * N, device=DEV)
        V = torch.zeros(8 * N, device=DEV)
        step = torch.full((1,), 5, dtype=torch.int32, device=DEV)
        opts = _lib.fit_opts(10, check_every=4, psnr_target=target, cfg=_lib.adam_cfg(LR))
        st = _lib.fit_frame(f.shape, dev(frame), *P, M, V, step, trace, f.ws, opts, check=False)
        torch.cuda.synchronize()
        assert st.code == _lib.GS2D_EINVAL, (target, st.code)
        assert np.all(host(buf)[8:] == -7.0)
        if target > 0:
            assert int(step.item()) == 5 and np.array_equal(host(P[0]), xy)
        else:
            assert int(step.item()) == 15 and np.all(host(buf)[5:8] > 0)


def test_fit_frame_1080p_matches_separate_calls():
    """1920x1080 / 30k Gaussians from the content-aware init, in the launch
    configuration the fitting benchmark times (tile 32, 2 px per lane, one
    graph-replayed chunk in which each Adam step runs inside the next
    iteration's projection kernel): 4 iterations of gs2d_fit_frame against
    the same 4 iterations as separate gs2d_project_bin, gs2d_render_fused and
    gs2d_adam_step calls (each pinned to the oracle by the tests above).
    Loss trace, parameters and moments agree up to the order of the float
    atomics that accumulate the gradients."""
    print("fit_frame 1080p vs separate calls", flush=True)
    from paper_2505_09324_amd import workloads
    W, H, N, K = 1920, 1080, 30000, 4
    f, m = synth.make_frame_torch(W, H, 61, 0, DEV)
    p0 = [p.contiguous() for p in workloads.plain_init_dev(f, m, N, 62)]
    shape = _lib.make_shape(W, H, N, 32, px_per_lane=2)
    lr = (2e-2, 5e-3, 5e-3)
    cfg = _lib.adam_cfg(lr)
    # the fitting loop
    pa = [q.clone() for q in p0]
    ma, va = torch.zeros(8 * N, device=DEV), torch.zeros(8 * N, device=DEV)
    sa = torch.zeros(1, dtype=torch.int32, device=DEV)
    tra = torch.zeros(K + 8, device=DEV)
    st = _lib.fit_frame(shape, f, *pa, ma, va, sa, tra, _lib.alloc_workspace(shape),
                        _lib.fit_opts(K, K, cfg=cfg))
    assert st.iters_run == K and st.status == 0
    # the same steps through the separate entry points
    ws = _lib.alloc_workspace(shape)
    pb = [q.clone() for q in p0]
    mb, vb = torch.zeros(8 * N, device=DEV), torch.zeros(8 * N, device=DEV)
    sb = torch.zeros(1, dtype=torch.int32, device=DEV)
    g = [torch.zeros(N, d, device=DEV) for d in (2, 3, 3)]
    losses = []
    for _ in range(K):
        _lib.project_bin(shape, pb[0], pb[1], ws)
        loss = torch.zeros((), device=DEV)
        _lib.render_fused(shape, ws, pb[2], f, *g, loss=loss)
        losses.append(float(loss))
        _lib.adam_step(*pb, *g, mb, vb, sb, cfg, zero_grads=True)
    torch.cuda.synchronize()
    assert int(sa.item()) == int(sb.item()) == K
    np.testing.assert_allclose(host(tra)[:K], losses, rtol=1e-5)
    for (name, a, b), step in zip((("xy", pa[0], pb[0]), ("chol", pa[1], pb[1]),
                                   ("rgb", pa[2], pb[2])), lr):
        a, b = host(a), host(b)
        err = np.abs(a - b)
        assert np.all(err <= 1e-3 * step + 1e-6 * np.abs(b)), (name, err.max())
    for a, b in ((ma, mb), (va, vb)):
        a, b = host(a), host(b)
        assert np.abs(a - b).max() <= 1e-4 * np.abs(b).max() + 1e-12
