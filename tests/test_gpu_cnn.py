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
# a frame whose sides are no multiple of 16, nor even at every layer (70 ->
# 35 -> 18 -> 9 -> 5, 117 -> 59 -> 30 -> 15 -> 8): ragged tiles and every
# stride-parity class of the grad-input kernels with odd extents
SIZES = [(96, 128), (70, 117)]
# the smallest frames the network accepts: a 1 x 1 and a 2 x 3 tile head,
# parity classes of extent 1 and layers whose input is a single pixel row
TINY = [(16, 16), (17, 33)]


def _frames(seed, hw=(H, W)):
    h, w = hw
    f0, _ = synth.make_frame(w, h, seed=seed, t=0)
    f1, _ = synth.make_frame(w, h, seed=seed, t=3)
    return f0, f1


def _x(f1, f0):
    return np.concatenate([f1, f1 - f0]).astype(np.float64)


@pytest.mark.parametrize("hw", SIZES + TINY)
def test_forward_matches_oracle(hw):
    h, w = hw
    print("cnn forward", hw, flush=True)
    f0, f1 = _frames(41, hw)
    net = _lib.CNNInit(h, w, seed=5)
    head = torch.empty(73, net.TY, net.TX, device=DEV)
    net.forward(dev(f1), dev(f0), head_out=head)
    torch.cuda.synchronize()
    ref, _ = ocnn.forward(_x(f1, f0), net.oracle_params(), bf16=True)
    got = host(head)
    assert got.shape == ref.shape == (73, (h + 15) // 16, (w + 15) // 16)
    scale = np.abs(ref).mean()
    assert np.abs(got - ref).max() <= 2e-2 * scale, np.abs(got - ref).max() / scale


def test_forward_1080p_matches_oracle_on_crops():
    """Full 1920 x 1080 frame, the launch shapes training and inference use.
    A head output depends on input pixels within 31 px of its tile (four
    stride-2 layers and the 3x3 head), so on a 256-px crop whose origin is a
    multiple of 16 the oracle reproduces every tile at least 32 px inside
    the crop, and every tile along a crop edge that is also the frame's edge."""
    print("cnn forward 1080p", flush=True)
    Hf, Wf = 1080, 1920
    f0, _ = synth.make_frame(Wf, Hf, seed=47, t=0)
    f1, _ = synth.make_frame(Wf, Hf, seed=47, t=2)
    net = _lib.CNNInit(Hf, Wf, seed=12)
    head = torch.empty(73, net.TY, net.TX, device=DEV)
    net.forward(dev(f1), dev(f0), head_out=head)
    torch.cuda.synchronize()
    got = host(head)
    assert got.shape == (73, 68, 120)
    params = net.oracle_params()
    x = _x(f1, f0)
    checked = 0
    # crop origins (pixels): top-left corner, interior, bottom-right corner
    for y0, x0 in [(0, 0), (400, 912), (Hf - 248, Wf - 256)]:
        ch, cw = min(256, Hf - y0), min(256, Wf - x0)
        ref, _ = ocnn.forward(x[:, y0:y0 + ch, x0:x0 + cw], params, bf16=True)
        ty0, tx0 = y0 // 16, x0 // 16
        lo_y = 0 if y0 == 0 else 2
        lo_x = 0 if x0 == 0 else 2
        hi_y = ref.shape[1] if y0 + ch == Hf else 15
        hi_x = ref.shape[2] if x0 + cw == Wf else 15
        g = got[:, ty0 + lo_y:ty0 + hi_y, tx0 + lo_x:tx0 + hi_x]
        r = ref[:, lo_y:hi_y, lo_x:hi_x]
        scale = np.abs(r).mean()
        assert np.abs(g - r).max() <= 2e-2 * scale, (y0, x0, np.abs(g - r).max() / scale)
        checked += r.shape[1] * r.shape[2]
    assert checked >= 3 * 13 * 13


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


# 288 x 352: layer 0's 144 x 176 outputs make 50 pixel splits of the grad-
# weight GEMM, so its partial tiles are summed in two chunks (combined with
# atomics), as at full resolution
@pytest.mark.parametrize("hw", SIZES + TINY + [(288, 352)])
def test_backward_matches_oracle(hw):
    H, W = hw
    print("cnn backward", hw, flush=True)
    f0, f1 = _frames(43, hw)
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


def test_trained_initialiser_beats_plain_init_at_fixed_budget():
    """What the learned initialiser gains over the method without it, at
    small scale and on scenes it never saw: the plain fitter fits 12
    synthetic 256 x 256 sequences of 8 frames (frame 0 from the
    content-aware init, then warm-started), the network is trained on those
    fits with the project's own kernels, and on frames of three held-out
    sequences (other seeds: other colours, texture and pose) the fitter
    started from the decoded prediction reaches a higher PSNR after a fixed
    number of iterations than the fitter started from the content-aware
    init.  The same frames also report the learned re-initialisation of a
    warm start (the previous frame's fit, the changed tiles replaced from
    the network) against the warm start alone; at this scale, as at 1080p,
    it does not beat it, so that comparison is printed, not asserted."""
    print("learned init gain", flush=True)
    from paper_2505_09324_amd import workloads
    W = H = 256
    N = 1500
    seqs = list(range(7000, 7012))
    frames = {}
    samples = workloads.make_training_set(seqs, 8, W, H, N, 400, 100, DEV, log=lambda m: None,
                                          frames=frames)
    net = _lib.CNNInit(H, W, seed=3)
    hist = workloads.train_initialiser(net, samples, W, H, 15, 3e-3, DEV, log=lambda m: None,
                                       frames=frames)
    assert hist[-1] < 0.7 * hist[0], hist
    shape = _lib.make_shape(W, H, N, 16, px_per_lane=1)
    ws = _lib.alloc_workspace(shape)
    cfg = _lib.adam_cfg(workloads.LR_DEFAULT)
    gains = {20: [], 50: [], 100: []}
    warm = {20: [], 50: [], 100: []}
    for sd in (7100, 7101, 7102):
        for t in (3, 5):
            f, m = synth.make_frame_torch(W, H, sd, t, DEV)
            prev, pm = synth.make_frame_torch(W, H, sd, t - 1, DEV)
            plain = [p.contiguous() for p in workloads.plain_init_dev(f, m, N, 99 + t)]
            net.forward(f, prev)
            xy, chol, rgb, npred = net.decode(N, *plain)
            assert int(npred.item()) >= N // 2  # the prediction is used, not the fallback
            cp = workloads.psnr_curve(shape, ws, f, plain, 101, tuple(gains), cfg)
            cl = workloads.psnr_curve(shape, ws, f, [xy, chol, rgb], 101, tuple(gains), cfg)
            for k in gains:
                gains[k].append(cl[k] - cp[k])
            # warm start: the previous frame fitted from its own plain init
            wp = [p.contiguous() for p in workloads.plain_init_dev(prev, pm, N, 199 + t)]
            mm = torch.zeros(8 * N, device=DEV)
            vv = torch.zeros(8 * N, device=DEV)
            stp = torch.zeros(1, dtype=torch.int32, device=DEV)
            trc = torch.zeros(500, device=DEV)
            _lib.fit_frame(shape, prev, *wp, mm, vv, stp, trc, ws, _lib.fit_opts(400, 50, cfg=cfg))
            rp = [p.clone() for p in wp]
            net.pframe_replace(f, prev, 1e-3, *rp)
            cw = workloads.psnr_curve(shape, ws, f, wp, 101, tuple(warm), cfg)
            cr = workloads.psnr_curve(shape, ws, f, rp, 101, tuple(warm), cfg)
            for k in warm:
                warm[k].append(cr[k] - cw[k])
    print("learned vs plain, cold:", {k: [round(x, 2) for x in v] for k, v in gains.items()},
          flush=True)
    print("learned re-initialisation vs warm start:",
          {k: [round(x, 2) for x in v] for k, v in warm.items()}, flush=True)
    # one measurement: +0.47 dB mean after 50 iterations (4 of 6 frames
    # ahead, both frames of one scene behind), +0.82 dB after 100; the
    # training itself is not bit-reproducible (float atomics)
    assert sum(g > 0 for g in gains[50]) >= 3, gains
    assert np.mean(gains[100]) > 0.25, gains


def _half_ulp_bf16(x):
    """Half a bfloat16 unit in the last place at magnitude |x| (normal
    range): bfloat16 keeps 8 significant bits."""
    a = np.maximum(np.abs(x), 2.0 ** -126)
    return 0.5 * 2.0 ** (np.floor(np.log2(a)) - 7)


def _close_bf16(got, want, acc, what):
    """A BF16 output rounded once from an FP32 accumulation: within half a
    BF16 ulp of (|want| + acc) plus the accumulation bound acc."""
    bound = _half_ulp_bf16(np.abs(want) + acc) + acc + 1e-30
    err = np.abs(got.astype(np.float64) - want)
    bad = err > bound
    assert not bad.any(), (what, int(bad.sum()), bad.size, float((err - bound)[bad].max()))


def _chamfer_ties(head, targets, rel=1e-4):
    """Slot rows of the head whose Chamfer gradient depends on a nearest-
    neighbour choice that is within `rel` of a tie (FP32 and FP64 may pick
    differently there): boolean [8, TY, TX]."""
    _, TY, TX = head.shape
    amb = np.zeros((8, TY, TX), bool)
    for t, Q in targets.items():
        ty, tx = divmod(t, TX)
        k = len(Q)
        if k == 0:
            continue
        _, P = ocnn.slot_vectors(head[:, ty, tx].astype(np.float64))
        d = ((P[:k, None, :] - np.asarray(Q)[None]) ** 2).sum(-1)
        for i in range(k):                     # nearest target of each slot
            s = np.sort(d[i])
            if k > 1 and s[1] - s[0] <= rel * max(s[1], 1e-30):
                amb[i, ty, tx] = True
        for j in range(k):                     # nearest slot of each target
            s = np.argsort(d[:, j])
            if k > 1 and d[s[1], j] - d[s[0], j] <= rel * max(d[s[1], j], 1e-30):
                amb[s[0], ty, tx] = amb[s[1], ty, tx] = True
    return amb


@pytest.mark.parametrize("hw", SIZES + TINY + [(288, 352)])
def test_layers_elementwise_against_oracle(hw):
    """Every convolution pass checked element by element, one layer at a
    time, on the GPU's own BF16 operands: each layer's input activations
    and output gradient are read from the workspace and fed to the oracle's
    direct convolution and its backward.
      - forward: the next layer's BF16 input equals bf16(ReLU(conv)) and the
        head equals conv, within half a BF16 ulp plus 1e-3 sum|w x|;
      - head gradient: the loss gradient of every head channel (slots whose
        Chamfer nearest neighbour is within 1e-4 of a tie excepted);
      - grad input: each hidden layer's BF16 dZ equals bf16(mask * W^T dZ);
      - grad weight and bias: every element within 1e-3 sum|dZ x|."""
    H, W = hw
    print("cnn layers element-wise", hw, flush=True)
    f0, f1 = _frames(49, hw)
    xy, chol, rgb = synth.random_gaussians(700, W, H, seed=50, scale_lo=0.6, scale_hi=3.0)
    net = _lib.CNNInit(H, W, seed=51)
    net.set_targets(dev(xy), dev(chol), dev(rgb))
    head = torch.empty(73, net.TY, net.TX, device=DEV)
    net.forward(dev(f1), dev(f0), head_out=head)
    net.backward()
    torch.cuda.synchronize()
    params = net.oracle_params()
    grads = net.oracle_grads()
    hd = host(head).astype(np.float64)
    # input of layer 0: the frame and the residual, BF16-rounded
    X0 = net.tensor(0, 0)
    assert X0.shape[0] == 8 and not X0[6:].any()
    np.testing.assert_array_equal(X0[:6], ocnn.bf16_round(_x(f1, f0)))
    X = [net.tensor(i, 0).astype(np.float64) for i in range(5)]
    X[0] = X[0][:6]
    for i, (w, b) in enumerate(params):
        wq = ocnn.bf16_round(w).astype(np.float64)
        stride = 2 if i < 4 else 1
        y = ocnn.conv3x3(X[i], wq, b, stride)
        acc = 1e-3 * ocnn.conv3x3(np.abs(X[i]), np.abs(wq), np.abs(b), stride)
        if i < 4:
            _close_bf16(X[i + 1], np.maximum(y, 0.0), acc, f"forward layer {i}")
        else:
            assert np.all(np.abs(hd - y) <= acc + 1e-30), "head"
    # loss gradient of the head, from the GPU's head output
    targets = ocnn.tile_targets(xy, chol, rgb, W, H, 16)
    _, hg = ocnn.head_loss(hd, targets)
    DZ4 = net.tensor(4, 1)[:73].astype(np.float64)
    keep = np.ones_like(hg, bool)
    amb = _chamfer_ties(hd, targets)
    for s in range(8):
        keep[9 + 8 * s:17 + 8 * s] &= ~amb[s][None]
    _close_bf16(DZ4[keep], hg[keep], 1e-5 * np.abs(hg[keep]), "head dZ")
    assert keep.mean() > 0.9
    # backward, layer by layer, from the GPU's own dZ
    for i in range(4, -1, -1):
        w, _ = params[i]
        wq = ocnn.bf16_round(w).astype(np.float64)
        stride = 2 if i < 4 else 1
        cout = 73 if i == 4 else 64
        DZ = net.tensor(i, 1)[:cout].astype(np.float64)
        dx, dw, db = ocnn.conv3x3_backward(X[i], wq, DZ, stride)
        adx, adw, adb = ocnn.conv3x3_backward(np.abs(X[i]), np.abs(wq), np.abs(DZ), stride)
        gw, gb = grads[i]
        assert np.all(np.abs(gw - dw) <= 1e-3 * adw + 1e-30), f"grad weight {i}"
        assert np.all(np.abs(gb - db) <= 1e-3 * adb + 1e-30), f"grad bias {i}"
        if i > 0:
            mask = X[i] > 0
            got = net.tensor(i - 1, 1)[:64]
            assert not got[~mask].any(), f"grad input {i}: masked entries not zero"
            _close_bf16(got[mask], dx[mask], 1e-3 * adx[mask], f"grad input into layer {i}")


def test_cnn_adam_matches_oracle_decoupled_decay():
    """Three Adam steps on the FP32 master weights with decoupled weight
    decay, each against the oracle fed the GPU's state (parameters within
    1e-6 relative plus 1e-6 lr; moments relative to their two terms); the
    gradient is cleared and both BF16 weight copies equal the rounded
    master weights."""
    print("cnn adam", flush=True)
    from oracle.adam import adamw_step
    net = _lib.CNNInit(H, W, seed=52)
    rng = np.random.default_rng(53)
    n = net.n_params
    lr, wd = 2e-3, 0.05
    t = 0
    for k in range(3):
        p0 = host(net.master).astype(np.float64)
        m0 = host(net.m).astype(np.float64)
        v0 = host(net.v).astype(np.float64)
        g = rng.normal(size=n).astype(np.float32) * np.float32(10.0 ** rng.uniform(-3, 1))
        net.grad.copy_(torch.from_numpy(g))
        net.step(lr=lr, weight_decay=wd)
        torch.cuda.synchronize()
        lr32, wd32 = float(np.float32(lr)), float(np.float32(wd))
        p1, m1, v1, t = adamw_step(p0, g, m0, v0, t, lr32, wd32, float(np.float32(0.9)),
                                   float(np.float32(0.999)), float(np.float32(1e-8)))
        assert int(net.step_count.item()) == t
        assert np.all(np.abs(host(net.master) - p1) <= 1e-6 * np.abs(p1) + 1e-6 * lr), k
        gd = g.astype(np.float64)
        assert np.all(np.abs(host(net.m) - m1) <= 1e-6 * (0.9 * np.abs(m0) + 0.1 * np.abs(gd)))
        assert np.all(np.abs(host(net.v) - v1) <= 1e-5 * (0.999 * v0 + 0.001 * gd * gd))
        assert not host(net.grad).any()
    master = host(net.master)
    wb = host(net.wbf16).view(np.uint16)
    bits = lambda a: (ocnn.bf16_round(a).view(np.uint32) >> 16).astype(np.uint16)
    wb_off = wt_off = 0
    n_wb = sum(net.layer_info(i)["Mpad"] * net.layer_info(i)["Kf"] for i in range(5))
    for i in range(5):
        d = net.layer_info(i)
        M = master[d["w_off"]:d["w_off"] + d["Mpad"] * d["Kf"]]
        np.testing.assert_array_equal(wb[wb_off:wb_off + M.size], bits(M))
        cs = (d["Cout"] + 7) // 8 * 8
        kb = (9 * cs + 31) // 32 * 32
        if i > 0:
            wt = wb[n_wb + wt_off:n_wb + wt_off + d["Cin"] * kb].reshape(d["Cin"], kb)
            Mw = M.reshape(d["Mpad"], d["Kf"])
            for tap in range(9):
                want = bits(Mw[:d["Cout"], tap * d["Cin"]:(tap + 1) * d["Cin"]].T.copy())
                np.testing.assert_array_equal(wt[:, tap * cs:tap * cs + d["Cout"]], want)
        wb_off += M.size
        wt_off += d["Cin"] * kb
