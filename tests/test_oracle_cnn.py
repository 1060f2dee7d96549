"""Pins for the learned-initialiser oracle: convolution against scipy's
correlate2d, identity and delta kernels, BF16 rounding against known values,
Chamfer and cross-entropy closed forms, and finite differences."""
import math

import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn


def test_bf16_round_known_values():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.140625, 1e-3], np.float32)
    r = cnn.bf16_round(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                    # tie -> even (mantissa 0)
    assert r[2] == 1.0 + 2 ** -7          # 1.5 ulp -> rounds up
    assert r[3] == -2.5
    assert r[4] == 3.140625               # exactly representable (8 bits)
    assert abs(r[5] - 1e-3) / 1e-3 < 2 ** -8


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_matches_scipy_correlate(stride):
    """P11: cross-correlation convention and padding against scipy."""
    rng = np.random.default_rng(0)
    x = rng.normal(size=(3, 11, 14))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    y = cnn.conv3x3(x, w, b, stride)
    for o in range(4):
        ref = sum(correlate2d(x[c], w[o, c], mode="same") for c in range(3)) + b[o]
        np.testing.assert_allclose(y[o], ref[::stride, ::stride], rtol=1e-12, atol=1e-12)
    assert y.shape[1:] == (math.ceil(11 / stride), math.ceil(14 / stride))


def test_identity_and_delta_kernels():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 6, 7))
    w = np.zeros((2, 2, 3, 3))
    w[0, 0, 1, 1] = w[1, 1, 1, 1] = 1.0
    np.testing.assert_array_equal(cnn.conv3x3(x, w, np.zeros(2), 1), x)
    delta = np.zeros((1, 7, 7))
    delta[0, 3, 3] = 1.0
    k = rng.normal(size=(1, 1, 3, 3))
    y = cnn.conv3x3(delta, k, np.zeros(1), 1)
    # cross-correlation: the response to a delta is the kernel rotated by 180
    np.testing.assert_array_equal(y[0, 2:5, 2:5], k[0, 0, ::-1, ::-1])


def test_conv_backward_matches_fd():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(3, 7, 8))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    for stride in (1, 2):
        dy = rng.normal(size=cnn.conv3x3(x, w, b, stride).shape)
        dx, dw, db = cnn.conv3x3_backward(x, w, dy, stride)
        f = lambda xx, ww, bb: float((dy * cnn.conv3x3(xx, ww, bb, stride)).sum())
        h = 1e-6
        for idx in [(0, 0, 0), (2, 6, 7), (1, 3, 4)]:
            e = np.zeros_like(x)
            e[idx] = h
            assert (f(x + e, w, b) - f(x - e, w, b)) / (2 * h) == pytest.approx(dx[idx], rel=1e-6, abs=1e-9)
        for idx in [(0, 0, 0, 0), (3, 2, 2, 1), (1, 1, 0, 2)]:
            e = np.zeros_like(w)
            e[idx] = h
            assert (f(x, w + e, b) - f(x, w - e, b)) / (2 * h) == pytest.approx(dw[idx], rel=1e-6, abs=1e-9)
        np.testing.assert_allclose(db, dy.sum(axis=(1, 2)))


def test_chamfer_closed_forms():
    """P12: identical sets -> 0; single points -> 2|p-q|^2; permutation
    invariant; gradient by FD."""
    rng = np.random.default_rng(3)
    P = rng.normal(size=(5, 8))
    assert cnn.chamfer(P, P)[0] == 0.0
    p, q = rng.normal(size=(1, 8)), rng.normal(size=(1, 8))
    assert cnn.chamfer(p, q)[0] == pytest.approx(2 * ((p - q) ** 2).sum())
    Q = rng.normal(size=(5, 8))
    perm = rng.permutation(5)
    assert cnn.chamfer(P[perm], Q)[0] == pytest.approx(cnn.chamfer(P, Q)[0])
    _, g = cnn.chamfer(P, Q)
    h = 1e-6
    for i, j in [(0, 0), (4, 7), (2, 3)]:
        e = np.zeros_like(P)
        e[i, j] = h
        fd = (cnn.chamfer(P + e, Q)[0] - cnn.chamfer(P - e, Q)[0]) / (2 * h)
        assert fd == pytest.approx(g[i, j], rel=1e-6, abs=1e-10)


def test_cross_entropy_uniform_and_gradient():
    ce, g = cnn.cross_entropy(np.zeros(9), 4)
    assert ce == pytest.approx(math.log(9))
    np.testing.assert_allclose(g, np.full(9, 1 / 9) - np.eye(9)[4])


def test_network_gradient_matches_fd():
    """Loss through the tiny network (FP64, no BF16 rounding) vs FD."""
    rng = np.random.default_rng(4)
    x = rng.normal(size=(6, 32, 32)) * 0.5
    chans = [6, 8, 8, 8, 8]
    params = []
    for i in range(4):
        params.append((rng.normal(size=(chans[i + 1], chans[i], 3, 3)) * 0.3, rng.normal(size=chans[i + 1]) * 0.1))
    params.append((rng.normal(size=(cnn.HEAD_CH, 8, 3, 3)) * 0.3, rng.normal(size=cnn.HEAD_CH) * 0.1))
    targets = {0: rng.normal(size=(2, 8)), 3: rng.normal(size=(1, 8))}

    def loss_of(ps):
        head, _ = cnn.forward(x, ps, bf16=False)
        return cnn.head_loss(head, targets)[0]

    head, _ = cnn.forward(x, params, bf16=False)
    _, hg = cnn.head_loss(head, targets)
    grads = cnn.backward(x, params, hg, bf16=False)
    h = 1e-6
    for li, idx in [(0, (3, 2, 1, 1)), (2, (1, 5, 0, 2)), (4, (10, 3, 1, 0)), (4, (0, 7, 2, 2))]:
        w, b = params[li]
        e = np.zeros_like(w)
        e[idx] = h
        pp = list(params)
        pp[li] = (w + e, b)
        pm = list(params)
        pm[li] = (w - e, b)
        fd = (loss_of(pp) - loss_of(pm)) / (2 * h)
        assert fd == pytest.approx(grads[li][0][idx], rel=1e-5, abs=1e-9)
    w, b = params[4]
    e = np.zeros_like(b)
    e[12] = h
    pp = list(params)
    pp[4] = (w, b + e)
    pm = list(params)
    pm[4] = (w, b - e)
    assert (loss_of(pp) - loss_of(pm)) / (2 * h) == pytest.approx(grads[4][1][12], rel=1e-5, abs=1e-9)


def test_tile_targets_selection():
    xy = np.array([[3.0, 4.0], [20.0, 5.0]] + [[8.0, 8.0]] * 9)
    chol = np.array([[1.0, 0.0, 1.0]] * 11)
    chol[2:, 0] = np.arange(1, 10)
    rgb = np.ones((11, 3))
    t = cnn.tile_targets(xy, chol, rgb, 32, 16, 16)
    assert sorted(t) == [0, 1]
    assert t[0].shape == (8, 8)           # 10 in tile 0, the 8 heaviest kept
    assert t[1][0, 0] == pytest.approx((20.0 - 16) / 16)


def _logit(p):
    return math.log(p / (1.0 - p))


def test_decode_inverts_the_slot_parameterisation():
    """A head written from known Gaussians by inverting the documented slot
    parameterisation (centre = tile origin + T sigmoid, scales = exp, count =
    argmax of one-hot logits) must decode to exactly those Gaussians, in tile
    order then slot order, topped up from the plain set."""
    T, W, H = 16, 48, 32
    TX, TY = W // T, H // T
    rng = np.random.default_rng(3)
    head = np.zeros((cnn.HEAD_CH, TY, TX))
    expect = []
    counts = {0: 2, 1: 0, 2: 3, 3: 1, 4: 0, 5: 2}
    for t in range(TX * TY):
        ty, tx = divmod(t, TX)
        k = counts[t]
        head[:9, ty, tx] = -1.0
        head[k, ty, tx] = 5.0
        for s in range(k):
            fx, fy = rng.uniform(0.1, 0.9, 2)
            l1, l3 = rng.uniform(0.5, 4.0, 2)
            l2 = rng.uniform(-1, 1)
            c = rng.uniform(0, 1, 3)
            head[9 + 8 * s:9 + 8 * s + 8, ty, tx] = (_logit(fx), _logit(fy), math.log(l1), l2,
                                                      math.log(l3), *c)
            expect.append((tx * T + T * fx, ty * T + T * fy, l1, l2, l3, *c))
        # slots beyond the count carry garbage that must be ignored
        for s in range(k, 8):
            head[9 + 8 * s:9 + 8 * s + 8, ty, tx] = 1e3
    expect = np.array(expect)
    n_pred = len(expect)                  # 8
    N = 12
    plain = (rng.uniform(0, 40, (N, 2)), rng.uniform(1, 2, (N, 3)), rng.uniform(0, 1, (N, 3)))
    xy, chol, rgb, used = cnn.decode(head, N, plain, T)
    assert used == n_pred
    np.testing.assert_allclose(xy[:n_pred], expect[:, 0:2], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(chol[:n_pred], expect[:, 2:5], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(rgb[:n_pred], expect[:, 5:8], rtol=1e-12, atol=1e-12)
    # top-up: the first N - n_pred plain Gaussians, in order
    np.testing.assert_array_equal(xy[n_pred:], plain[0][:N - n_pred])
    np.testing.assert_array_equal(chol[n_pred:], plain[1][:N - n_pred])
    # more predictions than N: trimmed to the first N in tile order
    xy2, _, _, used2 = cnn.decode(head, 5, plain, T)
    assert used2 == 5
    np.testing.assert_allclose(xy2, expect[:5, 0:2], rtol=1e-12, atol=1e-12)
    # fewer than N/2 predictions: the plain set unchanged
    big = (np.zeros((40, 2)), np.ones((40, 3)), np.zeros((40, 3)))
    xy3, chol3, _, used3 = cnn.decode(head, 40, big, T)
    assert used3 == 0 and np.array_equal(xy3, big[0]) and np.array_equal(chol3, big[1])
    # a non-finite prediction also falls back
    bad = head.copy()
    bad[9 + 3, 0, 0] = np.nan
    _, _, _, used4 = cnn.decode(bad, N, plain, T)
    assert used4 == 0


def test_targets_round_trip_through_decode():
    """tile_targets and decode use the same tile-local encoding: a head
    built from the targets (one-hot counts, slots by inverting the encoding)
    decodes back to the selected Gaussians."""
    T, W, H = 16, 64, 48
    rng = np.random.default_rng(9)
    n = 60
    xy = np.stack([rng.uniform(0, W, n), rng.uniform(0, H, n)], 1)
    chol = np.stack([rng.uniform(0.5, 3, n), rng.uniform(-1, 1, n), rng.uniform(0.5, 3, n)], 1)
    rgb = rng.uniform(0, 1, (n, 3))
    tg = cnn.tile_targets(xy, chol, rgb, W, H, T)
    TX, TY = W // T, H // T
    head = np.full((cnn.HEAD_CH, TY, TX), 0.0)
    head[:9] = -1.0
    expect = []
    for t in range(TX * TY):
        ty, tx = divmod(t, TX)
        v = tg.get(t, np.zeros((0, 8)))
        head[len(v), ty, tx] = 3.0
        for s, row in enumerate(v):
            head[9 + 8 * s:9 + 8 * s + 8, ty, tx] = (_logit(row[0]), _logit(row[1]), *row[2:])
            expect.append(row)
    m = len(expect)
    got_xy, got_chol, got_rgb, used = cnn.decode(head, m, (xy, chol, rgb), T)
    assert used == m
    # every selected Gaussian comes back, and nothing else
    pts = {tuple(np.round(r, 9)) for r in np.concatenate([got_xy, got_chol, got_rgb], 1)}
    src = {tuple(np.round(np.concatenate([xy[i], chol[i], rgb[i]]), 9)) for i in range(n)}
    assert pts <= src and len(pts) == m
