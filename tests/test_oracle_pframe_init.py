"""Pins of the learned re-initialisation of P-frames: the per-tile residual
energy and the replacement of the warm-started Gaussians of the tiles it
selects (Sec. 3.2.B applied at P-frames, Sec. 3.2.C)."""
import math

import numpy as np

from oracle.cnn import N_PARAM, N_SLOTS, decode_slot, pframe_replace, sigmoid, tile_residual_energy

F32 = np.float32


def test_energy_closed_forms_and_ragged_tiles():
    H, W = 20, 37                                   # tiles 3 x 2, ragged on both axes
    prev = np.zeros((3, H, W), F32)
    frame = prev.copy()
    frame[0] += 0.5
    frame[1] += 0.25                                # e = 0.25 + 0.0625 = 0.3125 everywhere
    e = tile_residual_energy(frame, prev)
    assert e.shape == (2, 3)
    assert np.all(e == F32(0.3125))
    # one pixel of 0.75 in red in the full tile (0, 1): mean 0.5625 / 256
    f2 = prev.copy()
    f2[0, 3, 20] = 0.75
    e2 = tile_residual_energy(f2, prev)
    assert e2[0, 1] == F32(0.5625 / 256) and np.count_nonzero(e2) == 1
    # the same pixel in the ragged corner tile (1, 2): 4 x 5 pixels
    f3 = prev.copy()
    f3[0, 19, 36] = 0.75
    assert tile_residual_energy(f3, prev)[1, 2] == F32(0.5625 / 20)


def test_energy_against_fp64_brute_force():
    rng = np.random.default_rng(4)
    H, W = 45, 70
    a = rng.uniform(0, 1, (3, H, W)).astype(F32)
    b = rng.uniform(0, 1, (3, H, W)).astype(F32)
    e = tile_residual_energy(a, b)
    d = a.astype(np.float64) - b
    px = (d * d).sum(0)
    for ty in range(e.shape[0]):
        for tx in range(e.shape[1]):
            ref = px[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16].mean()
            assert abs(float(e[ty, tx]) - ref) <= 1e-5 * ref


def _head(TY, TX, counts, rng):
    """Head [73, TY, TX] whose first count maximum is counts[ty][tx]."""
    h = rng.normal(0, 1, (73, TY, TX))
    h[:9] = -5.0
    for ty in range(TY):
        for tx in range(TX):
            h[counts[ty][tx], ty, tx] = 5.0
    return h


def _frames(H, W, changed_tiles):
    prev = np.zeros((3, H, W), F32)
    frame = prev.copy()
    for ty, tx in changed_tiles:
        frame[:, ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16] = 0.1   # e = 0.03
    return frame, prev


def test_replacement_fills_freed_slots_in_order():
    rng = np.random.default_rng(1)
    H, W = 32, 48                                   # tiles 2 x 3
    frame, prev = _frames(H, W, [(0, 1), (1, 2)])
    head = _head(2, 3, [[2, 3, 1], [4, 0, 2]], rng)
    # Gaussians: 1, 4, 6 in tile (0, 1); 3 in (1, 2); the rest elsewhere,
    # off-frame or not finite
    xy = np.array([[5, 5], [20, 3], [40, 5], [45.5, 31], [16.0, 15.999], [15.999, 1],
                   [31.999, 0], [-1, 4], [np.nan, 3], [60, 20]], F32)
    N = len(xy)
    chol = rng.uniform(0.5, 2, (N, 3)).astype(F32)
    rgb = rng.uniform(0, 1, (N, 3)).astype(F32)
    nx, nc, nr, info = pframe_replace(frame, prev, head, xy, chol, rgb, tau=0.02)
    np.testing.assert_array_equal(info["selected"], [[False, True, False], [False, False, True]])
    np.testing.assert_array_equal(info["freed"], [1, 3, 4, 6])
    # predictions: tile (0, 1) slots 0..2, then tile (1, 2) slots 0..1
    preds = [decode_slot(head[9:, 0, 1].reshape(N_SLOTS, N_PARAM)[s], 1, 0) for s in range(3)]
    preds += [decode_slot(head[9:, 1, 2].reshape(N_SLOTS, N_PARAM)[s], 2, 1) for s in range(2)]
    assert info["n_predicted"] == 5 and info["replaced"] == 4
    for i, n in enumerate([1, 3, 4, 6]):
        np.testing.assert_array_equal(nx[n], preds[i][0:2])
        np.testing.assert_array_equal(nc[n], preds[i][2:5])
        np.testing.assert_array_equal(nr[n], preds[i][5:8])
    keep = [0, 2, 5, 7, 8, 9]
    np.testing.assert_array_equal(nx[keep], xy[keep].astype(np.float64))
    np.testing.assert_array_equal(nc[keep], chol[keep].astype(np.float64))
    # the slot decoding: centre inside its tile, scales exp(clamp(p, +-4))
    q = head[9:, 0, 1].reshape(N_SLOTS, N_PARAM)[0]
    assert preds[0][0] == 16 + 16 * sigmoid(q[0]) and preds[0][2] == math.exp(min(max(q[2], -4), 4))


def test_fewer_predictions_keep_the_rest_and_guards():
    rng = np.random.default_rng(2)
    H, W = 32, 32
    frame, prev = _frames(H, W, [(0, 0)])
    head = _head(2, 2, [[1, 8], [8, 8]], rng)
    xy = np.array([[1, 1], [2, 2], [3, 3], [20, 20]], F32)
    chol = np.ones((4, 3), F32)
    rgb = np.full((4, 3), 0.5, F32)
    nx, _, _, info = pframe_replace(frame, prev, head, xy, chol, rgb, tau=0.02)
    assert info["replaced"] == 1 and list(info["freed"]) == [0, 1, 2]
    np.testing.assert_array_equal(nx[1:], xy[1:].astype(np.float64))
    # tau is strict: a tile whose mean equals tau is not selected
    e = tile_residual_energy(frame, prev)[0, 0]
    _, _, _, info = pframe_replace(frame, prev, head, xy, chol, rgb, tau=float(e))
    assert info["replaced"] == 0 and not info["selected"].any()
    # nothing changed: nothing selected
    _, _, _, info = pframe_replace(prev, prev, head, xy, chol, rgb, tau=0.0)
    assert not info["selected"].any() and info["replaced"] == 0
    # a non-finite raw parameter of a used slot: nothing replaced
    bad = head.copy()
    bad[9 + 3, 0, 0] = np.inf
    nx, _, _, info = pframe_replace(frame, prev, bad, xy, chol, rgb, tau=0.02)
    assert info["replaced"] == 0
    np.testing.assert_array_equal(nx, xy.astype(np.float64))
    # ... but a non-finite parameter of an unused slot does not matter
    bad = head.copy()
    bad[9 + 8 + 3, 0, 0] = np.nan
    _, _, _, info = pframe_replace(frame, prev, bad, xy, chol, rgb, tau=0.02)
    assert info["replaced"] == 1
