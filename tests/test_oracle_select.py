"""Pins of the P-frame selection oracle (Sec. 3.2.C): the change mask and the
set of reference Gaussians that influence a changed pixel."""
import numpy as np
from scipy.stats import multivariate_normal

from oracle.select import changed_pixels, influence_q, select, selected_gaussians

F32 = np.float32


def test_change_is_strictly_above_threshold_on_some_channel():
    prev = np.zeros((3, 2, 4), F32)
    cur = prev.copy()
    cur[0, 0, 0] = F32(0.25)                       # exactly tau: unchanged
    cur[1, 0, 1] = np.nextafter(F32(0.25), F32(1))  # one ulp above: changed
    cur[2, 0, 2] = F32(-0.5)                       # |d| above, negative change
    cur[:, 0, 3] = F32(0.1)                        # every channel below
    cur[0, 1, 0] = np.nan                          # not comparable: unchanged
    cur[1, 1, 2] = np.nan                          # a NaN channel does not veto another
    cur[2, 1, 2] = F32(0.75)
    cur[:, 1, 1] = [F32(0.0), F32(0.3), F32(0.0)]  # one channel decides
    got = changed_pixels(cur, prev, 0.25)
    want = np.array([[False, True, True, False], [False, True, True, False]])
    np.testing.assert_array_equal(got, want)


def test_cutoff_boundary_is_inclusive_and_exact_in_fp32():
    # l = (2, 0, 2): the pixel centre 6 px right of the mean has u1 = 3 exactly, q = 9
    chol = np.array([[2, 0, 2]], F32)
    on = np.array([[4.5, 5.5]], F32)               # pixel (10, 5): dx = 6, dy = 0
    off = np.array([[F32(4.5) - F32(2.0 ** -10), 5.5]], F32)
    mask = np.zeros((8, 16), bool)
    mask[5, 10] = True
    assert influence_q(on, chol, [10], [5])[0, 0] == F32(9.0)
    assert selected_gaussians(on, chol, mask)[0]
    assert influence_q(off, chol, [10], [5])[0, 0] > F32(9.0)
    assert not selected_gaussians(off, chol, mask)[0]
    # along y through l3 with l2 = 0: l = (1, 0, 0.5), dy = 1.5 -> u2 = 3
    xy = np.array([[3.5, 2.0]], F32)
    mask = np.zeros((8, 8), bool)
    mask[3, 3] = True                              # centre (3.5, 3.5): dx = 0, dy = 1.5
    assert influence_q(xy, np.array([[1, 0, 0.5]], F32), [3], [3])[0, 0] == F32(9.0)
    assert selected_gaussians(xy, np.array([[1, 0, 0.5]], F32), mask)[0]
    assert not selected_gaussians(xy, np.array([[1, 0, 0.4990234375]], F32), mask)[0]


def test_selection_agrees_with_an_independent_density_evaluation():
    """q from scipy's Gaussian log-density (q = 2 (log p(mu) - log p(x)) with
    Sigma = L L^T, Eq. 1): every Gaussian whose nearest changed pixel is not
    within 1e-4 of the q = 9 boundary is selected iff some changed pixel has
    q <= 9."""
    rng = np.random.default_rng(3)
    W, H, N = 48, 40, 120
    xy = np.stack([rng.uniform(-6, W + 6, N), rng.uniform(-6, H + 6, N)], 1).astype(F32)
    chol = np.stack([rng.uniform(0.4, 4, N), rng.uniform(-2, 2, N), rng.uniform(0.4, 4, N)],
                    1).astype(F32)
    prev = rng.uniform(0, 1, (3, H, W)).astype(F32)
    cur = prev.copy()
    blob = np.zeros((H, W), bool)
    blob[10:18, 20:31] = True
    blob[30, 5] = True
    cur[1][blob] += F32(0.2)
    ch, sel = select(cur, prev, 0.1, xy, chol)
    np.testing.assert_array_equal(ch, blob)
    ys, xs = np.nonzero(blob)
    pts = np.stack([xs + 0.5, ys + 0.5], 1)
    checked = 0
    for n in range(N):
        l1, l2, l3 = (float(c) for c in chol[n])
        cov = np.array([[l1 * l1, l1 * l2], [l1 * l2, l2 * l2 + l3 * l3]])
        mvn = multivariate_normal(mean=xy[n].astype(float), cov=cov)
        q = 2.0 * (mvn.logpdf(xy[n].astype(float)) - mvn.logpdf(pts))
        if np.min(np.abs(q - 9.0)) <= 1e-4:
            continue
        assert sel[n] == bool(np.any(q <= 9.0)), n
        checked += 1
    assert checked >= N - 2 and 5 < sel.sum() < N - 5


def test_degenerate_thresholds_and_culled_gaussians():
    rng = np.random.default_rng(4)
    W, H, N = 24, 20, 40
    xy = np.stack([rng.uniform(0, W, N), rng.uniform(0, H, N)], 1).astype(F32)
    chol = np.stack([rng.uniform(0.5, 2, N), np.zeros(N), rng.uniform(0.5, 2, N)], 1).astype(F32)
    xy[3] = [np.nan, 5]                          # culled: non-finite mean
    chol[4, 0] = 0                               # culled: singular covariance
    xy[5] = [-40, -40]                           # reaches no pixel
    a = rng.uniform(0, 1, (3, H, W)).astype(F32)
    b = rng.uniform(0, 1, (3, H, W)).astype(F32)
    ch, sel = select(a, b, 2.0, xy, chol)        # nothing changes by more than 1
    assert not ch.any() and not sel.any()
    ch, sel = select(a, b, -1.0, xy, chol)       # every pixel changed
    assert ch.all()
    want = np.ones(N, bool)
    want[[3, 4, 5]] = False                      # all others have their mean in the frame
    np.testing.assert_array_equal(sel, want)


def test_masked_fit_keeps_inactive_gaussians_and_moves_the_rest():
    """The loop with an active mask (Sec. 3.2.C): inactive Gaussians keep
    their parameters exactly through every step; the active ones equal an
    unmasked fit's first step (Adam's update is per parameter)."""
    from oracle.fit import fit
    from paper_2505_09324_amd import synth
    frame, _ = synth.make_frame(32, 24, seed=5)
    xy, chol, rgb = synth.random_gaussians(30, 32, 24, seed=6)
    act = np.zeros(30, bool)
    act[::3] = True
    th, losses = fit(xy, chol, rgb, frame, 3, lr=1e-2, active=act)
    for k, a in (("xy", xy), ("chol", chol), ("rgb", rgb)):
        np.testing.assert_array_equal(th[k][~act], np.asarray(a, np.float64)[~act])
        assert np.all(np.any(th[k][act] != np.asarray(a, np.float64)[act], axis=1))
    th1, _ = fit(xy, chol, rgb, frame, 1, lr=1e-2, active=act)
    full, _ = fit(xy, chol, rgb, frame, 1, lr=1e-2)
    for k in th1:
        np.testing.assert_array_equal(th1[k][act], full[k][act])
    assert losses[2] < losses[0]
