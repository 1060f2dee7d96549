"""Pins for the oracle's optimiser step and loss/PSNR."""
import math

import numpy as np
import pytest
import torch

from oracle.adam import adam_step
from oracle.loss import dloss_dimg, mse, psnr, psnr_from_mse

LR = {"xy": 1e-2, "chol": 2e-3, "rgb": 5e-3}


def _state(rng, N=7):
    th = {"xy": rng.normal(size=(N, 2)), "chol": rng.normal(size=(N, 3)), "rgb": rng.normal(size=(N, 3))}
    z = {k: np.zeros_like(v) for k, v in th.items()}
    return th, z, {k: np.zeros_like(v) for k, v in th.items()}


def test_first_step_closed_form():
    """P8: t=1 gives delta = -lr g / (|g| + eps)."""
    rng = np.random.default_rng(0)
    th, m, v = _state(rng)
    g = {k: rng.normal(size=x.shape) for k, x in th.items()}
    th2, _, _, t = adam_step(th, g, m, v, 0, LR)
    assert t == 1
    for k in th:
        np.testing.assert_allclose(th2[k] - th[k], -LR[k] * g[k] / (np.abs(g[k]) + 1e-8),
                                   rtol=1e-9, atol=1e-15)


def test_constant_gradient_constant_step():
    rng = np.random.default_rng(1)
    th, m, v = _state(rng)
    g = {k: rng.normal(size=x.shape) for k, x in th.items()}
    t = 0
    prev = th
    for _ in range(6):
        nxt, m, v, t = adam_step(prev, g, m, v, t, LR)
        for k in th:
            np.testing.assert_allclose(nxt[k] - prev[k], -LR[k] * g[k] / (np.abs(g[k]) + 1e-8),
                                       rtol=1e-7, atol=1e-12)
        prev = nxt


def test_zero_gradient_and_inactive_are_noops():
    rng = np.random.default_rng(2)
    th, m, v = _state(rng)
    g0 = {k: np.zeros_like(x) for k, x in th.items()}
    th2, m2, v2, _ = adam_step(th, g0, m, v, 0, LR)
    for k in th:
        np.testing.assert_array_equal(th2[k], th[k])
    g = {k: rng.normal(size=x.shape) for k, x in th.items()}
    active = np.array([1, 0, 1, 0, 0, 1, 1], bool)
    th3, m3, v3, _ = adam_step(th, g, m, v, 0, LR, active=active)
    for k in th:
        np.testing.assert_array_equal(th3[k][~active], th[k][~active])
        np.testing.assert_array_equal(m3[k][~active], m[k][~active])
        assert np.all(th3[k][active] != th[k][active])


def test_matches_torch_adam():
    """Five steps against torch.optim.Adam (FP64, CPU) with random gradients."""
    rng = np.random.default_rng(3)
    th, m, v = _state(rng)
    params = {k: torch.tensor(x.copy(), dtype=torch.float64, requires_grad=True) for k, x in th.items()}
    opt = torch.optim.Adam([{"params": [params[k]], "lr": LR[k]} for k in th],
                           betas=(0.9, 0.999), eps=1e-8)
    t = 0
    for _ in range(5):
        g = {k: rng.normal(size=x.shape) for k, x in th.items()}
        th, m, v, t = adam_step(th, g, m, v, t, LR)
        for k in params:
            params[k].grad = torch.tensor(g[k])
        opt.step()
    for k in th:
        np.testing.assert_allclose(th[k], params[k].detach().numpy(), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("delta", [0.01, 0.1, 0.003])
def test_psnr_constant_error(delta):
    """P9: a constant error delta gives PSNR = -20 log10(delta)."""
    t = np.full((3, 5, 6), 0.4)
    assert psnr(t + delta, t) == pytest.approx(-20 * math.log10(delta), rel=1e-12)


def test_loss_gradient_is_derivative_of_mse():
    rng = np.random.default_rng(4)
    a, b = rng.uniform(size=(3, 4, 5)), rng.uniform(size=(3, 4, 5))
    g = dloss_dimg(a, b)
    e = np.zeros_like(a)
    e[1, 2, 3] = 1e-6
    assert (mse(a + e, b) - mse(a - e, b)) / 2e-6 == pytest.approx(g[1, 2, 3], rel=1e-6)
    assert psnr_from_mse(0.0) == math.inf


@pytest.mark.parametrize("wd", [0.0, 0.05])
def test_adamw_matches_torch_adamw(wd):
    """Decoupled decay: six steps against torch.optim.AdamW (FP64, CPU)."""
    from oracle.adam import adamw_step
    rng = np.random.default_rng(9)
    p = rng.normal(size=257)
    m = np.zeros(257)
    v = np.zeros(257)
    tp = torch.tensor(p.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.AdamW([tp], lr=3e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=wd)
    t = 0
    for _ in range(6):
        g = rng.normal(size=257)
        p, m, v, t = adamw_step(p, g, m, v, t, 3e-3, wd)
        tp.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_adamw_decay_is_not_in_the_moments():
    """With a zero gradient the moments stay zero and the parameters shrink
    by exactly (1 - lr wd): the decay bypasses the adaptive scaling (an L2
    term added to the gradient would instead move p by about lr per step)."""
    from oracle.adam import adamw_step
    p0 = np.array([2.0, -0.5, 1e-3])
    p, m, v, t = adamw_step(p0, np.zeros(3), np.zeros(3), np.zeros(3), 0, 0.1, 0.2)
    np.testing.assert_allclose(p, p0 * (1 - 0.1 * 0.2), rtol=1e-15)
    assert not m.any() and not v.any() and t == 1
