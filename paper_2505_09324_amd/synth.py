"""Seeded synthetic inputs shared by the GPU path and the CPU oracle.

This module generates *inputs only*: frames, ROI masks, raw random draws.
It contains none of the fitting method's arithmetic (no rendering, no
gradients, no optimiser, no sampling rule), so that the oracle and the HIP
path can both consume its arrays without sharing any of the method's code.

The frames stand in for the paper's 1080p talking-head video-conferencing
sequences (Sec. 4, dataset paragraph), which are not available: a smooth
linear-gradient background and one textured elliptical "subject" covering
about a quarter of the frame, optionally translating and rotating over time.

Every generator uses ``numpy.random.Generator(PCG64(seed))`` and draws in a
fixed order, so arrays are a pure function of (seed, shape, frame index).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Texture amplitude of the subject (fixed once; see the input recipe).
TEXTURE_AMPLITUDE = 0.08
# Subject semi-axes as fractions of the frame width / height.
SUBJECT_AX = 0.19
SUBJECT_AY = 0.42


@dataclass(frozen=True)
class SceneParams:
    """Random scene constants drawn once per sequence seed."""
    theta_bg: float
    c0: np.ndarray          # [3] background colour at t_min
    c1: np.ndarray          # [3] background colour at t_max
    cs: np.ndarray          # [3] subject base colour
    freqs: np.ndarray       # [3, 2] texture wave vectors (cycles/px)
    phases: np.ndarray      # [3, 3] phase per (wave j, channel k)


def scene_params(seed: int) -> SceneParams:
    rng = np.random.Generator(np.random.PCG64(seed))
    theta_bg = rng.uniform(0.0, 2.0 * math.pi)
    c0 = rng.uniform(0.0, 1.0, size=3)
    c1 = rng.uniform(0.0, 1.0, size=3)
    cs = rng.uniform(0.0, 1.0, size=3)
    mag = rng.uniform(1.0 / 48.0, 1.0 / 12.0, size=3)
    ang = rng.uniform(0.0, 2.0 * math.pi, size=3)
    phases = rng.uniform(0.0, 2.0 * math.pi, size=(3, 3))
    freqs = np.stack([mag * np.cos(ang), mag * np.sin(ang)], axis=1)
    return SceneParams(theta_bg, c0, c1, cs, freqs, phases)


def subject_pose(W: int, H: int, t: int | None):
    """Centre (x, y) and rotation (radians) of the subject at frame t.

    t=None is the static pose. With motion the centre moves +-40 px
    horizontally with period 60 frames and the subject rotates +-10 degrees
    with period 40 frames; the background never moves.
    """
    if t is None:
        return W / 2.0, H / 2.0, 0.0
    cx = W / 2.0 + 40.0 * math.sin(2.0 * math.pi * t / 60.0)
    th = math.radians(10.0) * math.sin(2.0 * math.pi * t / 40.0)
    return cx, H / 2.0, th


def make_frame(W: int, H: int, seed: int, t: int | None = None):
    """Return (frame [3,H,W] float32 in [0,1], roi_mask [H,W] bool)."""
    sp = scene_params(seed)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    px = xs + 0.5
    py = ys + 0.5
    # background: linear ramp along direction theta_bg, normalised over the
    # four frame corners
    ct, st = math.cos(sp.theta_bg), math.sin(sp.theta_bg)
    corners = np.array([[0, 0], [W, 0], [0, H], [W, H]], dtype=np.float64)
    proj = corners[:, 0] * ct + corners[:, 1] * st
    tmin, tmax = proj.min(), proj.max()
    tt = (px * ct + py * st - tmin) / (tmax - tmin)
    bg = sp.c0[:, None, None] + (sp.c1 - sp.c0)[:, None, None] * tt[None]
    # subject in its local frame
    cx, cy, th = subject_pose(W, H, t)
    a = SUBJECT_AX * W
    b = SUBJECT_AY * H
    dx = px - cx
    dy = py - cy
    cth, sth = math.cos(th), math.sin(th)
    u = cth * dx + sth * dy       # R(-theta) (p - centre)
    v = -sth * dx + cth * dy
    tex = np.zeros((3, H, W))
    for k in range(3):
        acc = np.zeros((H, W))
        for j in range(3):
            acc += np.sin(2.0 * math.pi * (sp.freqs[j, 0] * u + sp.freqs[j, 1] * v)
                          + sp.phases[j, k])
        tex[k] = np.clip(sp.cs[k] + TEXTURE_AMPLITUDE * acc, 0.0, 1.0)
    rho = np.sqrt((u / a) ** 2 + (v / b) ** 2)
    alpha = np.clip(0.5 - (rho - 1.0) * min(a, b) / 1.5, 0.0, 1.0)
    img = alpha[None] * tex + (1.0 - alpha[None]) * bg
    mask = rho <= 1.0
    return img.astype(np.float32), mask


def make_sequence(W: int, H: int, seed: int, n_frames: int):
    """Frames 0..n_frames-1 of a moving-subject sequence."""
    frames, masks = [], []
    for t in range(n_frames):
        f, m = make_frame(W, H, seed, t)
        frames.append(f)
        masks.append(m)
    return frames, masks


def random_gaussians(N: int, W: int, H: int, seed: int,
                     scale_lo: float = 0.5, scale_hi: float = 3.0):
    """Uniform random Gaussians (the tiny plain-method workload).

    mu ~ U[0,W) x U[0,H); l1, l3 ~ U[scale_lo, scale_hi]; l2 = 0;
    colour ~ U[0,1]^3.  Returns float32 arrays xy [N,2], chol [N,3], rgb [N,3].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    mx = rng.uniform(0.0, W, size=N)
    my = rng.uniform(0.0, H, size=N)
    l1 = rng.uniform(scale_lo, scale_hi, size=N)
    l3 = rng.uniform(scale_lo, scale_hi, size=N)
    rgb = rng.uniform(0.0, 1.0, size=(N, 3))
    xy = np.stack([mx, my], axis=1).astype(np.float32)
    chol = np.stack([l1, np.zeros(N), l3], axis=1).astype(np.float32)
    return xy, chol, rgb.astype(np.float32)


@dataclass(frozen=True)
class InitDraws:
    """Raw random draws consumed by the content-aware initialiser.

    ``pick_roi`` / ``pick_out`` are uniform integers in [0, 2^62) that the
    initialiser reduces modulo its own totals; ``jit_*`` are uniform jitters
    in [-0.5, 0.5) for the x and y coordinate of each drawn pixel.
    """
    pick_roi: np.ndarray     # [n_roi] int64
    jit_roi: np.ndarray      # [n_roi, 2] float32
    pick_out: np.ndarray     # [n_out] int64
    jit_out: np.ndarray      # [n_out, 2] float32


def init_draws(N: int, seed: int, roi_fraction: float = 0.7) -> InitDraws:
    n_roi = int(round(roi_fraction * N))
    n_out = N - n_roi
    rng = np.random.Generator(np.random.PCG64(seed))
    pick_roi = rng.integers(0, 1 << 62, size=n_roi, dtype=np.int64)
    jit_roi = (rng.random(size=(n_roi, 2)) - 0.5).astype(np.float32)
    pick_out = rng.integers(0, 1 << 62, size=n_out, dtype=np.int64)
    jit_out = (rng.random(size=(n_out, 2)) - 0.5).astype(np.float32)
    return InitDraws(pick_roi, jit_roi, pick_out, jit_out)


# Frame sizes and per-size Gaussian counts of the batched workload: counts are
# affine in area between 3000 (320x240) and 50000 (1920x1080).
BATCH_SIZES = [(320, 240), (640, 480), (1280, 720), (1920, 1080)]


def batch_gaussian_count(W: int, H: int) -> int:
    a0 = 320 * 240
    a1 = 1920 * 1080
    return int(round(3000 + 47000 * (W * H - a0) / (a1 - a0)))


def batch_sizes(n_frames: int, seed: int):
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = rng.integers(0, len(BATCH_SIZES), size=n_frames)
    return [BATCH_SIZES[i] for i in idx]


def random_normal(shape, seed: int, std: float = 1.0) -> np.ndarray:
    """Plain seeded normal draws (network weight init, perturbations)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.standard_normal(size=shape) * std).astype(np.float32)


def random_uniform(shape, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=shape).astype(np.float32)


def make_frame_torch(W: int, H: int, seed: int, t: int | None = None, device="cuda"):
    """The same synthetic frame as make_frame, evaluated in FP32 with torch on
    `device` (fast enough to stream training sequences).  Values agree with
    make_frame to FP32 rounding.  Returns (frame [3,H,W] float32,
    roi_mask [H,W] bool)."""
    import torch
    sp = scene_params(seed)
    ys = torch.arange(H, device=device, dtype=torch.float32)[:, None] + 0.5
    xs = torch.arange(W, device=device, dtype=torch.float32)[None, :] + 0.5
    ct, st = math.cos(sp.theta_bg), math.sin(sp.theta_bg)
    corners = [(0, 0), (W, 0), (0, H), (W, H)]
    proj = [cx * ct + cy * st for cx, cy in corners]
    tmin, tmax = min(proj), max(proj)
    tt = (xs * ct + ys * st - tmin) / (tmax - tmin)
    c0 = torch.tensor(sp.c0, device=device, dtype=torch.float32)[:, None, None]
    c1 = torch.tensor(sp.c1, device=device, dtype=torch.float32)[:, None, None]
    bg = c0 + (c1 - c0) * tt[None]
    cx, cy, th = subject_pose(W, H, t)
    a = SUBJECT_AX * W
    b = SUBJECT_AY * H
    dx = xs - cx
    dy = ys - cy
    cth, sth = math.cos(th), math.sin(th)
    u = cth * dx + sth * dy
    v = -sth * dx + cth * dy
    tex = []
    for k in range(3):
        acc = torch.zeros((H, W), device=device)
        for j in range(3):
            acc = acc + torch.sin(2.0 * math.pi * (float(sp.freqs[j, 0]) * u + float(sp.freqs[j, 1]) * v)
                                  + float(sp.phases[j, k]))
        tex.append(torch.clamp(float(sp.cs[k]) + TEXTURE_AMPLITUDE * acc, 0.0, 1.0))
    tex = torch.stack(tex)
    rho = torch.sqrt((u / a) ** 2 + (v / b) ** 2)
    alpha = torch.clamp(0.5 - (rho - 1.0) * min(a, b) / 1.5, 0.0, 1.0)
    img = alpha[None] * tex + (1.0 - alpha[None]) * bg
    return img.contiguous(), (rho <= 1.0)


# "Mouth" of the local-change sequences: an ellipse inside the static
# subject whose height oscillates, the only part of the frame that moves.
MOUTH_AX = 0.045          # semi-axis along x, fraction of W
MOUTH_AY = 0.012          # mean semi-axis along y, fraction of H
MOUTH_DY = 0.22           # centre below the subject centre, fraction of b
MOUTH_PERIOD = 9          # frames per open/close cycle


def make_talking_frame_torch(W: int, H: int, seed: int, t: int, device="cuda"):
    """A frame of a local-change sequence: the static scene of make_frame
    (pose t=None) with a dark elliptical "mouth" inside the subject whose
    height is MOUTH_AY H (1 + 0.9 sin(2 pi t / MOUTH_PERIOD)), edge
    antialiased over 1.5 px; everything else is identical in every frame
    (the mostly static content of a talking-head call).  FP32 on `device`.
    Returns (frame [3,H,W], roi_mask [H,W] bool)."""
    import torch
    img, mask = make_frame_torch(W, H, seed, None, device)
    sp = scene_params(seed)
    ys = torch.arange(H, device=device, dtype=torch.float32)[:, None] + 0.5
    xs = torch.arange(W, device=device, dtype=torch.float32)[None, :] + 0.5
    ma = MOUTH_AX * W
    mb = MOUTH_AY * H * (1.0 + 0.9 * math.sin(2.0 * math.pi * t / MOUTH_PERIOD))
    mx, my = W / 2.0, H / 2.0 + MOUTH_DY * SUBJECT_AY * H
    rho = torch.sqrt(((xs - mx) / ma) ** 2 + ((ys - my) / mb) ** 2)
    alpha = torch.clamp(0.5 - (rho - 1.0) * min(ma, mb) / 1.5, 0.0, 1.0)
    dark = torch.tensor(0.25 * sp.cs, device=device, dtype=torch.float32)[:, None, None]
    out = alpha[None] * dark + (1.0 - alpha[None]) * img
    return out.contiguous(), mask
