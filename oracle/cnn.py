"""FP64 oracle of the learned initialiser: a small convolutional regressor
that predicts, per 16x16 screen tile, how many Gaussians the tile holds and
their initial parameters.

The paper's alternative I-frame initialiser (Sec. 3.2.B) is a CNN regressor
trained with a Chamfer set loss because Gaussians have no consistent order
(the "unordered Gaussian correspondence problem").  Here the regressor is
made local: one prediction per tile, a count (9-way classification, 0..8)
plus 8 slots of 8 parameters, and the set loss is applied per tile, so the
correspondence problem is confined to at most 8 Gaussians.

Conventions (FP64; BF16 rounding of operands is applied explicitly where the
GPU computes with BF16 operands):
  - activations [C, H, W]; weights [Cout, Cin, 3, 3]; bias [Cout];
  - conv3x3 with padding 1 is a cross-correlation:
        y[o, i, j] = b[o] + sum_{c, u, v} w[o, c, u, v] x[c, s*i + u - 1, s*j + v - 1]
    (zero outside), output size ceil(H / s);
  - network: 4 x (conv stride 2, 64 channels, ReLU), then a stride-1 head
    conv to 73 channels = 9 count logits + 8 slots x 8 parameters;
  - slot parameters p (8): mu_x = x0 + T sigmoid(p0), mu_y = y0 + T sigmoid(p1),
    l1 = exp(p2), l2 = p3, l3 = exp(p4), colour = (p5, p6, p7);
  - in the loss a slot is the 8-vector (sigmoid(p0), sigmoid(p1), p2..p7) and a
    target Gaussian the vector ((mu_x - x0)/T, (mu_y - y0)/T, log|l1|, l2,
    log|l3|, c'_0, c'_1, c'_2);
  - per tile: CE(count logits, k) with k = number of target Gaussians (<= 8),
    and the symmetric squared-Euclidean Chamfer distance between the first k
    slots and the k targets,
        CD(P, Q) = mean_p min_q |p - q|^2 + mean_q min_p |q - p|^2,
    ties of the min resolved to the lowest index, 0 when k = 0;
  - loss = mean over tiles of CE + mean over tiles with k > 0 of CD.
"""
from __future__ import annotations

import math

import numpy as np

N_SLOTS = 8
N_PARAM = 8
HEAD_CH = 9 + N_SLOTS * N_PARAM  # 73


def bf16_round(x) -> np.ndarray:
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as
    FP32.  Input is converted to FP32 first."""
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((u >> 16) & 1)
    r = ((u + bias) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).reshape(a.shape)


def out_size(n: int, stride: int) -> int:
    return (n + 2 - 3) // stride + 1


def conv3x3(x, w, b, stride: int):
    """Cross-correlation with padding 1 (see module docstring)."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    C, H, W = x.shape
    Ho, Wo = out_size(H, stride), out_size(W, stride)
    xp = np.zeros((C, H + 2, W + 2))
    xp[:, 1:H + 1, 1:W + 1] = x
    y = np.zeros((w.shape[0], Ho, Wo)) + np.asarray(b, np.float64)[:, None, None]
    for u in range(3):
        for v in range(3):
            patch = xp[:, u:u + stride * (Ho - 1) + 1:stride, v:v + stride * (Wo - 1) + 1:stride]
            y += np.einsum("oc,chw->ohw", w[:, :, u, v], patch)
    return y


def conv3x3_backward(x, w, dy, stride: int):
    """Gradients of sum(dy * conv3x3(x, w, b, stride)) w.r.t. x, w and b."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    dy = np.asarray(dy, np.float64)
    C, H, W = x.shape
    Ho, Wo = dy.shape[1:]
    xp = np.zeros((C, H + 2, W + 2))
    xp[:, 1:H + 1, 1:W + 1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for u in range(3):
        for v in range(3):
            sl = (slice(None), slice(u, u + stride * (Ho - 1) + 1, stride),
                  slice(v, v + stride * (Wo - 1) + 1, stride))
            dw[:, :, u, v] = np.einsum("ohw,chw->oc", dy, xp[sl])
            dxp[sl] += np.einsum("oc,ohw->chw", w[:, :, u, v], dy)
    return dxp[:, 1:H + 1, 1:W + 1], dw, dy.sum(axis=(1, 2))


def forward(x, params, bf16=True):
    """Network forward.  params: list of (w, b) for the 5 layers.  With bf16,
    every layer input and weight is rounded to bfloat16 first (the GPU's
    operand precision; accumulation stays exact here).  Returns the head
    output [73, h, w] and the list of layer inputs (as used)."""
    acts = []
    h = np.asarray(x, np.float64)
    for i, (w, b) in enumerate(params):
        hin = bf16_round(h).astype(np.float64) if bf16 else h
        wq = bf16_round(w).astype(np.float64) if bf16 else np.asarray(w, np.float64)
        acts.append(hin)
        stride = 2 if i < len(params) - 1 else 1
        h = conv3x3(hin, wq, b, stride)
        if i < len(params) - 1:
            h = np.maximum(h, 0.0)
    return h, acts


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def slot_vectors(head_tile):
    """head_tile [73] -> (logits [9], slot vectors [8, 8] in loss units)."""
    logits = head_tile[:9]
    p = head_tile[9:].reshape(N_SLOTS, N_PARAM).copy()
    p[:, 0] = sigmoid(p[:, 0])
    p[:, 1] = sigmoid(p[:, 1])
    return logits, p


def chamfer(P, Q):
    """Symmetric squared-Euclidean Chamfer distance and its gradient w.r.t. P."""
    P = np.asarray(P, np.float64)
    Q = np.asarray(Q, np.float64)
    k = P.shape[0]
    if k == 0:
        return 0.0, np.zeros_like(P)
    d = ((P[:, None, :] - Q[None, :, :]) ** 2).sum(-1)
    jq = d.argmin(axis=1)       # nearest target of each prediction (first on ties)
    ip = d.argmin(axis=0)       # nearest prediction of each target
    val = d[np.arange(k), jq].mean() + d[ip, np.arange(Q.shape[0])].mean()
    g = np.zeros_like(P)
    g += 2.0 * (P - Q[jq]) / k
    np.add.at(g, ip, 2.0 * (P[ip] - Q) / Q.shape[0])
    return float(val), g


def cross_entropy(logits, k):
    z = np.asarray(logits, np.float64)
    m = z.max()
    lse = m + math.log(np.exp(z - m).sum())
    p = np.exp(z - lse)
    g = p.copy()
    g[k] -= 1.0
    return float(lse - z[k]), g


def head_loss(head, targets):
    """head [73, TY, TX]; targets: dict tile_index -> array [k, 8] (k <= 8)
    in loss units.  Returns (loss, dloss/dhead)."""
    _, TY, TX = head.shape
    n_tiles = TY * TX
    g = np.zeros_like(head, dtype=np.float64)
    ce_sum = 0.0
    cd_sum = 0.0
    n_cd = sum(1 for t in range(n_tiles) if len(targets.get(t, ())) > 0)
    for t in range(n_tiles):
        ty, tx = divmod(t, TX)
        Q = np.asarray(targets.get(t, np.zeros((0, N_PARAM))), np.float64)
        k = Q.shape[0]
        logits, P = slot_vectors(head[:, ty, tx])
        ce, gl = cross_entropy(logits, k)
        ce_sum += ce
        g[:9, ty, tx] += gl / n_tiles
        if k > 0:
            cd, gp = chamfer(P[:k], Q)
            cd_sum += cd
            raw = head[9:, ty, tx].reshape(N_SLOTS, N_PARAM)
            gp_full = np.zeros((N_SLOTS, N_PARAM))
            gp_full[:k] = gp / n_cd
            for c in (0, 1):
                s = sigmoid(raw[:, c])
                gp_full[:, c] *= s * (1.0 - s)
            g[9:, ty, tx] += gp_full.ravel()
    loss = ce_sum / n_tiles + (cd_sum / n_cd if n_cd else 0.0)
    return loss, g


def backward(x, params, head_grad, bf16=True):
    """Gradients of the network w.r.t. its parameters given dloss/dhead,
    through the same BF16-rounded operands the forward used."""
    _, acts = forward(x, params, bf16)
    # recompute pre-activation outputs for the ReLU masks
    outs = []
    for i, (w, b) in enumerate(params):
        wq = bf16_round(w).astype(np.float64) if bf16 else np.asarray(w, np.float64)
        stride = 2 if i < len(params) - 1 else 1
        outs.append(conv3x3(acts[i], wq, b, stride))
    grads = [None] * len(params)
    dy = np.asarray(head_grad, np.float64)
    for i in range(len(params) - 1, -1, -1):
        w, _ = params[i]
        wq = bf16_round(w).astype(np.float64) if bf16 else np.asarray(w, np.float64)
        stride = 2 if i < len(params) - 1 else 1
        if i < len(params) - 1:
            dy = dy * (outs[i] > 0)
        dx, dw, db = conv3x3_backward(acts[i], wq, dy, stride)
        grads[i] = (dw, db)
        dy = dx
    return grads


def tile_targets(xy, chol, rgb, W, H, T=16):
    """Per-tile target sets from fitted Gaussians: those whose centre lies in
    the tile; if more than 8, the 8 with the largest |l1 l3| |c'|^2 (ties to
    the lower index), listed by increasing index."""
    xy = np.asarray(xy, np.float64)
    chol = np.asarray(chol, np.float64)
    rgb = np.asarray(rgb, np.float64)
    TX = (W + T - 1) // T
    TY = (H + T - 1) // T
    out = {}
    tx = np.floor(xy[:, 0] / T).astype(np.int64)
    ty = np.floor(xy[:, 1] / T).astype(np.int64)
    ok = (tx >= 0) & (tx < TX) & (ty >= 0) & (ty < TY) & np.all(np.isfinite(chol), 1)
    ok &= (np.abs(chol[:, 0]) > 0) & (np.abs(chol[:, 2]) > 0)
    # mass |l1 l3| * |c'|^2 evaluated in FP32 in a fixed order: the ranking
    # is a decision both implementations must take identically
    f = np.float32
    c32 = np.asarray(rgb, f)
    l32 = np.asarray(chol, f)
    mass = np.abs(l32[:, 0] * l32[:, 2]) * ((c32[:, 0] * c32[:, 0] + c32[:, 1] * c32[:, 1])
                                            + c32[:, 2] * c32[:, 2])
    for n in np.nonzero(ok)[0]:
        out.setdefault(int(ty[n] * TX + tx[n]), []).append(int(n))
    res = {}
    for t, ids in out.items():
        ids = sorted(ids, key=lambda n: (-mass[n], n))[:N_SLOTS]
        ids = sorted(ids)
        tyy, txx = divmod(t, TX)
        v = np.zeros((len(ids), N_PARAM))
        for r, n in enumerate(ids):
            v[r] = ((xy[n, 0] - txx * T) / T, (xy[n, 1] - tyy * T) / T, math.log(abs(chol[n, 0])),
                    chol[n, 1], math.log(abs(chol[n, 2])), *rgb[n])
        res[t] = v
    return res


def decode_slot(q, tx, ty, T=16):
    """Gaussian (mu_x, mu_y, l1, l2, l3, c0, c1, c2) of the slot parameters
    q [8] of tile (tx, ty)."""
    return (tx * T + T * sigmoid(q[0]), ty * T + T * sigmoid(q[1]),
            math.exp(min(max(q[2], -4.0), 4.0)), q[3], math.exp(min(max(q[4], -4.0), 4.0)),
            q[5], q[6], q[7])


def decode(head, N, plain, T=16):
    """Predicted Gaussians from the head output [73, TY, TX]: per tile
    k = argmax of the count logits (first maximum) and slots 0..k-1, in tile
    order; kept up to N, topped up with the plain initialisation `plain`
    (xy, chol, rgb) to N.  Falls back to the plain initialisation when fewer
    than N/2 Gaussians are predicted or any is not finite.  Returns
    (xy, chol, rgb, n_predicted_used)."""
    head = np.asarray(head, np.float64)
    _, TY, TX = head.shape
    out = []
    for t in range(TY * TX):
        ty, tx = divmod(t, TX)
        z = head[:9, ty, tx]
        k = int(np.argmax(z))
        p = head[9:, ty, tx].reshape(N_SLOTS, N_PARAM)
        for s in range(k):
            out.append(decode_slot(p[s], tx, ty, T))
    out = np.array(out, np.float64).reshape(-1, 8)
    pxy, pch, prgb = (np.asarray(a, np.float64) for a in plain)
    npred = min(len(out), N)
    if not np.all(np.isfinite(out)) or 2 * npred < N:
        return pxy[:N].copy(), pch[:N].copy(), prgb[:N].copy(), 0
    xy = np.concatenate([out[:npred, 0:2], pxy[:N - npred]])
    chol = np.concatenate([out[:npred, 2:5], pch[:N - npred]])
    rgb = np.concatenate([out[:npred, 5:8], prgb[:N - npred]])
    return xy, chol, rgb, npred


def tile_residual_energy(frame, prev, T=16):
    """Mean squared residual of every T x T tile [TY, TX], specified in FP32
    because it decides which tiles a P-frame re-initialises: per pixel
    e = (dr*dr + dg*dg) + db*db with d = frame - prev, each operation
    rounded once; a tile's sum adds its in-frame pixels one at a time in
    row-major order starting from 0, and is divided by their count."""
    f = np.asarray(frame, np.float32)
    p = np.asarray(prev, np.float32)
    d = f - p
    e = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
    _, H, W = f.shape
    TX, TY = (W + T - 1) // T, (H + T - 1) // T
    ep = np.zeros((TY * T, TX * T), np.float32)     # out-of-frame pixels add +0 exactly
    ep[:H, :W] = e
    acc = np.zeros((TY, TX), np.float32)
    for ry in range(T):
        for rx in range(T):
            acc = acc + ep[ry::T, rx::T]
    ys = np.minimum(T, H - np.arange(TY) * T)
    xs = np.minimum(T, W - np.arange(TX) * T)
    cnt = (ys[:, None] * xs[None, :]).astype(np.float32)
    return acc / cnt


def pframe_replace(frame, prev, head, xy, chol, rgb, tau, T=16):
    """Learned re-initialisation of a warm-started P-frame (Sec. 3.2.B used
    at P-frames, Sec. 3.2.C): tiles whose mean squared residual against the
    previous frame exceeds tau (FP32, strictly) are re-initialised.  The
    warm-started Gaussians centred in such a tile (floor(mu / T) in FP32)
    are freed, in increasing index order; the selected tiles' decoded
    predictions (argmax count, slots 0..k-1; tiles in raster order) fill the
    freed slots in that order.  Freed slots left over keep their Gaussians,
    predictions left over are dropped, so N is unchanged; if any raw slot
    parameter of a used prediction is not finite nothing is replaced.
    Returns (xy, chol, rgb) in FP64 and a dict of the integer decisions."""
    sel = tile_residual_energy(frame, prev, T) > np.float32(tau)
    TY, TX = sel.shape
    head = np.asarray(head, np.float64)
    xy64 = np.array(xy, np.float64)
    chol64 = np.array(chol, np.float64)
    rgb64 = np.array(rgb, np.float64)
    x32 = np.asarray(xy, np.float32)
    with np.errstate(invalid="ignore"):
        gx = np.floor(x32[:, 0] / np.float32(T))
        gy = np.floor(x32[:, 1] / np.float32(T))
        inside = (gx >= 0) & (gx < TX) & (gy >= 0) & (gy < TY)
    freed = [n for n in np.nonzero(inside)[0] if sel[int(gy[n]), int(gx[n])]]
    preds, raw_ok = [], True
    for t in range(TY * TX):
        ty, tx = divmod(t, TX)
        if not sel[ty, tx]:
            continue
        k = int(np.argmax(head[:9, ty, tx]))
        p = head[9:, ty, tx].reshape(N_SLOTS, N_PARAM)
        for s in range(k):
            raw_ok = raw_ok and bool(np.all(np.isfinite(p[s])))
            preds.append(decode_slot(p[s], tx, ty, T))
    m = min(len(freed), len(preds)) if raw_ok else 0
    for i in range(m):
        n = freed[i]
        q = preds[i]
        xy64[n] = q[0:2]
        chol64[n] = q[2:5]
        rgb64[n] = q[5:8]
    info = {"selected": sel, "freed": np.array(freed, np.int64), "n_predicted": len(preds),
            "replaced": m}
    return xy64, chol64, rgb64, info
