"""Drivers for the fitting workloads, on top of the C ABI.

Each driver only sequences library calls (initialise, fit, time); every step
of the fit runs in the HIP library.

    python -m paper_2505_09324_amd.workloads batch   # 48 uneven frames, one launch per stage
    python -m paper_2505_09324_amd.workloads video   # warm-started sequence
    python -m paper_2505_09324_amd.workloads pframe [--sequence motion|local] [--tau 0.02]
    python -m paper_2505_09324_amd.workloads compress   # PTQ, QAT, Eq. 3-4 bit count
    python -m paper_2505_09324_amd.workloads superpixel # superpixel vs content-aware ROI init
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import _lib, autotune, synth

LR_DEFAULT = (2e-2, 5e-3, 5e-3)   # mean, Cholesky vector, colour


def _dev(a, device):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def plain_init(frame, mask, N, seed, device="cuda"):
    """Content-aware ROI init (70 % in the ROI) on the GPU."""
    d = synth.init_draws(N, seed=seed)
    return _lib.init_plain(_dev(frame, device), _dev(mask.astype(np.uint8), device),
                           _dev(d.pick_roi, device), _dev(d.jit_roi, device),
                           _dev(d.pick_out, device), _dev(d.jit_out, device))


def psnr(mse):
    return float("inf") if mse <= 0 else 10.0 * np.log10(1.0 / mse)


# ------------------------------------------------------------------ batch --
def batch_inputs(n_frames=48, seed=400, device="cuda"):
    """Frames of sizes drawn uniformly from 320x240 .. 1920x1080, Gaussian
    counts affine in area (3k..50k), content-aware init per frame.
    Returns (sizes, targets, xy, chol, rgb, frames_np) with concatenated
    device tensors."""
    dims = synth.batch_sizes(n_frames, seed)
    sizes, frames, parts = [], [], []
    for i, (w, h) in enumerate(dims):
        n = synth.batch_gaussian_count(w, h)
        f, m = synth.make_frame(w, h, seed=4000 + i)
        sizes.append((w, h, n))
        frames.append(f)
        parts.append(plain_init(f, m, n, 4100 + i, device))
    targets = _dev(np.concatenate([f.ravel() for f in frames]), device)
    xy = torch.cat([p[0] for p in parts]).contiguous()
    chol = torch.cat([p[1] for p in parts]).contiguous()
    rgb = torch.cat([p[2] for p in parts]).contiguous()
    return sizes, targets, xy, chol, rgb, frames


def autotuned(sizes, targets, xy, chol, rgb, reps=3, cache_path=None):
    """(tile, px_per_lane) for the batch and the candidates' ms per round;
    with cache_path None every candidate is timed (the workload reports the
    timings)."""
    cfg, ms, _ = autotune.tuned_batch_config(sizes, targets, xy, chol, rgb, reps=reps,
                                             cache_path=cache_path)
    return cfg, ms


def run_batch(n_frames=48, iters=300, seed=400, check_every=50, device="cuda", lr=LR_DEFAULT):
    """Aggregate iterations/s of the batched fit vs the same frames fitted
    one by one (each with its own graph-replayed fit_frame)."""
    sizes, targets, xy, chol, rgb, _ = batch_inputs(n_frames, seed, device)
    (T, ppl), tune_ms = autotuned(sizes, targets, xy, chol, rgb)
    Nt = sum(n for _, _, n in sizes)
    cfg = _lib.adam_cfg(lr)
    # batched
    ws = torch.empty(_lib.batch_workspace_bytes(sizes, T, ppl), dtype=torch.uint8, device=device)
    bx, bc, br = xy.clone(), chol.clone(), rgb.clone()
    m = torch.zeros(8 * Nt, device=device)
    v = torch.zeros(8 * Nt, device=device)
    step = torch.zeros(1, dtype=torch.int32, device=device)
    trace = torch.zeros((iters + 8, n_frames), device=device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = _lib.fit_batch(sizes, T, ppl, targets, bx, bc, br, m, v, step, trace, ws,
                        _lib.fit_opts(iters, check_every, cfg=cfg))
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    final_b = trace[iters - 1].cpu().numpy()
    # one by one
    t_seq = 0.0
    final_s = []
    off = poff = 0
    for w, h, n in sizes:
        shape = _lib.make_shape(w, h, n, T, px_per_lane=ppl)
        wsf = _lib.alloc_workspace(shape)
        px, pc, pr = (t[off:off + n].clone() for t in (xy, chol, rgb))
        tgt = targets[poff:poff + 3 * w * h].view(3, h, w)
        mf = torch.zeros(8 * n, device=device)
        vf = torch.zeros(8 * n, device=device)
        sf = torch.zeros(1, dtype=torch.int32, device=device)
        tf = torch.zeros(iters + 8, device=device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _lib.fit_frame(shape, tgt, px, pc, pr, mf, vf, sf, tf, wsf,
                       _lib.fit_opts(iters, check_every, cfg=cfg))
        torch.cuda.synchronize()
        t_seq += time.perf_counter() - t0
        final_s.append(float(tf[iters - 1]))
        off += n
        poff += 3 * w * h
    pairs_note = {f"{w}x{h}": sum(1 for s in sizes if s[:2] == (w, h)) for w, h in synth.BATCH_SIZES}
    return {
        "workload": f"{n_frames} frames, sizes {pairs_note}, {Nt} Gaussians, {iters} iterations each",
        "tile": T, "px_per_lane": ppl, "autotune_ms_per_round": tune_ms,
        "batched_iters_per_s": round(n_frames * iters / t_batch, 1),
        "sequential_iters_per_s": round(n_frames * iters / t_seq, 1),
        "speedup": round(t_seq / t_batch, 3),
        "batched_seconds": round(t_batch, 3), "sequential_seconds": round(t_seq, 3),
        "mean_final_psnr_batched": round(float(np.mean([psnr(x) for x in final_b])), 3),
        "mean_final_psnr_sequential": round(float(np.mean([psnr(x) for x in final_s])), 3),
        "batched_tile_list_rebuilds": int(st.rebins),
        "status": int(st.status),
    }


# ------------------------------------------------------------------ video --
def fit_sequence(frames, masks, N, iters_first, iters_rest, init_seed, tile=32, ppl=2,
                 lr=LR_DEFAULT, psnr_target=0.0, check_every=None, device="cuda",
                 warm_start=True, init_fn=None):
    """Fit a sequence frame by frame.  Frame 0 starts from `init_fn` (default
    the content-aware init); with warm_start each later frame starts from the
    previous frame's fitted Gaussians with the Adam state reset, otherwise
    from its own init.  Tile 32 / 2 px per lane is what the autotuner picks
    at 1080p; without a PSNR target the loss is read back every 50
    iterations, with one every 10.  Returns per-frame records."""
    if check_every is None:
        check_every = 10 if psnr_target > 0 else 50
    H, W = frames[0].shape[1:]
    shape = _lib.make_shape(W, H, N, tile, px_per_lane=ppl)
    ws = _lib.alloc_workspace(shape, device)
    cfg = _lib.adam_cfg(lr)
    init_fn = init_fn or (lambda t, f, m: plain_init(f, m, N, init_seed + t, device))
    recs = []
    params = None
    for t, (f, m) in enumerate(zip(frames, masks)):
        T = _dev(f, device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if params is None or not warm_start:
            params = [p.contiguous() for p in init_fn(t, f, m)]
            iters = iters_first
        else:
            iters = iters_rest
        mm = torch.zeros(8 * N, device=device)
        vv = torch.zeros(8 * N, device=device)
        step = torch.zeros(1, dtype=torch.int32, device=device)
        trace = torch.zeros(iters + 8, device=device)
        st = _lib.fit_frame(shape, T, *params, mm, vv, step, trace, ws,
                            _lib.fit_opts(iters, check_every, psnr_target, cfg=cfg))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tr = trace[:st.iters_run].cpu().numpy()
        recs.append({"frame": t, "iters": int(st.iters_run), "seconds": dt,
                     "psnr_first": psnr(float(tr[0])), "psnr_last": psnr(float(tr[-1])),
                     "hit": int(st.iter_hit_target)})
    return recs, params


def run_video(n_frames=60, W=1920, H=1080, N=30000, iters_first=2000, iters_rest=200, seed=301,
              device="cuda"):
    frames, masks = synth.make_sequence(W, H, seed, n_frames)
    recs, _ = fit_sequence(frames, masks, N, iters_first, iters_rest, init_seed=seed + 1,
                           device=device)
    rest = recs[1:]
    return {
        "workload": f"{n_frames} frames {W}x{H}, {N} Gaussians, frame 0 {iters_first} iterations "
                    f"from the content-aware init, later frames {iters_rest} warm-started",
        "frame0_seconds": round(recs[0]["seconds"], 3), "frame0_psnr": round(recs[0]["psnr_last"], 3),
        "warm_mean_seconds": round(float(np.mean([r["seconds"] for r in rest])), 4) if rest else None,
        "warm_mean_psnr_start": round(float(np.mean([r["psnr_first"] for r in rest])), 3) if rest else None,
        "warm_mean_psnr_end": round(float(np.mean([r["psnr_last"] for r in rest])), 3) if rest else None,
        "per_frame": recs,
    }


# ------------------------------------------- P-frame selective optimisation --
def run_pframe(n_frames=30, W=1920, H=1080, N=30000, tau=0.02, psnr_target=35.0, cap=2000,
               iters_first=2000, seed=301, sequence="motion", device="cuda", lr=LR_DEFAULT):
    """P-frames fitted two ways from the same fitted I-frame (Sec. 3.2.C):
    a full refit (every Gaussian warm-started and optimised) and the
    selective optimisation (only the reference Gaussians influencing a pixel
    whose change since the previous source frame exceeds tau).  Each arm
    chains its own fitted frames.  Per P-frame the clock runs from the frame
    being resident to the first PSNR check >= psnr_target (every 10
    iterations), including the binning and selection.  sequence="motion":
    the moving subject (+-40 px, +-10 degrees); "local": a static subject
    whose mouth region alone changes."""
    make = ((lambda t: synth.make_frame_torch(W, H, seed, t, device)) if sequence == "motion"
            else (lambda t: synth.make_talking_frame_torch(W, H, seed, t, device)))
    frames = [make(t)[0] for t in range(n_frames)]
    f0, m0 = make(0)
    shape = _lib.make_shape(W, H, N, 32, px_per_lane=2)
    ws = _lib.alloc_workspace(shape, device)
    cfg = _lib.adam_cfg(lr)
    theta0 = [p.contiguous() for p in plain_init_dev(f0, m0, N, seed + 1)]
    m = torch.zeros(8 * N, device=device)
    v = torch.zeros(8 * N, device=device)
    step = torch.zeros(1, dtype=torch.int32, device=device)
    trace = torch.zeros(max(iters_first, cap) + 16, device=device)
    _lib.fit_frame(shape, frames[0], *theta0, m, v, step, trace, ws,
                   _lib.fit_opts(iters_first, 50, cfg=cfg))
    psnr0 = psnr(float(trace[iters_first - 1]))
    counts = torch.zeros(2, dtype=torch.int32, device=device)
    active = torch.zeros(N, dtype=torch.uint8, device=device)
    out = {"workload": f"{sequence} sequence, {n_frames} frames {W}x{H}, {N} Gaussians; I-frame "
                       f"{iters_first} iterations ({psnr0:.2f} dB); P-frames to {psnr_target} dB "
                       f"(cap {cap}), tau {tau}", "iframe_psnr": round(psnr0, 3)}
    for arm in ("full", "selective"):
        theta = [p.clone() for p in theta0]
        recs = []
        for t in range(1, n_frames):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sel = None
            if arm == "selective":
                _lib.project_bin(shape, theta[0], theta[1], ws)
                _lib.select_changed(shape, ws, theta[0], theta[1], frames[t], frames[t - 1], tau,
                                    active=active, counts=counts)
                sel = active
            m.zero_(), v.zero_(), step.zero_()
            st = _lib.fit_frame(shape, frames[t], *theta, m, v, step, trace, ws,
                                _lib.fit_opts(cap, 10, psnr_target, cfg=cfg, active=sel))
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            c = counts.cpu().numpy() if arm == "selective" else (None, N)
            recs.append({"frame": t, "seconds": dt, "iters": int(st.iters_run),
                         "hit": int(st.iter_hit_target), "psnr_start": psnr(float(trace[0])),
                         "psnr_end": float(st.final_psnr), "selected": int(c[1]),
                         "changed_px": None if c[0] is None else int(c[0])})
        hits = [r for r in recs if r["hit"] >= 0]
        out[arm] = {
            "mean_seconds": round(float(np.mean([r["seconds"] for r in recs])), 5),
            "mean_iters": round(float(np.mean([r["iters"] for r in recs])), 2),
            "frames_reaching_target": len(hits),
            "mean_fraction_selected": round(float(np.mean([r["selected"] for r in recs])) / N, 4),
            "mean_psnr_start": round(float(np.mean([r["psnr_start"] for r in recs])), 3),
            "per_frame": recs,
        }
    out["selective_over_full_seconds"] = round(out["selective"]["mean_seconds"]
                                               / out["full"]["mean_seconds"], 3)
    return out


# ------------------------------------------------ superpixel initialisation --
def run_superpixel(n_frames=3, W=1920, H=1080, N=30000, psnr_target=35.0, cap=3000, sp_iters=10,
                   compactness=0.1, sweep=(0.03, 0.3), seed=201, device="cuda", lr=LR_DEFAULT):
    """Initialisations of Sec. 3.2.A and Table 1 on the same frames: random
    (uniform positions, scales in [0.5, 3], uniform colours: the
    initialisation of the image codec the paper starts from), the
    content-aware draws alone, and the superpixel segmentation seeded by the
    same ROI draws (one Gaussian per K-means segment; the Gaussians outside
    the ROI are shared).  Per frame and arm: initialisation time, PSNR of
    the initial render, PSNR after 50/100/200/500/1000 iterations, and
    iterations and seconds (initialisation + fit) to psnr_target, checked
    every 10 iterations.  The compactness sweep runs on the first frame."""
    shape = _lib.make_shape(W, H, N, 32, px_per_lane=2)
    ws = _lib.alloc_workspace(shape, device)
    cfg = _lib.adam_cfg(lr)
    points = (50, 100, 200, 500, 1000)
    out = {"workload": f"{n_frames} frames {W}x{H}, {N} Gaussians (70 % in the ROI); superpixel "
                       f"{sp_iters} rounds, m {compactness}; fit to {psnr_target} dB (cap {cap})",
           "frames": []}

    def init(frame, mask, d, m_sp, rseed=0):
        n_roi = d.pick_roi.shape[0]
        picked = torch.empty(N, dtype=torch.int32, device=device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if m_sp == "random":
            xy, chol, rgb = (_dev(a, device) for a in synth.random_gaussians(N, W, H, rseed))
            torch.cuda.synchronize()
            return (xy, chol, rgb), time.perf_counter() - t0
        xy, chol, rgb = _lib.init_plain(frame, mask, _dev(d.pick_roi, device),
                                        _dev(d.jit_roi, device), _dev(d.pick_out, device),
                                        _dev(d.jit_out, device), picked=picked)
        if m_sp is not None:
            _lib.init_superpixel(frame, mask, picked[:n_roi], xy[:n_roi], chol[:n_roi],
                                 rgb[:n_roi], iters=sp_iters, compactness=m_sp)
        torch.cuda.synchronize()
        return (xy, chol, rgb), time.perf_counter() - t0

    def arm(frame, mask, d, m_sp, rseed=0):
        params, t_init = init(frame, mask, d, m_sp, rseed)
        rec = {"init_ms": round(t_init * 1e3, 3),
               "psnr_init": round(frame_psnr(shape, ws, frame, *params), 3)}
        curve = psnr_curve(shape, ws, frame, params, max(points), points, cfg)
        rec["psnr_at"] = {k: round(v, 3) for k, v in curve.items()}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hit, ran = fit_to_target(shape, ws, frame, params, psnr_target, cap, 10, cfg)
        torch.cuda.synchronize()
        rec["iters_to_target"] = hit
        rec["seconds_to_target"] = (round(t_init + time.perf_counter() - t0, 4)
                                    if hit is not None else None)
        return rec

    for f in range(n_frames):
        frame, mask = synth.make_frame_torch(W, H, seed + 2 * f, None, device)
        mask = mask.to(torch.uint8).contiguous()
        d = synth.init_draws(N, seed=seed + 2 * f + 1)
        if f == 0:                      # untimed warm-up of every initialiser
            for m_sp in ("random", None, compactness):
                init(frame, mask, d, m_sp)
        rec = {"frame_seed": seed + 2 * f, "random": arm(frame, mask, d, "random", seed + 2 * f + 1),
               "content_aware": arm(frame, mask, d, None),
               "superpixel": arm(frame, mask, d, compactness)}
        if f == 0:
            rec["sweep"] = {str(m): arm(frame, mask, d, m) for m in sweep}
        out["frames"].append(rec)
    for name in ("random", "content_aware", "superpixel"):
        recs = [r[name] for r in out["frames"]]
        hits = [r["iters_to_target"] for r in recs if r["iters_to_target"] is not None]
        out[name] = {"mean_init_ms": round(float(np.mean([r["init_ms"] for r in recs])), 3),
                     "mean_psnr_init": round(float(np.mean([r["psnr_init"] for r in recs])), 3),
                     "mean_iters_to_target": round(float(np.mean(hits)), 1) if hits else None,
                     "frames_reaching_target": len(hits)}
    return out


# ------------------------------------------------------------- compression --
def frame_psnr(shape, ws, target, xy, chol, rgb):
    """PSNR of the render of (xy, chol, rgb) against target (library calls)."""
    _lib.project_bin(shape, xy, chol, ws)
    loss = torch.zeros((), device=target.device)
    _lib.render_fwd(shape, ws, rgb, target=target, loss=loss)
    return psnr(float(loss))


def run_compress(W=1920, H=1080, N=30000, iters=1000, seed=201,
                 bit_pairs=((4, 4), (6, 6), (8, 8), (10, 10)), qat_bits=(6, 6), frames=60, gop=10,
                 device="cuda", lr=LR_DEFAULT):
    """Sec. 3.3: post-training quantisation of a fitted 1080p frame at several
    bit depths (PSNR after quantisation, entropy-coded bits, bpp, latency),
    quantisation-aware fitting against fitting + PTQ for the same iterations
    (time and PSNR after quantisation, the comparison of Table 3), and the
    sequence bit count of Eq. 3-4 for `frames` frames with an I-frame every
    `gop`, N/20 Gaussians per P-frame as in the paper."""
    import math
    f, m = synth.make_frame_torch(W, H, seed, None, device)
    shape = _lib.make_shape(W, H, N, 32, px_per_lane=2)
    ws = _lib.alloc_workspace(shape, device)
    cfg = _lib.adam_cfg(lr)
    theta0 = [p.contiguous() for p in plain_init_dev(f, m, N, seed + 1)]
    ctx = _lib.Context()

    def fit(qat, qat_iters=None):
        """Fit from theta0; with qat, the last qat_iters iterations (all when
        None) are quantisation-aware, the Adam state carried across."""
        th = [p.clone() for p in theta0]
        mm = torch.zeros(8 * N, device=device)
        vv = torch.zeros(8 * N, device=device)
        step = torch.zeros(1, dtype=torch.int32, device=device)
        trace = torch.zeros(iters + 8, device=device)
        k_q = 0 if qat is None else (iters if qat_iters is None else qat_iters)
        parts = [o for o in (_lib.fit_opts(iters - k_q, 50, cfg=cfg) if iters > k_q else None,
                             _lib.fit_opts(k_q, 50, cfg=cfg, qat=qat) if k_q else None) if o]
        for o in parts:
            _lib.fit_prepare(shape, f, *th, mm, vv, step, trace, ws, o, ctx=ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for o in parts:
            _lib.fit_frame(shape, f, *th, mm, vv, step, trace, ws, o, ctx=ctx)
        torch.cuda.synchronize()
        return th, time.perf_counter() - t0

    fit(None)                                   # warm: graphs, clocks
    theta, t_plain = fit(None)
    out = {"workload": f"{W}x{H}, {N} Gaussians fitted {iters} iterations from the content-aware "
                       f"init", "fit_psnr": round(frame_psnr(shape, ws, f, *theta), 3),
           "fit_seconds": round(t_plain, 4), "ptq": []}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for bc, br in bit_pairs:
        q = _lib.ptq(*theta, bc, br)
        e0.record()
        for _ in range(20):
            q = _lib.ptq(*theta, bc, br)
        e1.record()
        torch.cuda.synchronize()
        bits = q["bits"].cpu().numpy()
        out["ptq"].append({"bits_chol": bc, "bits_rgb": br,
                           "psnr": round(frame_psnr(shape, ws, f, q["xy"], q["chol"], q["rgb"]), 3),
                           "bits": round(float(bits[6])), "bits_per_gaussian": round(float(bits[6]) / N, 3),
                           "bpp": round(float(bits[6]) / (W * H), 5),
                           "latency_ms": round(e0.elapsed_time(e1) / 20, 4)})
    qp = _lib.ptq(*theta, *qat_bits)
    out["qat"] = {"bits": list(qat_bits),
                  "ptq_psnr_after_quantisation": round(frame_psnr(shape, ws, f, qp["xy"], qp["chol"], qp["rgb"]), 3)}
    for name, k_q in (("whole_fit", None), ("last_20pct", iters // 5)):
        fit(qat_bits, k_q)                      # warm the quantisation-aware graphs
        theta_q, t_qat = fit(qat_bits, k_q)
        qq = _lib.ptq(*theta_q, *qat_bits)
        out["qat"][name] = {
            "seconds": round(t_qat, 4),
            "psnr_after_quantisation": round(frame_psnr(shape, ws, f, qq["xy"], qq["chol"], qq["rgb"]), 3),
            "fp32_psnr": round(frame_psnr(shape, ws, f, *theta_q), 3),
            "overhead_seconds_per_1000_iterations": round((t_qat - t_plain) * 1000 / iters, 4)}
    # Eq. 3-4 for a sequence, the frame's quantised size standing for every frame
    i_bits = float(qp["bits"][6].item())
    n_p = N / 20
    p_bits = n_p * i_bits / N
    n_i = math.ceil(frames / gop)
    s_p = (math.lgamma(n_p + 1) - math.log(n_p)) / math.log(2)
    s_total = (frames - frames / gop) * s_p
    total = n_i * i_bits + (frames - n_i) * p_bits - s_total
    out["sequence"] = {"frames": frames, "gop": gop, "gaussians_per_p_frame": n_p,
                       "i_frame_bits": round(i_bits), "p_frame_bits": round(p_bits),
                       "bitsback_saving_per_p_frame": round(s_p, 1), "total_bits": round(total),
                       "bpp": round(total / (frames * W * H), 5),
                       "bpp_all_i_frames": round(i_bits / (W * H), 5)}
    return out


# ------------------------------------------------------ learned initialiser --
def plain_init_dev(frame, mask, N, seed):
    """Content-aware init from device tensors (frame [3,H,W], mask [H,W])."""
    d = synth.init_draws(N, seed=seed)
    dev = frame.device
    return _lib.init_plain(frame, mask.to(torch.uint8).contiguous(), _dev(d.pick_roi, dev),
                           _dev(d.jit_roi, dev), _dev(d.pick_out, dev), _dev(d.jit_out, dev))


def fit_to_target(shape, ws, target, params, psnr_target, cap, check_every, cfg):
    """Fit in place until PSNR >= target (checked every `check_every`) or
    `cap` iterations; returns (iterations to target or None, iterations run)."""
    N = shape.N
    dev = target.device
    m = torch.zeros(8 * N, device=dev)
    v = torch.zeros(8 * N, device=dev)
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    trace = torch.zeros(cap + check_every + 8, device=dev)
    st = _lib.fit_frame(shape, target, *params, m, v, step, trace, ws,
                        _lib.fit_opts(cap, check_every, psnr_target, cfg=cfg))
    hit = int(st.iter_hit_target)
    return (hit if hit >= 0 else None), int(st.iters_run)


def psnr_curve(shape, ws, target, params, budget, points, cfg):
    """PSNR of a cold fit at the given iteration counts (trace entry k is the
    loss of the parameters after k updates), run for `budget` iterations
    without a stop rule, on copies of `params`."""
    N = shape.N
    dev = target.device
    p = [q.clone() for q in params]
    m = torch.zeros(8 * N, device=dev)
    v = torch.zeros(8 * N, device=dev)
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    trace = torch.zeros(budget + 8, device=dev)
    _lib.fit_frame(shape, target, *p, m, v, step, trace, ws, _lib.fit_opts(budget, 50, cfg=cfg))
    tr = trace.cpu().numpy()
    return {int(k): psnr(float(tr[min(k, budget - 1)])) for k in points}


def make_training_set(seqs, n_frames, W, H, N, iters_first, iters_rest, device, lr=LR_DEFAULT,
                      log=print, frames=None):
    """Fitted Gaussians of every frame of the training sequences (frame 0
    from the content-aware init, later frames warm-started), the targets the
    learned initialiser is trained on.  `frames` (a dict, optional) receives
    every frame keyed by (seed, t) for reuse while training."""
    shape = _lib.make_shape(W, H, N, 32, px_per_lane=2)
    ws = _lib.alloc_workspace(shape, device)
    cfg = _lib.adam_cfg(lr)
    samples = []
    for si, seed in enumerate(seqs):
        params = None
        for t in range(n_frames):
            f, m = synth.make_frame_torch(W, H, seed, t, device)
            if frames is not None:
                frames[(seed, t)] = f
            if params is None:
                params = [p.contiguous() for p in plain_init_dev(f, m, N, seed + 7919)]
                iters = iters_first
            else:
                iters = iters_rest
            mm = torch.zeros(8 * N, device=device)
            vv = torch.zeros(8 * N, device=device)
            step = torch.zeros(1, dtype=torch.int32, device=device)
            trace = torch.zeros(iters + 8, device=device)
            _lib.fit_frame(shape, f, *params, mm, vv, step, trace, ws,
                           _lib.fit_opts(iters, 50, cfg=cfg))
            samples.append((seed, t, [p.clone() for p in params]))
        log(f"training sequence {si + 1}/{len(seqs)} fitted: last PSNR "
            f"{psnr(float(trace[iters - 1])):.2f} dB")
    return samples


def train_initialiser(net, samples, W, H, epochs, lr, device, log=print, seed=0, frames=None,
                      iframe_rate=0.1):
    """Epochs over the samples in a seeded random order; frames come from
    `frames` (keyed by (seed, t)) when given, else are synthesised again.
    A fraction `iframe_rate` of the P-frame samples is presented as an
    I-frame (no previous frame, zero residual input), so that the I-frame
    case is not limited to the first frame of each sequence."""
    rng = np.random.default_rng(seed)
    hist = []

    def frame(sd, t):
        if frames is not None and (sd, t) in frames:
            return frames[(sd, t)]
        return synth.make_frame_torch(W, H, sd, t, device)[0]

    for ep in range(epochs):
        order = rng.permutation(len(samples))
        tot = torch.zeros((), device=device)  # summed on the device: no per-step read-back
        for i, k in enumerate(order):
            sd, t, params = samples[k]
            f = frame(sd, t)
            as_iframe = t == 0 or rng.random() < iframe_rate
            prev = None if as_iframe else frame(sd, t - 1)
            net.forward(f, prev)
            net.set_targets(*params)
            loss = net.backward()
            net.step(lr=lr)
            tot += loss[0]
        hist.append(float(tot) / len(samples))
        log(f"epoch {ep + 1}/{epochs}: mean loss {hist[-1]:.4f}")
    return hist


def run_learned(train_seqs=34, frames_per_seq=60, max_samples=2000, epochs=6, eval_frames=60,
                W=1920, H=1080, N=30000, psnr_target=35.0, cap=10000, check_every=10,
                iters_first=2000, iters_rest=200, lr_cnn=1e-3, tau_pframe=1e-3,
                tau_sweep=(1e-2, 3e-2, 1e-1), device="cuda", log=print):
    """Train the per-tile initialiser on fitter outputs, then compare time and
    iterations to `psnr_target` on a held-out sequence for five arms:
    A plain init every frame, L learned init every frame, B plain init on
    frame 0 then warm start, C0 learned init on frame 0 then warm start, and
    C the network on every frame: learned init on frame 0, then each
    warm-started frame has the tiles whose mean squared residual exceeds
    tau_pframe re-initialised from the network's predictions (its forward
    pass and the replacement are inside the frame's clock).  Arm C is also
    run at each threshold of tau_sweep ("C@tau")."""
    t_all = time.perf_counter()
    seqs = [5000 + i for i in range(train_seqs)]
    # every training frame stays resident in HBM (34 x 60 1080p frames are
    # ~51 GB) when the device has room for it with a wide margin
    free, _ = torch.cuda.mem_get_info()
    frame_bytes = 3 * W * H * 4 * len(seqs) * frames_per_seq
    cache = {} if frame_bytes < 0.5 * free else None
    samples = make_training_set(seqs, frames_per_seq, W, H, N, iters_first, iters_rest, device,
                                log=log, frames=cache)[:max_samples]
    t_data = time.perf_counter() - t_all
    net = _lib.CNNInit(H, W, seed=11, device=device)
    t0 = time.perf_counter()
    hist = train_initialiser(net, samples, W, H, epochs, lr_cnn, device, log=log, frames=cache)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    resident = cache is not None
    del samples, cache
    # held-out evaluation
    shape = _lib.make_shape(W, H, N, 32, px_per_lane=2)
    ws = _lib.alloc_workspace(shape, device)
    cfg = _lib.adam_cfg(LR_DEFAULT)
    eval_seed = 5999
    frames = [synth.make_frame_torch(W, H, eval_seed, t, device) for t in range(eval_frames)]

    npred_log = {}

    def init_for(arm, t):
        f, m = frames[t]
        plain = [p.contiguous() for p in plain_init_dev(f, m, N, eval_seed + 31 * t + 1)]
        if arm in ("A", "B"):
            return plain
        prev = frames[t - 1][0] if t > 0 else None
        net.forward(f, prev)
        xy, chol, rgb, npred = net.decode(N, *plain)
        npred_log[t] = int(npred.item())
        return [xy, chol, rgb]

    # PSNR at a fixed iteration budget from cold starts: plain vs learned init
    points = (0, 50, 100, 200)
    budget = {"plain": {k: [] for k in points}, "learned": {k: [] for k in points}}
    for t in range(eval_frames):
        f = frames[t][0]
        for name, arm in (("plain", "A"), ("learned", "L")):
            curve = psnr_curve(shape, ws, f, init_for(arm, t), 201, points, cfg)
            for k in points:
                budget[name][k].append(curve[k])
    budget_mean = {name: {k: float(np.mean(v)) for k, v in d.items()} for name, d in budget.items()}
    log(f"PSNR at fixed budgets (mean over {eval_frames} frames): {budget_mean}")
    log(f"learned decode: predicted Gaussians per frame (N={N}): "
        f"{[npred_log[t] for t in sorted(npred_log)]}")

    res = {}
    stats = torch.zeros(4, dtype=torch.int32, device=device)
    replaced = {}
    arms = ["A", "L", "B", "C0", "C"] + [f"C@{tau:g}" for tau in tau_sweep]
    for arm in arms:
        tau = tau_pframe if arm == "C" else (float(arm[2:]) if arm.startswith("C@") else None)
        recs = []
        params = None
        for t in range(eval_frames):
            f = frames[t][0]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if arm in ("A", "L") or params is None:
                params = init_for(arm, t)
            elif tau is not None:
                prev = frames[t - 1][0]
                net.forward(f, prev)
                net.pframe_replace(f, prev, tau, *params, stats=stats)
            hit, run = fit_to_target(shape, ws, f, params, psnr_target, cap, check_every, cfg)
            torch.cuda.synchronize()
            recs.append({"iters": hit, "seconds": time.perf_counter() - t0, "iters_run": run})
            if tau is not None and t > 0:
                replaced.setdefault(arm, []).append([int(x) for x in stats.cpu()])
        ok = [r for r in recs if r["iters"] is not None]
        res[arm] = {"frames_reaching_target": len(ok),
                    "mean_seconds": float(np.mean([r["seconds"] for r in recs])),
                    "mean_iters_to_target": float(np.mean([r["iters"] for r in ok])) if ok else None,
                    "frame0_seconds": recs[0]["seconds"], "frame0_iters": recs[0]["iters"]}
        log(f"arm {arm}: {res[arm]}")
    ratio = lambda a, b: (res[a]["mean_seconds"] / res[b]["mean_seconds"])
    return {
        "workload": f"learned per-tile initialiser trained on {min(max_samples, train_seqs * frames_per_seq)} "
                    f"fitter outputs ({train_seqs} sequences x {frames_per_seq} frames, {W}x{H}, "
                    f"N={N}), {epochs} epochs; evaluated on {eval_frames} held-out frames",
        "target_psnr_db": psnr_target, "arms": res,
        "C_over_A_seconds": ratio("C", "A"), "C_over_B_seconds": ratio("C", "B"),
        "C0_over_B_seconds": ratio("C0", "B"), "tau_pframe": tau_pframe,
        "pframe_reinit_mean": {a: {k: float(np.mean([r[i] for r in rs])) for i, k in
                                   enumerate(("selected_tiles", "freed", "predicted", "replaced"))}
                               for a, rs in replaced.items()},
        "C_sweep_over_B_seconds": {a: ratio(a, "B") for a in arms if a.startswith("C@")},
        "L_over_A_seconds": ratio("L", "A"),
        "psnr_at_budget_cold": budget_mean,
        "learned_predicted_per_frame": [npred_log[t] for t in sorted(npred_log)],
        "train_loss_per_epoch": hist, "data_seconds": t_data, "train_seconds": t_train,
        "train_frames_resident": resident,
    }


def run_fit(W=640, H=360, N=1000, iters=1000, psnr_target=30.0, seed=950, device="cuda"):
    """One synthetic frame fitted from the content-aware init: iterations and
    seconds (init included) to `psnr_target`, and the iteration rate of an
    `iters`-iteration fit without a stop rule.  (tile, px per lane) from the
    autotuner on this frame."""
    f, m = synth.make_frame_torch(W, H, seed, 0, device)
    plain_init_dev(f, m, N, seed + 2)  # first use loads the library's code objects
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    params = [p.contiguous() for p in plain_init_dev(f, m, N, seed + 1)]
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    (T, ppl), _ = autotuned([(W, H, N)], f.reshape(-1), *params)
    shape = _lib.make_shape(W, H, N, T, px_per_lane=ppl)
    ws = _lib.alloc_workspace(shape, device)
    cfg = _lib.adam_cfg(LR_DEFAULT)
    # time to the target (read-backs every 10 iterations), from the same init
    p1 = [q.clone() for q in params]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hit, run = fit_to_target(shape, ws, f, p1, psnr_target, 10000, 10, cfg)
    torch.cuda.synchronize()
    t_target = time.perf_counter() - t0
    # iteration rate over a fixed budget
    p2 = [q.clone() for q in params]
    mm = torch.zeros(8 * N, device=device)
    vv = torch.zeros(8 * N, device=device)
    step = torch.zeros(1, dtype=torch.int32, device=device)
    trace = torch.zeros(iters + 8, device=device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _lib.fit_frame(shape, f, *p2, mm, vv, step, trace, ws, _lib.fit_opts(iters, 50, cfg=cfg))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"workload": f"one {W}x{H} synthetic frame, {N} Gaussians from the content-aware init",
            "tile": T, "px_per_lane": ppl, "init_seconds": t_init,
            "iters_to_target": hit, "target_psnr_db": psnr_target,
            "seconds_to_target_incl_init": (t_init + t_target) if hit is not None else None,
            "iters_per_s": iters / dt, "ms_per_iter": dt / iters * 1e3,
            "psnr_after_iters": psnr(float(trace[iters - 1])), "iters": iters}


def cnn_conv_flops(H, W):
    """Multiply-add FLOPs of the initialiser's convolutions for one H x W
    frame, counting real channels only (6 input channels, 73 head outputs):
    per layer 2 * Hout * Wout * Cout * 9 * Cin."""
    out, h, w, cin = [], H, W, 6
    for i in range(5):
        s = 2 if i < 4 else 1
        h, w = (h - 1) // s + 1, (w - 1) // s + 1
        cout = 64 if i < 4 else 73
        out.append(2.0 * h * w * cout * 9 * cin)
        cin = cout
    return out


def run_cnn_step(steps=20, warmup=3, W=1920, H=1080, N=30000, seed=900, device="cuda"):
    """Training steps of the initialiser on one synthetic frame pair and a
    synthetic fitted-Gaussian target set: forward, loss + backward, Adam.
    Times each phase with events on the stream the library launches on."""
    f0, _ = synth.make_frame_torch(W, H, seed, 0, device)
    f1, _ = synth.make_frame_torch(W, H, seed, 1, device)
    xy, chol, rgb = (torch.from_numpy(a).to(device) for a in
                     synth.random_gaussians(N, W, H, seed=seed + 1, scale_lo=0.6, scale_hi=3.0))
    net = _lib.CNNInit(H, W, seed=seed + 2, device=device)
    net.set_targets(xy, chol, rgb)
    for _ in range(warmup):
        net.forward(f1, f0)
        net.backward()
        net.step(lr=1e-4)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    t0 = time.perf_counter()
    for e in ev:
        e[0].record()
        net.forward(f1, f0)
        e[1].record()
        net.backward()
        e[2].record()
        net.step(lr=1e-4)
        e[3].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    fwd = sum(e[0].elapsed_time(e[1]) for e in ev) / steps
    bwd = sum(e[1].elapsed_time(e[2]) for e in ev) / steps
    adam = sum(e[2].elapsed_time(e[3]) for e in ev) / steps
    fl = cnn_conv_flops(H, W)
    return {"workload": "cnn_train_step", "size": [W, H], "steps": steps,
            "ms_forward": fwd, "ms_backward": bwd, "ms_adam": adam, "ms_step_wall": wall * 1e3,
            "conv_gflop_forward": sum(fl) / 1e9, "conv_gflop_step": 3 * sum(fl) / 1e9,
            "loss": float(net.loss3[0])}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["batch", "video", "learned", "cnn-step", "fit", "pframe",
                                      "compress", "superpixel"])
    ap.add_argument("--sequence", choices=["motion", "local"], default="motion")
    ap.add_argument("--tau", type=float, default=0.02)
    ap.add_argument("--tau-reinit", type=float, default=1e-3)
    ap.add_argument("--target", type=float, default=35.0)
    ap.add_argument("--frames", type=int, default=None)
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--train-seqs", type=int, default=34)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--eval-frames", type=int, default=60)
    ap.add_argument("--size", type=str, default="1920x1080")
    ap.add_argument("--N", type=int, default=30000)
    args = ap.parse_args(argv)
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    if args.which == "batch":
        out = run_batch(n_frames=args.frames or 48, iters=args.iters or 300)
    elif args.which == "video":
        out = run_video(n_frames=args.frames or 60, iters_rest=args.iters or 200)
    elif args.which == "fit":
        W, H = (int(x) for x in (args.size if args.size != "1920x1080" else "640x360").split("x"))
        out = run_fit(W=W, H=H, N=args.N if args.N != 30000 else 1000, iters=args.iters or 1000)
    elif args.which == "pframe":
        out = run_pframe(n_frames=args.frames or 30, tau=args.tau, sequence=args.sequence,
                         psnr_target=args.target)
        for arm in ("full", "selective"):
            out[arm].pop("per_frame")
    elif args.which == "compress":
        out = run_compress(iters=args.iters or 1000)
    elif args.which == "superpixel":
        W, H = (int(x) for x in args.size.split("x"))
        out = run_superpixel(n_frames=args.frames or 3, W=W, H=H, N=args.N,
                             psnr_target=args.target, cap=args.iters or 3000)
    elif args.which == "cnn-step":
        W, H = (int(x) for x in args.size.split("x"))
        out = run_cnn_step(steps=args.iters or 20, W=W, H=H, N=args.N)
    else:
        W, H = (int(x) for x in args.size.split("x"))
        out = run_learned(train_seqs=args.train_seqs, frames_per_seq=args.frames or 60,
                          epochs=args.epochs, eval_frames=args.eval_frames, W=W, H=H, N=args.N,
                          tau_pframe=args.tau_reinit, log=log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    sys.exit(main())
