"""Drivers for the fitting workloads, on top of the C ABI.

Each driver only sequences library calls (initialise, fit, time); every step
of the fit runs in the HIP library.

    python -m paper_2505_09324_amd.workloads batch   # 48 uneven frames, one launch per stage
    python -m paper_2505_09324_amd.workloads video   # warm-started sequence
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import _lib, synth

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


def autotuned(sizes, targets, xy, chol, rgb, reps=3):
    cands = [(8, 1), (16, 1), (16, 2), (32, 1), (32, 2), (32, 4)]
    best, ms = _lib.autotune_batch(sizes, targets, xy, chol, rgb, cands, reps=reps)
    return cands[best], dict(zip([f"{t}/{p}" for t, p in cands], ms))


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
        "status": int(st.status),
    }


# ------------------------------------------------------------------ video --
def fit_sequence(frames, masks, N, iters_first, iters_rest, init_seed, tile=16, ppl=1,
                 lr=LR_DEFAULT, psnr_target=0.0, check_every=10, device="cuda",
                 warm_start=True, init_fn=None):
    """Fit a sequence frame by frame.  Frame 0 starts from `init_fn` (default
    the content-aware init); with warm_start each later frame starts from the
    previous frame's fitted Gaussians with the Adam state reset, otherwise
    from its own init.  Returns per-frame records."""
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


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["batch", "video"])
    ap.add_argument("--frames", type=int, default=None)
    ap.add_argument("--iters", type=int, default=None)
    args = ap.parse_args(argv)
    if args.which == "batch":
        out = run_batch(n_frames=args.frames or 48, iters=args.iters or 300)
    else:
        out = run_video(n_frames=args.frames or 60, iters_rest=args.iters or 200)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    sys.exit(main())
