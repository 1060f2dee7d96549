#!/usr/bin/env python
"""Fitting-iteration throughput on one MI355X: one 1920x1080 synthetic frame,
30,000 Gaussians from the content-aware ROI initialisation, Adam.

A step is one fitting iteration: projection + tile binning + tile sort,
fused forward render / MSE / backward render, Adam.  The tile lists are
binned lazily (--bin-skin pixels of margin; rebuilt when a Gaussian's exact
tile rectangle leaves its binned one, and at every chunk start): every
iteration still projects every Gaussian and renders with exact per-pixel
cutoffs.  Prints one JSON line.

    python bench.py [--steps 1950] [--warmup 50] [--no-cpu-baseline]

Besides the throughput the line carries
  roofline      the dominant kernel (fused per-tile forward+backward): back
                to back launches on the torch stream captured in a graph, as
                the fitting loop replays them, timed with HIP events around
                the replay; against the FP32 vector peak, with its
                algorithmic FLOPs = 52 per (pixel, Gaussian) pair inside the
                3-sigma cutoff; traffic from the committed counter record;
  cpu_baseline  the FP64 oracle timed on this host's cores on a bounded
                sample (a few full iterations of the same workload);
  m2            seconds per frame to 35 dB on held-out 1080p frames for the
                initialisation arms (A plain init every frame, L learned
                init every frame, B plain init then warm start, C the
                network on every frame: learned init, then learned
                re-initialisation of the changed tiles of each warm-started
                frame; C0 learned init then warm start), with the network
                trained on a reduced set of fitter outputs stated in its
                config (outside the timed region).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

W, H, N, TILE = 1920, 1080, 30000, 16
FRAME_SEED, INIT_SEED = 201, 202
LR = (2e-2, 5e-3, 5e-3)        # per group: mean, Cholesky vector, colour
FLOPS_PER_PAIR = 52            # 16 forward + 36 backward per in-cutoff pair
PEAK_FP32 = 157.3              # TFLOP/s, MI355X FP32 vector (datasheet)
HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------ CPU baseline --
_CPU = {}


def _cpu_worker_init(shm_names, shape_img, P):
    from multiprocessing import shared_memory
    _CPU["shm"] = [shared_memory.SharedMemory(name=n) for n in shm_names]
    _CPU["parts"] = np.ndarray((P,) + shape_img, np.float64, buffer=_CPU["shm"][0].buf)
    _CPU["dl"] = np.ndarray(shape_img, np.float64, buffer=_CPU["shm"][1].buf)


def _cpu_render(args):
    from oracle.render import render_box
    slot, xy, chol, rgb = args
    _CPU["parts"][slot] = render_box(xy, chol, rgb, H, W, want_bounds=False)["img"]
    return slot


def _cpu_grads(args):
    from oracle.grads import gradients
    xy, chol, rgb = args
    g = gradients(xy, chol, rgb, _CPU["dl"], H, W)
    return g["g_xy"], g["g_chol"], g["g_rgb"]


def cpu_baseline(iters: int):
    """The oracle (render, MSE, gradients, Adam in FP64) on the host cores:
    Gaussians split into one contiguous chunk per process, partial images
    and gradients summed.  Runs before anything touches the GPU."""
    import multiprocessing as mp
    from multiprocessing import shared_memory

    from oracle.adam import adam_step
    from oracle.init import init_from_frame
    from oracle.loss import dloss_dimg, mse
    from paper_2505_09324_amd import synth

    frame, mask = synth.make_frame(W, H, seed=FRAME_SEED)
    xy, chol, rgb, _ = init_from_frame(frame, mask, synth.init_draws(N, seed=INIT_SEED))
    P = max(1, min(os.cpu_count() or 1, 16))
    shape_img = (3, H, W)
    nb = int(np.prod(shape_img)) * 8
    shm = [shared_memory.SharedMemory(create=True, size=nb * P),
           shared_memory.SharedMemory(create=True, size=nb)]
    try:
        parts = np.ndarray((P,) + shape_img, np.float64, buffer=shm[0].buf)
        dl = np.ndarray(shape_img, np.float64, buffer=shm[1].buf)
        theta = {"xy": xy.astype(np.float64), "chol": chol.astype(np.float64),
                 "rgb": rgb.astype(np.float64)}
        m = {k: np.zeros_like(v) for k, v in theta.items()}
        v = {k: np.zeros_like(x) for k, x in theta.items()}
        lr = {"xy": LR[0], "chol": LR[1], "rgb": LR[2]}
        bounds = np.linspace(0, N, P + 1).astype(int)
        ctx = mp.get_context("fork")
        with ctx.Pool(P, initializer=_cpu_worker_init,
                      initargs=([s.name for s in shm], shape_img, P)) as pool:
            t0 = time.perf_counter()
            t = 0
            for _ in range(iters):
                ch = [(i, theta["xy"][a:b], theta["chol"][a:b], theta["rgb"][a:b])
                      for i, (a, b) in enumerate(zip(bounds[:-1], bounds[1:]))]
                pool.map(_cpu_render, ch)
                img = parts.sum(axis=0)
                _ = mse(img, frame)
                dl[:] = dloss_dimg(img, frame)
                res = pool.map(_cpu_grads, [c[1:] for c in ch])
                grad = {"xy": np.concatenate([r[0] for r in res]),
                        "chol": np.concatenate([r[1] for r in res]),
                        "rgb": np.concatenate([r[2] for r in res])}
                theta, m, v, t = adam_step(theta, grad, m, v, t, lr)
            dt = time.perf_counter() - t0
    finally:
        for s in shm:
            s.close()
            s.unlink()
    cpu_model = None
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")),
                             None)
    except OSError:
        pass
    return {"value": iters / dt, "unit": "iters/s", "cores": P, "kind": "oracle",
            "cpu_model": cpu_model, "os_cpu_count": os.cpu_count(),
            "sample": f"{iters} full FP64 iterations (render, MSE, gradients, Adam) of the "
                      f"1920x1080 / 30k-Gaussian workload from its initialisation, "
                      f"{P} processes", "seconds": round(dt, 3)}


# ------------------------------------------------------------------- GPU --
def traffic_record(kernel_src_digest: str):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(HERE, "profiles", "render_fused_1080p_30k_traffic.txt")
    try:
        with open(path) as f:
            rec = json.load(f)
    except OSError:
        return None
    if rec.get("kernel_source_sha256") != kernel_src_digest:
        return None
    return rec.get("bytes_per_launch")


def kernel_digest():
    import hashlib
    h = hashlib.sha256()
    for fn in ("raster.hip", "raster_tile.h", "gs2d_internal.h"):
        with open(os.path.join(HERE, "paper_2505_09324_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def time_graph(fn, reps):
    """Mean seconds per call of `fn` (library launches on the current
    stream), the calls captured back to back in one graph as the fitting
    loop replays them, timed with HIP events around the replay."""
    import torch
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(reps):
            fn()
    graph.replay()  # warm
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    graph.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1950)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--check-every", type=int, default=50)
    ap.add_argument("--tile", type=int, default=0,
                    help="tile size (8/16/32); 0 = choose with the autotuner")
    ap.add_argument("--ppl", type=int, default=0,
                    help="pixels per lane of the raster kernels (1/2/4); 0 = autotuner")
    ap.add_argument("--sweep", action="store_true",
                    help="also time the fused kernel for every (tile, ppl) variant (stderr)")
    ap.add_argument("--launch", choices=("graph", "eager"), default="graph",
                    help="fitting chunks replayed as captured hipGraphs, or launched directly")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--bin-skin", type=float, default=1.0,
                    help="lazy tile binning margin in pixels (0: rebuild the lists every iteration)")
    ap.add_argument("--cpu-iters", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-m2", action="store_true")
    ap.add_argument("--m2-seqs", type=int, default=8, help="training sequences of the M2 network")
    ap.add_argument("--m2-frames", type=int, default=30, help="frames per training sequence")
    ap.add_argument("--m2-eval", type=int, default=30, help="held-out evaluation frames")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (independent frames or "
              "groups of pictures would be sharded across GPUs, one process each); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_iters)    # before the GPU is initialised

    import torch
    from paper_2505_09324_amd import _lib, synth

    dev = "cuda"
    frame, mask = synth.make_frame(W, H, seed=FRAME_SEED)
    draws = synth.init_draws(N, seed=INIT_SEED)
    T = torch.from_numpy(frame).to(dev)
    M8 = torch.from_numpy(mask.astype(np.uint8)).to(dev)
    td = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    xy, chol, rgb = _lib.init_plain(T, M8, td(draws.pick_roi), td(draws.jit_roi),
                                    td(draws.pick_out), td(draws.jit_out))
    tune = None
    if args.tile == 0 or args.ppl == 0:
        cands = [(8, 1), (16, 1), (16, 2), (32, 1), (32, 2), (32, 4)]
        best, ms = _lib.autotune_frame(W, H, N, T, xy, chol, rgb, cands, reps=5)
        args.tile, args.ppl = cands[best]
        tune = {f"{t}/{p}": round(x * 1e3, 1) for (t, p), x in zip(cands, ms)}
    shape = _lib.make_shape(W, H, N, args.tile, px_per_lane=args.ppl)
    ws = _lib.alloc_workspace(shape)
    m = torch.zeros(8 * N, device=dev)
    v = torch.zeros(8 * N, device=dev)
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    trace = torch.zeros(args.warmup + args.steps + 8, device=dev)
    cfg = _lib.adam_cfg(LR)
    ctx = _lib.Context()
    use_graph = args.launch == "graph"
    fit = lambda iters, chunk: (shape, T, xy, chol, rgb, m, v, step, trace, ws,
                                _lib.fit_opts(iters, chunk, use_graph=use_graph, cfg=cfg,
                                              bin_skin=args.bin_skin))

    if args.warmup > 0:
        _lib.fit_frame(*fit(args.warmup, min(args.check_every, args.warmup)), ctx=ctx)
    # the warm-up also instantiates the graphs the timed call replays; its
    # arguments are built once, outside the timed region
    timed = fit(args.steps, args.check_every)
    _lib.fit_prepare(*timed, ctx=ctx)
    call = _lib.FitCall(*timed, ctx=ctx)
    captures0 = ctx.stats()[1]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = call()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert ctx.stats()[1] == captures0, "the timed call captured a graph"
    tr = trace[:args.warmup + args.steps].cpu().numpy()
    psnr_final = float(10 * np.log10(1.0 / tr[-1]))

    # --- dominant kernel, timed live with events on its own stream ---------
    _lib.project_bin(shape, xy, chol, ws)
    p_in = _lib.count_pairs(shape, ws)
    n_pairs = int(_lib.read_bins(shape, ws)["n_pairs"])
    g = [torch.zeros(N, d, device=dev) for d in (2, 3, 3)]
    _lib.render_fused(shape, ws, rgb, T, *g)          # warm
    t_fused = time_graph(lambda: _lib.render_fused(shape, ws, rgb, T, *g), args.kernel_reps)
    # other stages, same way
    t_bin = time_graph(lambda: _lib.project_bin(shape, xy, chol, ws), args.kernel_reps)
    step2 = torch.zeros(1, dtype=torch.int32, device=dev)
    mm, vv = m.clone(), v.clone()
    xs, cs, rs = xy.clone(), chol.clone(), rgb.clone()
    t_adam = time_graph(lambda: _lib.adam_step(xs, cs, rs, *g, mm, vv, step2, cfg), args.kernel_reps)
    # the unfused raster entry points (the autograd path): forward with the
    # loss and dL/dC, and the backward from dL/dC (which first clears g)
    dl = torch.empty(3, H, W, device=dev)
    loss_d = torch.zeros((), device=dev)
    t_fwd = time_graph(lambda: _lib.render_fwd(shape, ws, rgb, target=T, dl_dimg=dl, loss=loss_d),
                       args.kernel_reps)
    t_bwd = time_graph(lambda: _lib.render_bwd(shape, ws, rgb, dl, *g), args.kernel_reps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    if args.sweep:
        for tt, pp in ((8, 1), (16, 1), (16, 2), (32, 1), (32, 2), (32, 4)):
            sh = _lib.make_shape(W, H, N, tt, px_per_lane=pp)
            wsv = _lib.alloc_workspace(sh)
            _lib.project_bin(sh, xy, chol, wsv)
            _lib.render_fused(sh, wsv, rgb, T, *g)
            e0.record()
            for _ in range(args.kernel_reps):
                _lib.render_fused(sh, wsv, rgb, T, *g)
            e1.record()
            torch.cuda.synchronize()
            print(f"variant tile={tt} ppl={pp}: {e0.elapsed_time(e1) / args.kernel_reps * 1e3:.1f} us",
                  file=sys.stderr, flush=True)
            del wsv

    flops = FLOPS_PER_PAIR * p_in
    achieved = flops / t_fused / 1e12
    traffic = traffic_record(kernel_digest())
    out = {
        "metric": "1080p fit iters/s (fwd+bwd, 30k Gaussians); s/frame to 35 dB, learned vs plain init",
        "value": round(args.steps / dt, 2),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "one 1920x1080 synthetic talking-head-like frame, 30000 Gaussians "
                               "from the content-aware ROI init (70% in ROI), Adam iterations "
                               f"{args.warmup}..{args.warmup + args.steps}",
                   "W": W, "H": H, "N": N, "tile": args.tile, "px_per_lane": args.ppl,
                   "lr": list(LR),
                   "launch": args.launch, "chunk": args.check_every,
                   "bin_skin_px": args.bin_skin},
        "tile_list_rebuilds": int(st.rebins),
        "psnr_final_db": round(psnr_final, 3),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32, 4),
                     "traffic": traffic, "kernel": f"k_render_fused<{args.tile}, {args.ppl}>",
                     "launch_us": round(t_fused * 1e6, 2), "pairs_in_cutoff": p_in,
                     "flops_per_launch": flops},
        "stages_us": {"project_bin": round(t_bin * 1e6, 2), "render_fused": round(t_fused * 1e6, 2),
                      "adam": round(t_adam * 1e6, 2), "render_fwd_loss": round(t_fwd * 1e6, 2),
                      "render_bwd": round(t_bwd * 1e6, 2)},
        "n_pairs": n_pairs,
        "autotune_us_per_round": tune,
        "autotune_kernels": "one-frame binning + k_render_fused per candidate (tile/px per lane)",
        "cpu_baseline": cpu,
    }
    if not args.no_m2:
        out["m2"] = m2_record(args)
    print(json.dumps(out), flush=True)


def m2_record(args):
    """s/frame to 35 dB per initialisation arm (learned vs plain init), from
    the learned-initialiser workload on a reduced training set."""
    from paper_2505_09324_amd import workloads
    log = lambda msg: print(msg, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    r = workloads.run_learned(train_seqs=args.m2_seqs, frames_per_seq=args.m2_frames,
                              max_samples=args.m2_seqs * args.m2_frames, epochs=6,
                              eval_frames=args.m2_eval, W=W, H=H, N=N, psnr_target=35.0,
                              tau_sweep=(), log=log)
    arms = r["arms"]
    return {
        "metric": "s/frame to 35 dB, learned vs plain init",
        "unit": "s/frame",
        "higher_is_better": False,
        "config": {"workload": f"per-tile initialiser trained on {args.m2_seqs * args.m2_frames} "
                               f"fitter outputs ({args.m2_seqs} synthetic sequences x "
                               f"{args.m2_frames} frames, seeds 5000..{5000 + args.m2_seqs - 1}; "
                               "frame 0 fitted 2000 iterations, the rest warm-started 200), "
                               f"6 epochs; evaluated on {args.m2_eval} held-out frames (seed "
                               "5999), 1920x1080, 30000 Gaussians, PSNR checked every 10 "
                               "iterations, clock from the frame resident to the first check "
                               ">= 35 dB including the initialisation",
                   "tau_reinit": r["tau_pframe"]},
        "s_per_frame": {a: round(v["mean_seconds"], 5) for a, v in arms.items()},
        "iters_to_target": {a: v["mean_iters_to_target"] for a, v in arms.items()},
        "frames_reaching_target": {a: v["frames_reaching_target"] for a, v in arms.items()},
        "C_over_A": round(r["C_over_A_seconds"], 4), "C_over_B": round(r["C_over_B_seconds"], 4),
        "L_over_A": round(r["L_over_A_seconds"], 4), "C0_over_B": round(r["C0_over_B_seconds"], 4),
        "reinit_per_frame": r["pframe_reinit_mean"].get("C"),
        "seconds_total": round(time.perf_counter() - t0, 1),
    }


if __name__ == "__main__":
    main()
