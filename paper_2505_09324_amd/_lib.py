"""ctypes binding of libgs2d.so (the C ABI in include/gs2d.h).

Argument marshalling only: every call checks tensor devices, dtypes, shapes
and contiguity, converts them to raw device pointers and passes the current
torch stream.  All computation happens in the HIP library; if the library
is missing the import of any entry point raises instead of falling back.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t, c_uint32,
                    c_void_p)

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgs2d.so")

GS2D_OK, GS2D_EINVAL, GS2D_ENOSPACE, GS2D_EOVERFLOW, GS2D_EHIP = 0, -1, -2, -3, -4
STATUS_OVERFLOW, STATUS_CULLED = 1, 2
GS2D_STATIC_WORKSPACE_BYTES = 16 << 20   # gs2d_fit_frame_static's device array


class Shape(ctypes.Structure):
    _fields_ = [("W", c_int32), ("H", c_int32), ("N", c_int32), ("tile", c_int32),
                ("max_pairs", c_int32), ("px_per_lane", c_int32)]


class Bins(ctypes.Structure):
    _fields_ = [("geom", c_void_p), ("counts", c_void_p), ("offsets", c_void_p),
                ("keys", c_void_p), ("tile_start", c_void_p), ("n_pairs", c_void_p),
                ("status", c_void_p), ("n_culled", c_void_p),
                ("n_tiles", c_int32), ("tiles_x", c_int32), ("tiles_y", c_int32)]


class AdamCfg(ctypes.Structure):
    _fields_ = [("lr", c_float * 3), ("beta1", c_float), ("beta2", c_float), ("eps", c_float)]


class QuantCfg(ctypes.Structure):
    _fields_ = [("bits_chol", c_int32), ("bits_rgb", c_int32)]


class FitOpts(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("check_every", c_int32), ("psnr_target", c_float),
                ("use_graph", c_int32), ("adam", AdamCfg), ("active", c_void_p),
                ("qat", POINTER(QuantCfg)), ("bin_skin", c_float), ("batch_persistent", c_int32)]


class FitStats(ctypes.Structure):
    _fields_ = [("iters_run", c_int32), ("iter_hit_target", c_int32), ("final_loss", c_float),
                ("final_psnr", c_float), ("seconds", c_double), ("status", c_uint32),
                ("n_culled", c_int32), ("rebins", c_int32)]


class Frame(ctypes.Structure):
    _fields_ = [("W", c_int32), ("H", c_int32), ("N", c_int32)]


class GS2DError(RuntimeError):
    def __init__(self, fn, code):
        super().__init__(f"{fn} failed: {status_str(code)} ({code})")
        self.code = code


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "gs2d_status_str": (c_char_p, [c_int32]),
    "gs2d_workspace_bytes": (c_size_t, [POINTER(Shape)]),
    "gs2d_bins_view": (c_int32, [POINTER(Shape), c_void_p, c_size_t, POINTER(Bins)]),
    "gs2d_project_bin": (c_int32, [POINTER(Shape), c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "gs2d_render_fwd": (c_int32, [POINTER(Shape), c_void_p, c_size_t, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_void_p]),
    "gs2d_render_bwd": (c_int32, [POINTER(Shape), c_void_p, c_size_t, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_void_p]),
    "gs2d_adam_step": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_void_p, c_void_p, c_void_p, POINTER(AdamCfg), c_void_p, c_int32,
                                 c_void_p]),
    "gs2d_select_changed": (c_int32, [POINTER(Shape), c_void_p, c_size_t, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_float, c_void_p, c_void_p, c_void_p]),
    "gs2d_ptq_workspace_bytes": (c_size_t, [c_int32]),
    "gs2d_ptq": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p, POINTER(QuantCfg), c_void_p,
                           c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                           c_void_p]),
    "gs2d_ctx_create": (c_int32, [POINTER(c_void_p), c_int32]),
    "gs2d_ctx_destroy": (None, [c_void_p]),
    "gs2d_ctx_stats": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int64)]),
    "gs2d_fit_frame": (c_int32, [c_void_p, POINTER(Shape), c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_size_t,
                                 POINTER(FitOpts), POINTER(FitStats), c_void_p]),
    "gs2d_fit_frame_static": (c_int32, [POINTER(Shape), c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p, c_void_p, c_void_p, c_void_p, c_int32,
                                        POINTER(FitOpts), POINTER(FitStats), c_void_p]),
    "gs2d_fit_prepare": (c_int32, [c_void_p, POINTER(Shape), c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32,
                                   c_void_p, c_size_t, POINTER(FitOpts)]),
    "gs2d_autotune_frame": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_void_p,
                                      c_void_p, c_size_t, c_void_p, c_void_p, c_void_p]),
    "gs2d_render_fused": (c_int32, [POINTER(Shape), c_void_p, c_size_t, c_void_p, c_void_p, c_void_p,
                                    c_void_p, c_void_p, c_void_p, c_void_p]),
    "gs2d_count_pairs": (c_int32, [POINTER(Shape), c_void_p, c_size_t, c_void_p, c_void_p]),
    "gs2d_batch_workspace_bytes": (c_size_t, [c_int32, POINTER(Frame), c_int32, c_int32]),
    "gs2d_fit_batch": (c_int32, [c_void_p, c_int32, POINTER(Frame), c_int32, c_int32, c_void_p, c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_int32, c_void_p, c_size_t, POINTER(FitOpts), POINTER(FitStats),
                                 c_void_p]),
    "gs2d_batch_render_grads": (c_int32, [c_int32, POINTER(Frame), c_int32, c_int32, c_void_p,
                                          c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                          c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "gs2d_batch_bins_view": (c_int32, [c_int32, POINTER(Frame), c_int32, c_int32, c_int32,
                                       c_void_p, c_size_t, POINTER(Bins)]),
    "gs2d_autotune_batch": (c_int32, [c_int32, POINTER(Frame), c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_void_p,
                                      c_void_p, c_size_t, c_void_p, c_void_p, c_void_p]),
    "gs2d_cnn_param_count": (c_size_t, [c_int32, c_int32]),
    "gs2d_cnn_workspace_bytes": (c_size_t, [c_int32, c_int32]),
    "gs2d_cnn_bf16_weight_count": (c_size_t, [c_int32, c_int32]),
    "gs2d_cnn_layer_info": (c_int32, [c_int32, c_int32, c_int32, c_void_p]),
    "gs2d_cnn_init_params": (c_int32, [c_int32, c_int32, c_void_p, c_void_p, c_void_p]),
    "gs2d_cnn_sync_weights": (c_int32, [c_int32, c_int32, c_void_p, c_void_p, c_void_p]),
    "gs2d_cnn_forward": (c_int32, [c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_void_p, c_size_t, c_void_p]),
    "gs2d_cnn_targets": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_size_t, c_void_p, c_size_t, c_void_p]),
    "gs2d_cnn_read_targets": (c_int32, [c_int32, c_int32, c_void_p, c_size_t, c_void_p, c_void_p,
                                        c_void_p]),
    "gs2d_cnn_tensor_view": (c_int32, [c_int32, c_int32, c_int32, c_int32, c_void_p, c_size_t,
                                       POINTER(c_void_p), c_void_p]),
    "gs2d_cnn_backward": (c_int32, [c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_void_p, c_size_t, c_void_p]),
    "gs2d_cnn_adam": (c_int32, [c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_void_p, c_float, c_float, c_void_p, c_void_p]),
    "gs2d_cnn_decode": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                  c_void_p, c_size_t, c_void_p]),
    "gs2d_init_workspace_bytes": (c_size_t, [c_int32, c_int32]),
    "gs2d_init_plain": (c_int32, [c_int32, c_int32, c_void_p, c_void_p, c_int32, c_void_p, c_void_p,
                                  c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_size_t, c_void_p]),
    "gs2d_cnn_pframe_scratch_bytes": (c_size_t, [c_int32, c_int32, c_int32]),
    "gs2d_cnn_pframe_replace": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_void_p, c_float,
                                          c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                          c_void_p, c_void_p, c_size_t, c_void_p, c_size_t,
                                          c_void_p]),
    "gs2d_superpixel_workspace_bytes": (c_size_t, [c_int32, c_int32, c_int32]),
    "gs2d_init_superpixel": (c_int32, [c_int32, c_int32, c_void_p, c_void_p, c_int32, c_void_p,
                                       c_int32, c_float, c_void_p, c_void_p, c_void_p, c_void_p,
                                       c_void_p, c_void_p, c_size_t, c_void_p]),
}


def exported_symbols():
    return sorted(_SIGS)


def lib():
    """Load libgs2d.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2505_09324_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def status_str(code: int) -> str:
    return lib().gs2d_status_str(int(code)).decode()


def _check(fn, code):
    if code != GS2D_OK:
        raise GS2DError(fn, code)


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, name, dtype=torch.float32, shape=None, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return c_void_p(t.data_ptr())


def make_shape(W, H, N, tile=16, max_pairs=None, px_per_lane=1) -> Shape:
    if max_pairs is None:
        max_pairs = default_max_pairs(W, H, N, tile)
    return Shape(int(W), int(H), int(N), int(tile), int(max_pairs), int(px_per_lane))


def default_max_pairs(W, H, N, tile) -> int:
    tx, ty = -(-W // tile), -(-H // tile)
    return int(min(1 << 30, max(1 << 16, 16 * N + 4 * tx * ty)))


def workspace_bytes(shape: Shape) -> int:
    n = lib().gs2d_workspace_bytes(ctypes.byref(shape))
    if n == 0:
        raise GS2DError("gs2d_workspace_bytes", GS2D_EINVAL)
    return int(n)


def alloc_workspace(shape: Shape, device="cuda") -> torch.Tensor:
    return torch.empty(workspace_bytes(shape), dtype=torch.uint8, device=device)


def bins_view(shape: Shape, ws: torch.Tensor) -> Bins:
    b = Bins()
    _check("gs2d_bins_view", lib().gs2d_bins_view(ctypes.byref(shape), _ptr(ws, "ws", torch.uint8),
                                                  ws.numel(), ctypes.byref(b)))
    return b


def _slice(ws: torch.Tensor, ptr: int, count: int, dtype) -> torch.Tensor:
    off = ptr - ws.data_ptr()
    nbytes = count * torch.empty((), dtype=dtype).element_size()
    return ws[off:off + nbytes].view(dtype)


def read_bins(shape: Shape, ws: torch.Tensor) -> dict:
    """Copies of the binning results (host tensors)."""
    b = bins_view(shape, ws)
    n_pairs = int(_slice(ws, b.n_pairs, 1, torch.int32).item())
    keys = _slice(ws, b.keys, n_pairs, torch.int32).cpu().numpy().view("uint32")
    return {
        "n_pairs": n_pairs,
        "keys": keys,
        "pair_ids": (keys & 0xFFFF).astype("int64"),
        "pair_tiles": (keys >> 16).astype("int64"),
        "tile_start": _slice(ws, b.tile_start, b.n_tiles + 1, torch.int32).cpu().numpy().astype("int64"),
        "counts": _slice(ws, b.counts, shape.N, torch.int32).cpu().numpy().astype("int64"),
        "offsets": _slice(ws, b.offsets, shape.N + 1, torch.int32).cpu().numpy().astype("int64"),
        "status": int(_slice(ws, b.status, 1, torch.int32).item()),
        "n_culled": int(_slice(ws, b.n_culled, 1, torch.int32).item()),
        "n_tiles": b.n_tiles, "TX": b.tiles_x, "TY": b.tiles_y,
    }


def project_bin(shape: Shape, xy, chol, ws):
    N = shape.N
    _check("gs2d_project_bin", lib().gs2d_project_bin(
        ctypes.byref(shape), _ptr(xy, "xy", shape=(N, 2)), _ptr(chol, "chol", shape=(N, 3)),
        _ptr(ws, "ws", torch.uint8), ws.numel(), _stream()))


def render_fwd(shape: Shape, ws, rgb, target=None, img=None, dl_dimg=None, loss=None):
    N, H, W = shape.N, shape.H, shape.W
    _check("gs2d_render_fwd", lib().gs2d_render_fwd(
        ctypes.byref(shape), _ptr(ws, "ws", torch.uint8), ws.numel(),
        _ptr(rgb, "rgb", shape=(N, 3)),
        _ptr(target, "target", shape=(3, H, W), allow_none=True),
        _ptr(img, "img", shape=(3, H, W), allow_none=True),
        _ptr(dl_dimg, "dl_dimg", shape=(3, H, W), allow_none=True),
        _ptr(loss, "loss", shape=(), allow_none=True), _stream()))


def render_bwd(shape: Shape, ws, rgb, dl_dimg, g_xy, g_chol, g_rgb):
    N, H, W = shape.N, shape.H, shape.W
    _check("gs2d_render_bwd", lib().gs2d_render_bwd(
        ctypes.byref(shape), _ptr(ws, "ws", torch.uint8), ws.numel(),
        _ptr(rgb, "rgb", shape=(N, 3)), _ptr(dl_dimg, "dl_dimg", shape=(3, H, W)),
        _ptr(g_xy, "g_xy", shape=(N, 2)), _ptr(g_chol, "g_chol", shape=(N, 3)),
        _ptr(g_rgb, "g_rgb", shape=(N, 3)), _stream()))


def render_fused(shape: Shape, ws, rgb, target, g_xy, g_chol, g_rgb, loss=None):
    """Fused forward + MSE + backward; gradients are accumulated into g_*."""
    N, H, W = shape.N, shape.H, shape.W
    _check("gs2d_render_fused", lib().gs2d_render_fused(
        ctypes.byref(shape), _ptr(ws, "ws", torch.uint8), ws.numel(),
        _ptr(rgb, "rgb", shape=(N, 3)), _ptr(target, "target", shape=(3, H, W)),
        _ptr(g_xy, "g_xy", shape=(N, 2)), _ptr(g_chol, "g_chol", shape=(N, 3)),
        _ptr(g_rgb, "g_rgb", shape=(N, 3)), _ptr(loss, "loss", shape=(), allow_none=True),
        _stream()))


def count_pairs(shape: Shape, ws) -> int:
    """In-cutoff (pixel, Gaussian) pairs of the current tile lists."""
    out = torch.zeros(1, dtype=torch.int64, device=ws.device)
    _check("gs2d_count_pairs", lib().gs2d_count_pairs(
        ctypes.byref(shape), _ptr(ws, "ws", torch.uint8), ws.numel(), _ptr(out, "out", torch.int64),
        _stream()))
    return int(out.item())


def adam_cfg(lr=(1e-2, 1e-2, 1e-2), beta1=0.9, beta2=0.999, eps=1e-8) -> AdamCfg:
    if isinstance(lr, (int, float)):
        lr = (lr, lr, lr)
    return AdamCfg((c_float * 3)(*lr), beta1, beta2, eps)


def adam_step(xy, chol, rgb, g_xy, g_chol, g_rgb, m, v, step, cfg: AdamCfg, active=None,
              zero_grads=False):
    N = xy.shape[0]
    _check("gs2d_adam_step", lib().gs2d_adam_step(
        N, _ptr(xy, "xy", shape=(N, 2)), _ptr(chol, "chol", shape=(N, 3)),
        _ptr(rgb, "rgb", shape=(N, 3)), _ptr(g_xy, "g_xy", shape=(N, 2)),
        _ptr(g_chol, "g_chol", shape=(N, 3)), _ptr(g_rgb, "g_rgb", shape=(N, 3)),
        _ptr(m, "m", shape=(8 * N,)), _ptr(v, "v", shape=(8 * N,)),
        _ptr(step, "step", torch.int32, shape=(1,)), ctypes.byref(cfg),
        _ptr(active, "active", torch.uint8, shape=(N,), allow_none=True), int(bool(zero_grads)),
        _stream()))


def fit_opts(iters, check_every=50, psnr_target=0.0, use_graph=True, cfg=None,
             active=None, qat=None, bin_skin=1.0, batch_persistent=False) -> FitOpts:
    """Fitting options; active: [N] uint8 device tensor (only Gaussians with
    a non-zero flag are optimised) or None; qat: (bits_chol, bits_rgb) for
    quantisation-aware fitting, or None; bin_skin: lazy tile binning margin
    in pixels (0: rebuild the lists every iteration); batch_persistent: the
    batched fit's raster as one persistent work-queue launch instead of one
    workgroup per (frame, tile)."""
    o = FitOpts(int(iters), int(check_every), float(psnr_target), int(bool(use_graph)),
                cfg if cfg is not None else adam_cfg(), None, None, float(bin_skin),
                int(bool(batch_persistent)))
    if active is not None:
        o.active = _ptr(active, "active", torch.uint8)
        o._active_ref = active  # keep the tensor alive with the options
    if qat is not None:
        q = QuantCfg(int(qat[0]), int(qat[1]))
        o.qat = ctypes.pointer(q)
        o._qat_ref = q
    return o


class Context:
    """A gs2d_ctx: the device's cache of instantiated fitting-chunk graphs."""

    def __init__(self, device=None):
        dev = torch.cuda.current_device() if device is None else int(device)
        h = c_void_p()
        _check("gs2d_ctx_create", lib().gs2d_ctx_create(ctypes.byref(h), dev))
        self.handle, self.device = h, dev

    def stats(self):
        """(graphs cached now, graphs instantiated so far)."""
        n, c = c_int32(), c_int64()
        _check("gs2d_ctx_stats", lib().gs2d_ctx_stats(self.handle, ctypes.byref(n), ctypes.byref(c)))
        return int(n.value), int(c.value)

    def close(self):
        if self.handle:
            lib().gs2d_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = {}


def default_context() -> Context:
    """One context per device for callers that pass none."""
    dev = torch.cuda.current_device()
    if dev not in _default_ctx:
        _default_ctx[dev] = Context(dev)
    return _default_ctx[dev]


def _fit_args(shape: Shape, target, xy, chol, rgb, m, v, step, loss_trace, ws):
    N, H, W = shape.N, shape.H, shape.W
    return (ctypes.byref(shape), _ptr(target, "target", shape=(3, H, W)),
            _ptr(xy, "xy", shape=(N, 2)), _ptr(chol, "chol", shape=(N, 3)),
            _ptr(rgb, "rgb", shape=(N, 3)), _ptr(m, "m", shape=(8 * N,)), _ptr(v, "v", shape=(8 * N,)),
            _ptr(step, "step", torch.int32, shape=(1,)), _ptr(loss_trace, "loss_trace"),
            int(loss_trace.numel()), _ptr(ws, "ws", torch.uint8), ws.numel())


def fit_frame(shape: Shape, target, xy, chol, rgb, m, v, step, loss_trace, ws, opts: FitOpts,
              check=True, ctx: Context | None = None) -> FitStats:
    """gs2d_fit_frame on the current stream; ctx defaults to the device's
    shared context (pass ctx=False for none)."""
    if ctx is None:
        ctx = default_context()
    stats = FitStats()
    code = lib().gs2d_fit_frame(
        ctx.handle if ctx else None,
        *_fit_args(shape, target, xy, chol, rgb, m, v, step, loss_trace, ws),
        ctypes.byref(opts), ctypes.byref(stats), _stream())
    if check:
        _check("gs2d_fit_frame", code)
    stats.code = code
    return stats


def ptq(xy, chol, rgb, bits_chol=6, bits_rgb=6, want_codes=False):
    """Post-training quantisation on the GPU.  Returns a dict of device
    tensors: xy, chol, rgb (dequantised), ranges [6, 2], bits [7] (float64:
    six components' entropy-coded bits, then the frame total) and, with
    want_codes, codes [N, 8] (int32 view of the uint16 codes)."""
    N = xy.shape[0]
    dev = xy.device
    ws = torch.empty(int(lib().gs2d_ptq_workspace_bytes(N)), dtype=torch.uint8, device=dev)
    out = {"xy": torch.empty(N, 2, device=dev), "chol": torch.empty(N, 3, device=dev),
           "rgb": torch.empty(N, 3, device=dev), "ranges": torch.empty(6, 2, device=dev),
           "bits": torch.empty(7, dtype=torch.float64, device=dev)}
    codes = torch.empty(N, 8, dtype=torch.int16, device=dev) if want_codes else None
    cfg = QuantCfg(int(bits_chol), int(bits_rgb))
    _check("gs2d_ptq", lib().gs2d_ptq(
        N, _ptr(xy, "xy", shape=(N, 2)), _ptr(chol, "chol", shape=(N, 3)),
        _ptr(rgb, "rgb", shape=(N, 3)), ctypes.byref(cfg), _ptr(out["xy"], "q_xy"),
        _ptr(out["chol"], "q_chol"), _ptr(out["rgb"], "q_rgb"),
        _ptr(codes, "codes", torch.int16, allow_none=True), _ptr(out["ranges"], "ranges"),
        _ptr(out["bits"], "bits", torch.float64), _ptr(ws, "ws", torch.uint8), ws.numel(),
        _stream()))
    if codes is not None:
        out["codes"] = codes.to(torch.int32) & 0xFFFF
    return out


def select_changed(shape: Shape, ws, xy, chol, frame, prev, tau, active=None, counts=None):
    """P-frame selection on the reference Gaussians binned in ws: fills
    active [N] uint8 (allocated if None); counts (int32 [2], optional) gets
    (changed pixels, selected Gaussians).  Returns active."""
    N, H, W = shape.N, shape.H, shape.W
    if active is None:
        active = torch.empty(N, dtype=torch.uint8, device=xy.device)
    _check("gs2d_select_changed", lib().gs2d_select_changed(
        ctypes.byref(shape), _ptr(ws, "ws", torch.uint8), ws.numel(),
        _ptr(xy, "xy", shape=(N, 2)), _ptr(chol, "chol", shape=(N, 3)),
        _ptr(frame, "frame", shape=(3, H, W)), _ptr(prev, "prev", shape=(3, H, W)), float(tau),
        _ptr(active, "active", torch.uint8, shape=(N,)),
        _ptr(counts, "counts", torch.int32, shape=(2,), allow_none=True), _stream()))
    return active


class FitCall:
    """gs2d_fit_frame with its arguments checked and marshalled once: a
    fitting loop called again and again with the same buffers (a video
    encoder, once per frame) pays only the library call each time.  The
    tensors must stay allocated and unresized, and keep the options, while
    the object is used; the call runs on the stream current at each call."""

    def __init__(self, shape: Shape, target, xy, chol, rgb, m, v, step, loss_trace, ws,
                 opts: FitOpts, ctx: Context | None = None):
        if ctx is None:
            ctx = default_context()
        self._keep = (shape, target, xy, chol, rgb, m, v, step, loss_trace, ws, opts, ctx)
        self._args = ((ctx.handle if ctx else None,)
                      + _fit_args(shape, target, xy, chol, rgb, m, v, step, loss_trace, ws)
                      + (ctypes.byref(opts),))

    def __call__(self, check=True) -> FitStats:
        stats = FitStats()
        code = lib().gs2d_fit_frame(*self._args, ctypes.byref(stats), _stream())
        if check:
            _check("gs2d_fit_frame", code)
        stats.code = code
        return stats


def fit_frame_static(shape: Shape, target, xy, chol, rgb, m, v, step, loss_trace, opts: FitOpts,
                     check=True) -> FitStats:
    """gs2d_fit_frame_static: the fitting loop with the library's own
    device-resident workspace (no allocation; shapes up to its size)."""
    N, H, W = shape.N, shape.H, shape.W
    stats = FitStats()
    code = lib().gs2d_fit_frame_static(
        ctypes.byref(shape), _ptr(target, "target", shape=(3, H, W)),
        _ptr(xy, "xy", shape=(N, 2)), _ptr(chol, "chol", shape=(N, 3)),
        _ptr(rgb, "rgb", shape=(N, 3)), _ptr(m, "m", shape=(8 * N,)), _ptr(v, "v", shape=(8 * N,)),
        _ptr(step, "step", torch.int32, shape=(1,)), _ptr(loss_trace, "loss_trace"),
        int(loss_trace.numel()), ctypes.byref(opts), ctypes.byref(stats), _stream())
    if check:
        _check("gs2d_fit_frame_static", code)
    stats.code = code
    return stats


def fit_prepare(shape: Shape, target, xy, chol, rgb, m, v, step, loss_trace, ws, opts: FitOpts,
                ctx: Context | None = None):
    """Instantiate the graphs fit_frame with these arguments will replay."""
    if ctx is None:
        ctx = default_context()
    _check("gs2d_fit_prepare", lib().gs2d_fit_prepare(
        ctx.handle, *_fit_args(shape, target, xy, chol, rgb, m, v, step, loss_trace, ws),
        ctypes.byref(opts)))


def autotune_frame(W, H, N, target, xy, chol, rgb, candidates, reps=5):
    """Time binning + fused raster for every (tile, px_per_lane) candidate on
    one frame; returns (best_index, [ms per round])."""
    shapes = [make_shape(W, H, N, t, px_per_lane=p) for t, p in candidates]
    need = max(workspace_bytes(s) for s in shapes)
    ws = torch.empty(need, dtype=torch.uint8, device=xy.device)
    scratch = torch.zeros(8 * N, device=xy.device)
    ct = (c_int32 * len(candidates))(*[int(t) for t, _ in candidates])
    cp = (c_int32 * len(candidates))(*[int(p) for _, p in candidates])
    out = (c_float * len(candidates))()
    best = c_int32(-1)
    _check("gs2d_autotune_frame", lib().gs2d_autotune_frame(
        int(W), int(H), int(N), _ptr(target, "target", shape=(3, H, W)),
        _ptr(xy, "xy", shape=(N, 2)), _ptr(chol, "chol", shape=(N, 3)),
        _ptr(rgb, "rgb", shape=(N, 3)), len(candidates), ct, cp, int(reps),
        _ptr(scratch, "scratch"), _ptr(ws, "ws", torch.uint8), ws.numel(), out,
        ctypes.byref(best), _stream()))
    return int(best.value), [float(x) for x in out]


def init_plain(target, roi_mask, pick_roi, jit_roi, pick_out, jit_out, ws=None, picked=None):
    """Content-aware ROI initialisation on the GPU.  Returns (xy, chol, rgb)."""
    H, W = int(target.shape[1]), int(target.shape[2])
    n_roi, n_out = int(pick_roi.shape[0]), int(pick_out.shape[0])
    N = n_roi + n_out
    need = int(lib().gs2d_init_workspace_bytes(W, H))
    if need == 0:
        raise GS2DError("gs2d_init_workspace_bytes", GS2D_EINVAL)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=target.device)
    xy = torch.empty(N, 2, device=target.device)
    chol = torch.empty(N, 3, device=target.device)
    rgb = torch.empty(N, 3, device=target.device)
    _check("gs2d_init_plain", lib().gs2d_init_plain(
        W, H, _ptr(target, "target", shape=(3, H, W)),
        _ptr(roi_mask, "roi_mask", torch.uint8, shape=(H, W)),
        n_roi, _ptr(pick_roi, "pick_roi", torch.int64, shape=(n_roi,), allow_none=n_roi == 0),
        _ptr(jit_roi, "jit_roi", shape=(n_roi, 2), allow_none=n_roi == 0),
        n_out, _ptr(pick_out, "pick_out", torch.int64, shape=(n_out,), allow_none=n_out == 0),
        _ptr(jit_out, "jit_out", shape=(n_out, 2), allow_none=n_out == 0),
        _ptr(xy, "xy"), _ptr(chol, "chol"), _ptr(rgb, "rgb"),
        _ptr(picked, "picked", torch.int32, shape=(N,), allow_none=True),
        _ptr(ws, "ws", torch.uint8), ws.numel(), _stream()))
    return xy, chol, rgb


def init_superpixel(target, roi_mask, seeds, xy, chol, rgb, iters=10, compactness=0.1,
                    ws=None, labels=None, centres=None):
    """Superpixel ROI initialisation on the GPU, in place: xy/chol/rgb [K]
    hold the Gaussians empty segments keep and receive the segment Gaussians.
    seeds [K] int32 pixel indices; labels [H, W] int32 and centres [2, 5, K]
    FP32 are optional outputs."""
    H, W = int(target.shape[1]), int(target.shape[2])
    K = int(seeds.shape[0])
    need = int(lib().gs2d_superpixel_workspace_bytes(W, H, K))
    if need == 0:
        raise GS2DError("gs2d_superpixel_workspace_bytes", GS2D_EINVAL)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=target.device)
    _check("gs2d_init_superpixel", lib().gs2d_init_superpixel(
        W, H, _ptr(target, "target", shape=(3, H, W)),
        _ptr(roi_mask, "roi_mask", torch.uint8, shape=(H, W)), K,
        _ptr(seeds, "seeds", torch.int32, shape=(K,)), int(iters), float(compactness),
        _ptr(xy, "xy", shape=(K, 2)), _ptr(chol, "chol", shape=(K, 3)),
        _ptr(rgb, "rgb", shape=(K, 3)),
        _ptr(labels, "labels", torch.int32, shape=(H, W), allow_none=True),
        _ptr(centres, "centres", shape=(2, 5, K), allow_none=True),
        _ptr(ws, "ws", torch.uint8), ws.numel(), _stream()))
    return xy, chol, rgb


# ------------------------------------------------------------------ batches --
def frames_array(sizes):
    """sizes: list of (W, H, N) -> ctypes array of Frame."""
    arr = (Frame * len(sizes))()
    for i, (w, h, n) in enumerate(sizes):
        arr[i] = Frame(int(w), int(h), int(n))
    return arr


def batch_workspace_bytes(sizes, tile=16, px_per_lane=1) -> int:
    fr = frames_array(sizes)
    n = lib().gs2d_batch_workspace_bytes(len(sizes), fr, int(tile), int(px_per_lane))
    if n == 0:
        raise GS2DError("gs2d_batch_workspace_bytes", GS2D_EINVAL)
    return int(n)


def _batch_totals(sizes):
    return sum(n for _, _, n in sizes), sum(3 * w * h for w, h, _ in sizes)


def fit_batch(sizes, tile, px_per_lane, targets, xy, chol, rgb, m, v, step, loss_trace, ws,
              opts: FitOpts, check=True, ctx: Context | None = None) -> FitStats:
    F = len(sizes)
    Nt, Pt = _batch_totals(sizes)
    if loss_trace.dim() != 2 or loss_trace.shape[1] != F:
        raise ValueError("loss_trace must be [rows, n_frames]")
    if ctx is None:
        ctx = default_context()
    stats = FitStats()
    code = lib().gs2d_fit_batch(
        ctx.handle if ctx else None, F, frames_array(sizes), int(tile), int(px_per_lane), _ptr(targets, "targets", shape=(Pt,)),
        _ptr(xy, "xy", shape=(Nt, 2)), _ptr(chol, "chol", shape=(Nt, 3)),
        _ptr(rgb, "rgb", shape=(Nt, 3)), _ptr(m, "m", shape=(8 * Nt,)), _ptr(v, "v", shape=(8 * Nt,)),
        _ptr(step, "step", torch.int32, shape=(1,)), _ptr(loss_trace, "loss_trace"),
        int(loss_trace.shape[0]), _ptr(ws, "ws", torch.uint8), ws.numel(), ctypes.byref(opts),
        ctypes.byref(stats), _stream())
    if check:
        _check("gs2d_fit_batch", code)
    stats.code = code
    return stats


def batch_render_grads(sizes, tile, px_per_lane, targets, xy, chol, rgb, g_xy, g_chol, g_rgb, ws,
                       loss_per_frame=None):
    F = len(sizes)
    Nt, Pt = _batch_totals(sizes)
    _check("gs2d_batch_render_grads", lib().gs2d_batch_render_grads(
        F, frames_array(sizes), int(tile), int(px_per_lane), _ptr(targets, "targets", shape=(Pt,)),
        _ptr(xy, "xy", shape=(Nt, 2)), _ptr(chol, "chol", shape=(Nt, 3)),
        _ptr(rgb, "rgb", shape=(Nt, 3)), _ptr(g_xy, "g_xy", shape=(Nt, 2)),
        _ptr(g_chol, "g_chol", shape=(Nt, 3)), _ptr(g_rgb, "g_rgb", shape=(Nt, 3)),
        _ptr(loss_per_frame, "loss_per_frame", shape=(F,), allow_none=True),
        _ptr(ws, "ws", torch.uint8), ws.numel(), _stream()))


def read_batch_bins(sizes, tile, px_per_lane, f, ws) -> dict:
    b = Bins()
    _check("gs2d_batch_bins_view", lib().gs2d_batch_bins_view(
        len(sizes), frames_array(sizes), int(tile), int(px_per_lane), int(f),
        _ptr(ws, "ws", torch.uint8), ws.numel(), ctypes.byref(b)))
    N = sizes[f][2]
    n_pairs = int(_slice(ws, b.n_pairs, 1, torch.int32).item())
    keys = _slice(ws, b.keys, n_pairs, torch.int32).cpu().numpy().view("uint32")
    return {"n_pairs": n_pairs, "keys": keys,
            "tile_start": _slice(ws, b.tile_start, b.n_tiles + 1, torch.int32).cpu().numpy().astype("int64"),
            "counts": _slice(ws, b.counts, N, torch.int32).cpu().numpy().astype("int64"),
            "geom": _slice(ws, b.geom, 8 * N, torch.float32).cpu().numpy().reshape(N, 8),
            "status": int(_slice(ws, b.status, 1, torch.int32).item())}


def autotune_batch(sizes, targets, xy, chol, rgb, candidates, reps=5):
    """Time every (tile, px_per_lane) candidate on this batch; returns
    (best_index, [ms per round])."""
    F = len(sizes)
    Nt, Pt = _batch_totals(sizes)
    need = max(batch_workspace_bytes(sizes, t, p) for t, p in candidates)
    ws = torch.empty(need, dtype=torch.uint8, device=xy.device)
    scratch = torch.zeros(8 * Nt, device=xy.device)
    ct = (c_int32 * len(candidates))(*[int(t) for t, _ in candidates])
    cp = (c_int32 * len(candidates))(*[int(p) for _, p in candidates])
    out = (c_float * len(candidates))()
    best = c_int32(-1)
    _check("gs2d_autotune_batch", lib().gs2d_autotune_batch(
        F, frames_array(sizes), _ptr(targets, "targets", shape=(Pt,)), _ptr(xy, "xy", shape=(Nt, 2)),
        _ptr(chol, "chol", shape=(Nt, 3)), _ptr(rgb, "rgb", shape=(Nt, 3)), len(candidates), ct, cp,
        int(reps), _ptr(scratch, "scratch"), _ptr(ws, "ws", torch.uint8), ws.numel(), out,
        ctypes.byref(best), _stream()))
    return int(best.value), [float(x) for x in out]


# -------------------------------------------------------- learned initialiser --
class CNNInit:
    """Device state of the per-tile regressor for H x W frames: FP32 master
    weights, their BF16 (and transposed BF16) copies, Adam moments, the
    activation workspace.  Every method is one or a few C ABI calls."""

    def __init__(self, H, W, seed=7, device="cuda"):
        from . import synth
        L = lib()
        self.H, self.W = int(H), int(W)
        self.n_params = int(L.gs2d_cnn_param_count(self.H, self.W))
        if self.n_params == 0:
            raise GS2DError("gs2d_cnn_param_count", GS2D_EINVAL)
        self.master = torch.zeros(self.n_params, device=device)
        draws = torch.from_numpy(synth.random_normal(self.n_params, seed)).to(device)
        _check("gs2d_cnn_init_params", L.gs2d_cnn_init_params(
            self.H, self.W, _ptr(draws, "draws"), _ptr(self.master, "master"), _stream()))
        self.wbf16 = torch.zeros(int(L.gs2d_cnn_bf16_weight_count(self.H, self.W)), dtype=torch.int16,
                                 device=device)
        self.sync()
        self.ws = torch.empty(int(L.gs2d_cnn_workspace_bytes(self.H, self.W)), dtype=torch.uint8,
                              device=device)
        self.grad = torch.zeros_like(self.master)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.step_count = torch.zeros(1, dtype=torch.int32, device=device)
        self.scratch = torch.empty(1 << 20, dtype=torch.uint8, device=device)
        self.loss3 = torch.zeros(3, device=device)
        hd = self.layer_info(4)
        self.TY, self.TX = hd["Hout"], hd["Wout"]

    def sync(self):
        _check("gs2d_cnn_sync_weights", lib().gs2d_cnn_sync_weights(
            self.H, self.W, _ptr(self.master, "master"), _ptr(self.wbf16, "wbf16", torch.int16),
            _stream()))

    def layer_info(self, i):
        info = (c_int32 * 12)()
        _check("gs2d_cnn_layer_info", lib().gs2d_cnn_layer_info(self.H, self.W, i, info))
        keys = ("Hin", "Win", "Cin", "Hout", "Wout", "Cout", "stride", "relu", "Mpad", "Kf",
                "w_off", "b_off")
        return dict(zip(keys, list(info)))

    def forward(self, frame, prev=None, head_out=None):
        _check("gs2d_cnn_forward", lib().gs2d_cnn_forward(
            self.H, self.W, _ptr(frame, "frame", shape=(3, self.H, self.W)),
            _ptr(prev, "prev", shape=(3, self.H, self.W), allow_none=True),
            _ptr(self.master, "master"), _ptr(self.wbf16, "wbf16", torch.int16),
            _ptr(head_out, "head_out", allow_none=True), _ptr(self.ws, "ws", torch.uint8),
            self.ws.numel(), _stream()))

    def set_targets(self, xy, chol, rgb):
        N = xy.shape[0]
        need = 2 * (((4 * N + 255) // 256) * 256) + (1 << 18) + 4 * (self.TX * self.TY + 1) + 4096
        if self.scratch.numel() < need:
            self.scratch = torch.empty(need, dtype=torch.uint8, device=xy.device)
        _check("gs2d_cnn_targets", lib().gs2d_cnn_targets(
            self.H, self.W, N, _ptr(xy, "xy", shape=(N, 2)), _ptr(chol, "chol", shape=(N, 3)),
            _ptr(rgb, "rgb", shape=(N, 3)), _ptr(self.ws, "ws", torch.uint8), self.ws.numel(),
            _ptr(self.scratch, "scratch", torch.uint8), self.scratch.numel(), _stream()))

    def read_targets(self):
        n = self.TX * self.TY
        counts = torch.zeros(n, dtype=torch.int32, device=self.ws.device)
        vec = torch.zeros(n, 8, 8, device=self.ws.device)
        _check("gs2d_cnn_read_targets", lib().gs2d_cnn_read_targets(
            self.H, self.W, _ptr(self.ws, "ws", torch.uint8), self.ws.numel(),
            _ptr(counts, "counts", torch.int32), _ptr(vec, "vec"), _stream()))
        return counts, vec

    def tensor(self, layer, which):
        """A copy of a layer tensor the last forward / backward pass left in
        the workspace (which = 0: the layer's BF16 input activations, 1: the
        BF16 gradient w.r.t. its output), as a float32 host array
        [channels][rows][columns] (all stored channels, padding included)."""
        import numpy as np
        ptr = c_void_p()
        dims = (c_int32 * 3)()
        _check("gs2d_cnn_tensor_view", lib().gs2d_cnn_tensor_view(
            self.H, self.W, int(layer), int(which), _ptr(self.ws, "ws", torch.uint8), self.ws.numel(),
            ctypes.byref(ptr), dims))
        rows, cols, ch = dims[0], dims[1], dims[2]
        raw = _slice(self.ws, ptr.value, rows * cols * ch, torch.int16).cpu().numpy()
        bits = raw.view(np.uint16).astype(np.uint32) << 16
        return bits.view(np.float32).reshape(rows, cols, ch).transpose(2, 0, 1).copy()

    def backward(self):
        """Head loss + full backward; gradients ADDED to self.grad (cleared by step)."""
        _check("gs2d_cnn_backward", lib().gs2d_cnn_backward(
            self.H, self.W, _ptr(self.master, "master"), _ptr(self.wbf16, "wbf16", torch.int16),
            _ptr(self.grad, "grad"), _ptr(self.loss3, "loss3"), _ptr(self.ws, "ws", torch.uint8),
            self.ws.numel(), _stream()))
        return self.loss3

    def step(self, lr=1e-3, weight_decay=0.0):
        _check("gs2d_cnn_adam", lib().gs2d_cnn_adam(
            self.H, self.W, _ptr(self.master, "master"), _ptr(self.grad, "grad"),
            _ptr(self.m, "m"), _ptr(self.v, "v"), _ptr(self.step_count, "step", torch.int32),
            float(lr), float(weight_decay), _ptr(self.wbf16, "wbf16", torch.int16), _stream()))

    def decode(self, N, plain_xy, plain_chol, plain_rgb):
        dev = plain_xy.device
        xy = torch.empty(N, 2, device=dev)
        chol = torch.empty(N, 3, device=dev)
        rgb = torch.empty(N, 3, device=dev)
        npred = torch.zeros(1, dtype=torch.int32, device=dev)
        _check("gs2d_cnn_decode", lib().gs2d_cnn_decode(
            self.H, self.W, int(N), _ptr(plain_xy, "plain_xy", shape=(N, 2)),
            _ptr(plain_chol, "plain_chol", shape=(N, 3)), _ptr(plain_rgb, "plain_rgb", shape=(N, 3)),
            _ptr(xy, "xy"), _ptr(chol, "chol"), _ptr(rgb, "rgb"), _ptr(npred, "npred", torch.int32),
            _ptr(self.ws, "ws", torch.uint8), self.ws.numel(),
            _ptr(self.scratch, "scratch", torch.uint8), self.scratch.numel(), _stream()))
        return xy, chol, rgb, npred

    def pframe_replace(self, frame, prev, tau, xy, chol, rgb, head=None, tile_sel=None,
                       stats=None):
        """Replace, in place, the warm-started Gaussians of the tiles whose
        mean squared residual exceeds tau by the predictions of `head` (None:
        the last forward's).  Returns the device int32 stats [4] (selected
        tiles, freed, predicted, replaced)."""
        N = int(xy.shape[0])
        dev = xy.device
        need = int(lib().gs2d_cnn_pframe_scratch_bytes(self.H, self.W, N))
        if need == 0:
            raise GS2DError("gs2d_cnn_pframe_scratch_bytes", GS2D_EINVAL)
        if self.scratch.numel() < need:
            self.scratch = torch.empty(need, dtype=torch.uint8, device=dev)
        if stats is None:
            stats = torch.zeros(4, dtype=torch.int32, device=dev)
        _check("gs2d_cnn_pframe_replace", lib().gs2d_cnn_pframe_replace(
            self.H, self.W, N, _ptr(frame, "frame", shape=(3, self.H, self.W)),
            _ptr(prev, "prev", shape=(3, self.H, self.W)), float(tau),
            _ptr(head, "head", shape=(73, self.TY, self.TX), allow_none=True),
            _ptr(xy, "xy", shape=(N, 2)), _ptr(chol, "chol", shape=(N, 3)),
            _ptr(rgb, "rgb", shape=(N, 3)), _ptr(stats, "stats", torch.int32, shape=(4,)),
            _ptr(tile_sel, "tile_sel", torch.uint8, shape=(self.TY, self.TX), allow_none=True),
            _ptr(self.ws, "ws", torch.uint8), self.ws.numel(),
            _ptr(self.scratch, "scratch", torch.uint8), self.scratch.numel(), _stream()))
        return stats

    def oracle_params(self):
        """Master weights as a list of (w [Cout, Cin, 3, 3], b [Cout]) numpy
        arrays in the oracle's layout (input layer: 6 real channels)."""
        import numpy as np
        mw = self.master.detach().cpu().numpy()
        out = []
        for i in range(5):
            d = self.layer_info(i)
            cin_real = 6 if i == 0 else d["Cin"]
            M = mw[d["w_off"]:d["w_off"] + d["Mpad"] * d["Kf"]].reshape(d["Mpad"], d["Kf"])
            w = np.zeros((d["Cout"], cin_real, 3, 3), np.float32)
            for tap in range(9):
                w[:, :, tap // 3, tap % 3] = M[:d["Cout"], tap * d["Cin"]:tap * d["Cin"] + cin_real]
            b = mw[d["b_off"]:d["b_off"] + d["Cout"]].copy()
            out.append((w, b))
        return out

    def oracle_grads(self):
        import numpy as np
        gw = self.grad.detach().cpu().numpy()
        out = []
        for i in range(5):
            d = self.layer_info(i)
            cin_real = 6 if i == 0 else d["Cin"]
            M = gw[d["w_off"]:d["w_off"] + d["Mpad"] * d["Kf"]].reshape(d["Mpad"], d["Kf"])
            w = np.zeros((d["Cout"], cin_real, 3, 3), np.float32)
            for tap in range(9):
                w[:, :, tap // 3, tap % 3] = M[:d["Cout"], tap * d["Cin"]:tap * d["Cin"] + cin_real]
            out.append((w, gw[d["b_off"]:d["b_off"] + d["Cout"]].copy()))
        return out
