// C ABI of the frame fitter: argument validation, workspace carving and the
// host side of the fitting loop (chunked, optionally replayed from hipGraphs
// cached in a gs2d_ctx, with a PSNR stop rule checked between chunks).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "bin_common.h"
#include "gs2d_internal.h"

namespace gs2d {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool make_layout(const gs2d_shape &s, Layout *L) {
  if (s.W < 1 || s.H < 1 || s.N < 1 || s.N > 65536) return false;
  if (s.tile != 8 && s.tile != 16 && s.tile != 32) return false;
  if (s.max_pairs < 1 || s.max_pairs > (1 << 30)) return false;
  const int ppl = s.px_per_lane == 0 ? 1 : s.px_per_lane;
  if (ppl != 1 && ppl != 2 && ppl != 4) return false;
  if (8 * ppl > s.tile) return false;
  const long long TX = (s.W + (long long)s.tile - 1) / s.tile;
  const long long TY = (s.H + (long long)s.tile - 1) / s.tile;
  if (TX * TY > 65536) return false;
  L->W = s.W;
  L->H = s.H;
  L->N = s.N;
  L->T = s.tile;
  L->max_pairs = s.max_pairs;
  L->ppl = ppl;
  L->TX = (int)TX;
  L->TY = (int)TY;
  L->n_tiles = (int)(TX * TY);
  int bits = 1;
  while ((1LL << bits) < (long long)L->n_tiles) ++bits;
  // at most 2048 tiles: one pass on the whole tile index, else 8-bit passes
  L->wide = L->n_tiles <= 2048;
  L->digit_bits = bits < 8 ? 8 : bits;
  L->D = 1 << L->digit_bits;
  L->sort_passes = L->wide ? 1 : (bits + RADIX_BITS - 1) / RADIX_BITS;
  // about one sort chunk per 256 Gaussians (chunks hold ~3 keys per Gaussian)
  const int G = (s.N + 255) / 256;
  L->sort_blocks = G > SORT_MAX_BLOCKS ? SORT_MAX_BLOCKS : G;
  size_t o = 0;
  auto take = [&o](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  const size_t N = (size_t)s.N;
  L->geom = take(N * 32);
  L->rect = take(N * 16);
  L->brect = take(N * 16);  // lazy binning: the rectangles the lists were built from
  L->counts = take(N * 4);
  L->offsets = take((N + 1) * 4);
  L->blocks = take(2048);  // per-projection-block sums (<= 256 blocks): pairs, culled
  L->keys_a = take((size_t)s.max_pairs * 4);
  L->keys_b = take((size_t)s.max_pairs * 4);
  // radix histogram rows: one per emission block (<= 256 rows of 256 words,
  // or <= 64 rows of up to 2048 words on the single-pass path), then one
  // per sort chunk of the second pass (<= 128 rows of 256 words)
  L->hist = take(HIST_BYTES);
  L->tile_start = take(((size_t)L->n_tiles + 1) * 4);
  L->loss_parts = L->n_tiles * (s.tile / 8) * (s.tile / (8 * ppl));
  L->loss_part = take((size_t)L->loss_parts * 4);
  L->grads = take(N * 8 * 4);
  L->qparams = take(N * 8 * 4);               // quantised xy | chol | rgb (QAT)
  L->qws = take(quantise_workspace_bytes(s.N));
  L->misc = take(MISC_COUNT * 4);
  L->total = o;
  // FNV-1a over the shape and the buffer offsets: the lazy lists' stamp
  uint64_t h = 1469598103934665603ull;
  const uint64_t words[] = {(uint64_t)L->W,        (uint64_t)L->H,         (uint64_t)L->N,
                            (uint64_t)L->T,        (uint64_t)L->max_pairs, (uint64_t)L->ppl,
                            (uint64_t)L->geom,     (uint64_t)L->brect,     (uint64_t)L->keys_a,
                            (uint64_t)L->keys_b,   (uint64_t)L->tile_start, (uint64_t)L->misc,
                            (uint64_t)L->total};
  for (uint64_t w : words)
    for (int b = 0; b < 8; ++b) {
      h ^= (w >> (8 * b)) & 0xFF;
      h *= 1099511628211ull;
    }
  L->sig_lo = (uint32_t)h;
  L->sig_hi = (uint32_t)(h >> 32);
  if (L->sig_lo == 0 && L->sig_hi == 0) L->sig_lo = 1;
  return true;
}

}  // namespace gs2d

using namespace gs2d;

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? GS2D_OK : GS2D_EHIP; }

int check_ws(const gs2d_shape *shape, void *ws, size_t ws_bytes, Layout *L) {
  if (!shape || !make_layout(*shape, L)) return GS2D_EINVAL;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return GS2D_EINVAL;
  if (ws_bytes < L->total) return GS2D_ENOSPACE;
  return GS2D_OK;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

extern "C" {

const char *gs2d_status_str(int status) {
  switch (status) {
    case GS2D_OK: return "ok";
    case GS2D_EINVAL: return "invalid argument";
    case GS2D_ENOSPACE: return "workspace too small";
    case GS2D_EOVERFLOW: return "tile-pair capacity exceeded";
    case GS2D_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

size_t gs2d_workspace_bytes(const gs2d_shape *shape) {
  Layout L;
  if (!shape || !make_layout(*shape, &L)) return 0;
  return L.total;
}

int gs2d_bins_view(const gs2d_shape *shape, void *ws, size_t ws_bytes, gs2d_bins *out) {
  Layout L;
  const int rc = check_ws(shape, ws, ws_bytes, &L);
  if (rc != GS2D_OK) return rc;
  if (!out) return GS2D_EINVAL;
  out->geom = at<const float>(ws, L.geom);
  out->counts = at<const int32_t>(ws, L.counts);
  out->offsets = at<const int32_t>(ws, L.offsets);
  out->keys = at<const uint32_t>(ws, L.keys_sorted());
  out->tile_start = at<const int32_t>(ws, L.tile_start);
  out->n_pairs = at<const int32_t>(ws, L.misc) + MISC_N_PAIRS;
  out->status = reinterpret_cast<const uint32_t *>(at<const int32_t>(ws, L.misc) + MISC_STATUS);
  out->n_culled = at<const int32_t>(ws, L.misc) + MISC_N_CULLED;
  out->n_tiles = L.n_tiles;
  out->tiles_x = L.TX;
  out->tiles_y = L.TY;
  return GS2D_OK;
}

int gs2d_project_bin(const gs2d_shape *shape, const float *xy, const float *chol, void *ws,
                     size_t ws_bytes, void *stream) {
  try {
    Layout L;
    const int rc = check_ws(shape, ws, ws_bytes, &L);
    if (rc != GS2D_OK) return rc;
    if (!xy || !chol) return GS2D_EINVAL;
    return hip_status(launch_binning(L, xy, chol, ws, as_stream(stream)));
  } catch (...) {
    return GS2D_EHIP;
  }
}

int gs2d_render_fwd(const gs2d_shape *shape, void *ws, size_t ws_bytes, const float *rgb,
                    const float *target, float *img, float *dl_dimg, float *loss, void *stream) {
  try {
    Layout L;
    const int rc = check_ws(shape, ws, ws_bytes, &L);
    if (rc != GS2D_OK) return rc;
    if (!rgb) return GS2D_EINVAL;
    if (!target && (dl_dimg || loss)) return GS2D_EINVAL;
    hipStream_t st = as_stream(stream);
    hipError_t e = launch_render_fwd(L, ws, rgb, target, img, dl_dimg, st);
    if (e == hipSuccess && loss) e = launch_loss_reduce(L, ws, loss, st);
    return hip_status(e);
  } catch (...) {
    return GS2D_EHIP;
  }
}

int gs2d_render_bwd(const gs2d_shape *shape, void *ws, size_t ws_bytes, const float *rgb,
                    const float *dl_dimg, float *g_xy, float *g_chol, float *g_rgb, void *stream) {
  try {
    Layout L;
    const int rc = check_ws(shape, ws, ws_bytes, &L);
    if (rc != GS2D_OK) return rc;
    if (!rgb || !dl_dimg || !g_xy || !g_chol || !g_rgb) return GS2D_EINVAL;
    hipStream_t st = as_stream(stream);
    const size_t N = (size_t)L.N;
    hipError_t e = launch_fill_zero(g_xy, 2 * N, st);
    if (e == hipSuccess) e = launch_fill_zero(g_chol, 3 * N, st);
    if (e == hipSuccess) e = launch_fill_zero(g_rgb, 3 * N, st);
    if (e == hipSuccess) e = launch_render_bwd(L, ws, rgb, dl_dimg, g_xy, g_chol, g_rgb, st);
    return hip_status(e);
  } catch (...) {
    return GS2D_EHIP;
  }
}

int gs2d_render_fused(const gs2d_shape *shape, void *ws, size_t ws_bytes, const float *rgb,
                      const float *target, float *g_xy, float *g_chol, float *g_rgb, float *loss,
                      void *stream) {
  try {
    Layout L;
    const int rc = check_ws(shape, ws, ws_bytes, &L);
    if (rc != GS2D_OK) return rc;
    if (!rgb || !target || !g_xy || !g_chol || !g_rgb) return GS2D_EINVAL;
    hipStream_t st = as_stream(stream);
    hipError_t e = launch_render_fused(L, ws, rgb, target, g_xy, g_chol, g_rgb, st);
    if (e == hipSuccess && loss) e = launch_loss_reduce(L, ws, loss, st);
    return hip_status(e);
  } catch (...) {
    return GS2D_EHIP;
  }
}

int gs2d_count_pairs(const gs2d_shape *shape, void *ws, size_t ws_bytes, uint64_t *out,
                     void *stream) {
  try {
    Layout L;
    const int rc = check_ws(shape, ws, ws_bytes, &L);
    if (rc != GS2D_OK) return rc;
    if (!out || (reinterpret_cast<uintptr_t>(out) & 7)) return GS2D_EINVAL;
    return hip_status(launch_count_pairs(L, ws, reinterpret_cast<unsigned long long *>(out),
                                         as_stream(stream)));
  } catch (...) {
    return GS2D_EHIP;
  }
}

int gs2d_adam_step(int32_t N, float *xy, float *chol, float *rgb, float *g_xy, float *g_chol,
                   float *g_rgb, float *m, float *v, int32_t *step, const gs2d_adam_cfg *cfg,
                   const uint8_t *active, int32_t zero_grads, void *stream) {
  try {
    if (N < 1 || !xy || !chol || !rgb || !g_xy || !g_chol || !g_rgb || !m || !v || !step || !cfg)
      return GS2D_EINVAL;
    hipStream_t st = as_stream(stream);
    hipError_t e = launch_step_tick(step, st);
    if (e == hipSuccess)
      e = launch_adam(N, xy, chol, rgb, g_xy, g_chol, g_rgb, m, v, step, *cfg, active, zero_grads,
                      nullptr, 0, 0.f, nullptr, 0, st);
    return hip_status(e);
  } catch (...) {
    return GS2D_EHIP;
  }
}

}  // extern "C"

namespace {

// k fitting iterations: binning, fused render/loss/backward and Adam (which
// clears the gradients and records the iteration's loss) each.  The Adam
// step of iteration i < k - 1 runs inside the first binning kernel of
// iteration i + 1; the last one runs on its own, so that after the k
// iterations the parameters, moments, step count and loss trace are those
// of k complete steps.
hipError_t enqueue_iterations(const Layout &L, void *ws, const float *target, float *xy,
                              float *chol, float *rgb, float *m, float *v, int32_t *step,
                              float *trace, int trace_len, const gs2d_adam_cfg &cfg,
                              const uint8_t *active, int k, hipStream_t st, int qat_bits_chol = 0,
                              int qat_bits_rgb = 0, float bin_skin = 0.f) {
  float *g = at<float>(ws, L.grads);
  float *g_xy = g, *g_chol = g + 2 * (size_t)L.N, *g_rgb = g + 5 * (size_t)L.N;
  const float loss_scale = (float)(1.0 / (3.0 * L.W * (double)L.H));
  // lazy binning on the single-pass path (fit_frame_run forces a rebuild at
  // the start of a call unless the workspace holds complete lists of this
  // layout)
  const float skin = (L.wide && bin_skin > 0.f) ? bin_skin : 0.f;
  if (qat_bits_chol > 0) {
    // quantisation-aware: quantise, bin and render the quantised copy, then
    // Adam on the FP32 parameters with its gradients (straight through); the
    // lazy lists follow the quantised Gaussians (the raster ticks the step)
    float *q = at<float>(ws, L.qparams);
    float *q_xy = q, *q_chol = q + 2 * (size_t)L.N, *q_rgb = q + 5 * (size_t)L.N;
    hipError_t e = hipSuccess;
    for (int i = 0; i < k && e == hipSuccess; ++i) {
      e = launch_quantise(L.N, xy, chol, rgb, qat_bits_chol, qat_bits_rgb, q_xy, q_chol, q_rgb,
                          nullptr, nullptr, nullptr, at<void>(ws, L.qws), st);
      if (e == hipSuccess) e = launch_binning(L, q_xy, q_chol, ws, st, step, nullptr, skin);
      if (e == hipSuccess)
        e = launch_render_fused(L, ws, q_rgb, target, g_xy, g_chol, g_rgb, st, active, skin > 0.f,
                                skin > 0.f ? step : nullptr);
      if (e == hipSuccess)
        e = launch_adam(L.N, xy, chol, rgb, g_xy, g_chol, g_rgb, m, v, step, cfg, active, 1,
                        at<const float>(ws, L.loss_part), L.loss_parts, loss_scale, trace,
                        trace_len, st, at<int32_t>(ws, L.misc) + MISC_STEP);
    }
    return e;
  }
  const PendingAdam pending{xy,    chol, rgb,  g_xy, g_chol, g_rgb, m,         v,
                            step,  cfg,  at<const float>(ws, L.loss_part), L.loss_parts,
                            loss_scale, trace, trace_len, active};
  hipError_t e = hipSuccess;
  for (int i = 0; i < k && e == hipSuccess; ++i) {
    e = launch_binning(L, xy, chol, ws, st, step, i > 0 ? &pending : nullptr, skin);
    if (e == hipSuccess)
      e = launch_render_fused(L, ws, rgb, target, g_xy, g_chol, g_rgb, st, active, skin > 0.f,
                              skin > 0.f ? step : nullptr);
  }
  if (e == hipSuccess && k > 0)
    e = launch_adam(L.N, xy, chol, rgb, g_xy, g_chol, g_rgb, m, v, step, cfg, active, 1,
                    at<const float>(ws, L.loss_part), L.loss_parts, loss_scale, trace, trace_len,
                    st, at<int32_t>(ws, L.misc) + MISC_STEP);
  return e;
}

// The start of a fitting call (launch_fit_begin) on the call's workspace.
hipError_t enqueue_fit_begin(const Layout &L, const FitArgs &a, hipStream_t st) {
  return launch_fit_begin(at<int32_t>(a.ws, L.misc), at<float>(a.ws, L.grads), 8 * (size_t)L.N,
                          L.wide && a.bin_skin > 0.f, L.sig_lo, L.sig_hi, st);
}

GraphKey frame_chunk_key(const Layout &L, const FitArgs &a, int k, bool first) {
  GraphKey key{1,
               (uint64_t)L.W,
               (uint64_t)L.H,
               (uint64_t)L.N,
               (uint64_t)L.T,
               (uint64_t)L.max_pairs,
               (uint64_t)L.ppl,
               key_word(a.target),
               key_word(a.xy),
               key_word(a.chol),
               key_word(a.rgb),
               key_word(a.m),
               key_word(a.v),
               key_word(a.step),
               key_word(a.trace),
               (uint64_t)a.trace_len,
               key_word(a.ws),
               key_word(a.active),
               (uint64_t)a.qat_bits_chol,
               (uint64_t)a.qat_bits_rgb,
               key_word(a.bin_skin),
               (uint64_t)k};
  for (float f : a.cfg.lr) key.push_back(key_word(f));
  key.push_back(key_word(a.cfg.beta1));
  key.push_back(key_word(a.cfg.beta2));
  key.push_back(key_word(a.cfg.eps));
  key.push_back(first ? 1 : 0);
  return key;
}

// Enqueue a chunk of k iterations on `st`: the context's cached graph when
// graphs are used, else direct launches.
int run_chunk(gs2d_ctx *ctx, bool use_graph, const Layout &L, const FitArgs &a, int k,
              hipStream_t st, bool launch, bool first) {
  // the call's first chunk starts with launch_fit_begin (in its graph: the
  // call's first submission is then the graph launch alone)
  auto enqueue = [&](hipStream_t s) {
    hipError_t e = first ? enqueue_fit_begin(L, a, s) : hipSuccess;
    if (e == hipSuccess)
      e = enqueue_iterations(L, a.ws, a.target, a.xy, a.chol, a.rgb, a.m, a.v, a.step, a.trace,
                             a.trace_len, a.cfg, a.active, k, s, a.qat_bits_chol, a.qat_bits_rgb,
                             a.bin_skin);
    return e;
  };
  if (!use_graph) return launch ? hip_status(enqueue(st)) : GS2D_OK;
  hipGraphExec_t x = nullptr;
  hipError_t e = ctx->graph_for(frame_chunk_key(L, a, k, first), enqueue, &x);
  if (e == hipSuccess && launch) e = hipGraphLaunch(x, st);
  return hip_status(e);
}

int check_fit_args(gs2d_ctx *ctx, const gs2d_shape *shape, const float *target, float *xy,
                   float *chol, float *rgb, float *m, float *v, int32_t *step, float *loss_trace,
                   void *ws, size_t ws_bytes, const gs2d_fit_opts *opts, Layout *L) {
  int rc = check_ws(shape, ws, ws_bytes, L);
  if (rc != GS2D_OK) return rc;
  if (!target || !xy || !chol || !rgb || !m || !v || !step || !loss_trace || !opts)
    return GS2D_EINVAL;
  if (opts->iters < 0 || opts->check_every < 1) return GS2D_EINVAL;
  if (opts->qat && (opts->qat->bits_chol < 1 || opts->qat->bits_chol > 12 ||
                    opts->qat->bits_rgb < 1 || opts->qat->bits_rgb > 12))
    return GS2D_EINVAL;
  if (!(opts->bin_skin >= 0.f && opts->bin_skin <= 64.f)) return GS2D_EINVAL;
  return gs2d_ctx_check(ctx);
}

}  // namespace

extern "C" int gs2d_fit_prepare(gs2d_ctx *ctx, const gs2d_shape *shape, const float *target,
                                float *xy, float *chol, float *rgb, float *m, float *v,
                                int32_t *step, float *loss_trace, int32_t trace_len, void *ws,
                                size_t ws_bytes, const gs2d_fit_opts *opts) {
  try {
    Layout L;
    if (!ctx) return GS2D_EINVAL;
    int rc = check_fit_args(ctx, shape, target, xy, chol, rgb, m, v, step, loss_trace, ws,
                            ws_bytes, opts, &L);
    if (rc != GS2D_OK) return rc;
    if (!opts->use_graph || opts->iters == 0) return GS2D_OK;
    const FitArgs a{target,       xy,
                    chol,         rgb,
                    m,            v,
                    step,         loss_trace,
                    trace_len,    ws,
                    opts->adam,   opts->active,
                    opts->qat ? opts->qat->bits_chol : 0,
                    opts->qat ? opts->qat->bits_rgb : 0,
                    opts->bin_skin};
    // the first chunk (with the call's start), the full chunks after it
    // and the last, shorter one
    const int k0 = std::min(opts->check_every, opts->iters);
    rc = run_chunk(ctx, true, L, a, k0, nullptr, false, true);
    if (rc == GS2D_OK && opts->iters >= 2 * opts->check_every)
      rc = run_chunk(ctx, true, L, a, k0, nullptr, false, false);
    const int rem = opts->iters % opts->check_every;
    if (rc == GS2D_OK && opts->iters > opts->check_every && rem != 0)
      rc = run_chunk(ctx, true, L, a, rem, nullptr, false, false);
    return rc;
  } catch (...) {
    return GS2D_EHIP;
  }
}

namespace gs2d {

int fit_frame_run(gs2d_ctx *ctx, const Layout &L, const FitArgs &a, const gs2d_fit_opts &opts,
                  gs2d_fit_stats *stats, hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  if (stats) {
    stats->iters_run = 0;
    stats->iter_hit_target = -1;
    stats->final_loss = NAN;
    stats->final_psnr = NAN;
    stats->seconds = 0.0;
    stats->status = 0;
    stats->n_culled = 0;
    stats->rebins = 0;
  }
  // Without a PSNR target nothing is read back until the end: the step count
  // the loop's last Adam step reports gives step[0] at the start, and the
  // trace bound is checked then (the kernels write no entry past trace_len).
  const bool at_end = !(opts.psnr_target > 0.f) && opts.iters > 0;
  int32_t step0 = 0;
  if (!at_end) {
    if (hipMemcpyAsync(&step0, a.step, sizeof(int32_t), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return GS2D_EHIP;
    if (step0 < 0 || (long long)step0 + opts.iters >= (long long)a.trace_len) return GS2D_EINVAL;
  }

  // without a context the call's graphs live until it returns
  gs2d_ctx local;
  gs2d_ctx *cx = ctx ? ctx : &local;
  const bool use_graph = opts.use_graph != 0;
  int32_t *misc = at<int32_t>(a.ws, L.misc);
  // misc and the gradients cleared, lazy lists rebuilt at the call's first
  // iteration unless the workspace holds complete lists of this layout:
  // at the head of the first chunk (a call without iterations runs it alone)
  if (opts.iters == 0 && enqueue_fit_begin(L, a, st) != hipSuccess) return GS2D_EHIP;

  constexpr int TRACE_PIECE = 256;  // loss values read back per copy
  float trace_host[TRACE_PIECE];
  int32_t misc_local[gs2d_ctx::HOST_MISC_WORDS] = {};
  // the context's pinned copy when there is one (an asynchronous read-back)
  int32_t *misc_host = (ctx && ctx->host_misc) ? ctx->host_misc : misc_local;
  constexpr size_t MISC_BYTES = gs2d_ctx::HOST_MISC_WORDS * sizeof(int32_t);
  std::memset(misc_host, 0, MISC_BYTES);  // no copy in flight: every call waits for its own
  int done = 0, hit = -1;
  float last_loss = NAN;
  uint32_t sticky = 0;
  bool bad_trace = false;
  if (at_end) {
    // no early stop to check: every chunk back to back, one wait at the end
    while (done < opts.iters) {
      const int k = std::min(opts.check_every, opts.iters - done);
      const int rc = run_chunk(cx, use_graph, L, a, k, st, true, done == 0);
      if (rc != GS2D_OK) return rc;
      done += k;
    }
    if (hipMemcpyAsync(misc_host, misc, MISC_BYTES, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return GS2D_EHIP;
    sticky = (uint32_t)misc_host[MISC_STICKY];
    std::memcpy(&last_loss, &misc_host[MISC_LAST_LOSS], sizeof(float));
    step0 = misc_host[MISC_STEP] - opts.iters;
    bad_trace = step0 < 0 || misc_host[MISC_STEP] >= a.trace_len;
  }
  while (done < opts.iters) {
    const int k = std::min(opts.check_every, opts.iters - done);
    int rc = run_chunk(cx, use_graph, L, a, k, st, true, done == 0);
    if (rc != GS2D_OK) return rc;
    if (hipMemcpyAsync(misc_host, misc, MISC_BYTES, hipMemcpyDeviceToHost, st) !=
        hipSuccess)
      return GS2D_EHIP;
    for (int i0 = 0; i0 < k; i0 += TRACE_PIECE) {
      const int n = std::min(TRACE_PIECE, k - i0);
      if (hipMemcpyAsync(trace_host, a.trace + step0 + done + i0, sizeof(float) * n,
                         hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return GS2D_EHIP;
      for (int i = 0; i < n; ++i) {
        last_loss = trace_host[i];
        if (hit < 0 && opts.psnr_target > 0.f && last_loss > 0.f &&
            10.0 * std::log10(1.0 / last_loss) >= opts.psnr_target)
          hit = done + i0 + i;
      }
    }
    sticky = (uint32_t)misc_host[MISC_STICKY];
    done += k;
    if (sticky & (STATUS_OVERFLOW | STATUS_STALLED)) break;
    if (hit >= 0) break;
  }
  if (stats) {
    stats->iters_run = done;
    stats->iter_hit_target = hit;
    stats->final_loss = last_loss;
    stats->final_psnr = (last_loss > 0.f) ? (float)(10.0 * std::log10(1.0 / last_loss)) : INFINITY;
    stats->status = sticky;
    stats->n_culled = misc_host[MISC_N_CULLED];
    stats->rebins = misc_host[MISC_REBINS];
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (bad_trace) return GS2D_EINVAL;
  if (sticky & STATUS_STALLED) return GS2D_EHIP;  // a device-side wait ran out
  return (sticky & STATUS_OVERFLOW) ? GS2D_EOVERFLOW : GS2D_OK;
}

}  // namespace gs2d

extern "C" int gs2d_fit_frame(gs2d_ctx *ctx, const gs2d_shape *shape, const float *target,
                              float *xy, float *chol, float *rgb, float *m, float *v,
                              int32_t *step, float *loss_trace, int32_t trace_len, void *ws,
                              size_t ws_bytes, const gs2d_fit_opts *opts, gs2d_fit_stats *stats,
                              void *stream) {
  try {
    Layout L;
    const int rc = check_fit_args(ctx, shape, target, xy, chol, rgb, m, v, step, loss_trace, ws,
                                  ws_bytes, opts, &L);
    if (rc != GS2D_OK) return rc;
    const FitArgs a{target,       xy,
                    chol,         rgb,
                    m,            v,
                    step,         loss_trace,
                    trace_len,    ws,
                    opts->adam,   opts->active,
                    opts->qat ? opts->qat->bits_chol : 0,
                    opts->qat ? opts->qat->bits_rgb : 0,
                    opts->bin_skin};
    return fit_frame_run(ctx, L, a, *opts, stats, as_stream(stream));
  } catch (...) {
    return GS2D_EHIP;
  }
}

// One-frame autotuner: for each candidate (tile, px_per_lane) the binning
// and the fused raster that gs2d_fit_frame runs per iteration, timed with
// HIP events over `reps` rounds after one untimed round.
extern "C" int gs2d_autotune_frame(int32_t W, int32_t H, int32_t N, const float *target,
                                   const float *xy, const float *chol, const float *rgb,
                                   int32_t n_cand, const int32_t *cand_tile,
                                   const int32_t *cand_ppl, int32_t reps, float *grad_scratch,
                                   void *ws, size_t ws_bytes, float *out_ms, int32_t *best,
                                   void *stream) {
  struct Events {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Events() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  };
  try {
    if (n_cand < 1 || !cand_tile || !cand_ppl || reps < 1 || !out_ms || !best || !grad_scratch ||
        !target || !xy || !chol || !rgb)
      return GS2D_EINVAL;
    hipStream_t st = as_stream(stream);
    Events E;
    if (hipEventCreate(&E.e0) != hipSuccess || hipEventCreate(&E.e1) != hipSuccess)
      return GS2D_EHIP;
    float best_ms = INFINITY;
    *best = -1;
    for (int c = 0; c < n_cand; ++c) {
      gs2d_shape s{W, H, N, cand_tile[c], 0, cand_ppl[c]};
      if (s.tile != 8 && s.tile != 16 && s.tile != 32) return GS2D_EINVAL;
      const long long tiles =
          (long long)((W + s.tile - 1) / s.tile) * (long long)((H + s.tile - 1) / s.tile);
      s.max_pairs = (int32_t)std::min<long long>(1LL << 30,
                                                 std::max<long long>(65536, 16LL * N + 4 * tiles));
      Layout L;
      const int rc = check_ws(&s, ws, ws_bytes, &L);
      if (rc != GS2D_OK) return rc;
      float *g_xy = grad_scratch, *g_chol = g_xy + 2 * (size_t)N, *g_rgb = g_xy + 5 * (size_t)N;
      hipError_t e = hipSuccess;
      for (int r = 0; r <= reps && e == hipSuccess; ++r) {
        if (r == 1) e = hipEventRecord(E.e0, st);
        if (e == hipSuccess) e = launch_binning(L, xy, chol, ws, st);
        if (e == hipSuccess) e = launch_render_fused(L, ws, rgb, target, g_xy, g_chol, g_rgb, st);
      }
      if (e == hipSuccess) e = hipEventRecord(E.e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(E.e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, E.e0, E.e1);
      if (e != hipSuccess) return GS2D_EHIP;
      out_ms[c] = ms / reps;
      if (out_ms[c] < best_ms) {
        best_ms = out_ms[c];
        *best = c;
      }
    }
    return GS2D_OK;
  } catch (...) {
    return GS2D_EHIP;
  }
}
