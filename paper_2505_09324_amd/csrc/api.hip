// C ABI of the frame fitter: argument validation, workspace carving and the
// host side of the fitting loop (chunked, optionally replayed from a
// captured hipGraph, with a PSNR stop rule checked between chunks).
#include <chrono>
#include <cmath>
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
  L->misc = take(MISC_COUNT * 4);
  L->total = o;
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
                              float *trace, int trace_len, const gs2d_adam_cfg &cfg, int k,
                              hipStream_t st) {
  float *g = at<float>(ws, L.grads);
  float *g_xy = g, *g_chol = g + 2 * (size_t)L.N, *g_rgb = g + 5 * (size_t)L.N;
  const float loss_scale = (float)(1.0 / (3.0 * L.W * (double)L.H));
  const PendingAdam pending{xy,    chol, rgb,  g_xy, g_chol, g_rgb, m,         v,
                            step,  cfg,  at<const float>(ws, L.loss_part), L.loss_parts,
                            loss_scale, trace, trace_len};
  hipError_t e = hipSuccess;
  for (int i = 0; i < k && e == hipSuccess; ++i) {
    e = launch_binning(L, xy, chol, ws, st, step, i > 0 ? &pending : nullptr);
    if (e == hipSuccess) e = launch_render_fused(L, ws, rgb, target, g_xy, g_chol, g_rgb, st);
  }
  if (e == hipSuccess && k > 0)
    e = launch_adam(L.N, xy, chol, rgb, g_xy, g_chol, g_rgb, m, v, step, cfg, nullptr, 1,
                    at<const float>(ws, L.loss_part), L.loss_parts, loss_scale, trace, trace_len,
                    st);
  return e;
}

struct StreamGuard {
  hipStream_t s = nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  ~StreamGuard() {
    if (x) (void)hipGraphExecDestroy(x);
    if (g) (void)hipGraphDestroy(g);
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  }
};

}  // namespace

extern "C" int gs2d_fit_frame(const gs2d_shape *shape, const float *target, float *xy,
                              float *chol, float *rgb, float *m, float *v, int32_t *step,
                              float *loss_trace, int32_t trace_len, void *ws, size_t ws_bytes,
                              const gs2d_fit_opts *opts, gs2d_fit_stats *stats, void *stream) {
  try {
    const auto t0 = std::chrono::steady_clock::now();
    Layout L;
    int rc = check_ws(shape, ws, ws_bytes, &L);
    if (rc != GS2D_OK) return rc;
    if (!target || !xy || !chol || !rgb || !m || !v || !step || !loss_trace || !opts)
      return GS2D_EINVAL;
    if (opts->iters < 0 || opts->check_every < 1) return GS2D_EINVAL;
    if (stats) {
      stats->iters_run = 0;
      stats->iter_hit_target = -1;
      stats->final_loss = NAN;
      stats->final_psnr = NAN;
      stats->seconds = 0.0;
      stats->status = 0;
      stats->n_culled = 0;
    }
    if (hipStreamSynchronize(as_stream(stream)) != hipSuccess) return GS2D_EHIP;
    int32_t step0 = 0;
    if (hipMemcpy(&step0, step, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
      return GS2D_EHIP;
    if (step0 < 0 || (long long)step0 + opts->iters >= (long long)trace_len) return GS2D_EINVAL;

    StreamGuard G;
    if (hipStreamCreateWithFlags(&G.s, hipStreamNonBlocking) != hipSuccess) return GS2D_EHIP;
    hipStream_t st = G.s;
    int32_t *misc = at<int32_t>(ws, L.misc);
    hipError_t e = launch_fill_zero_u32(reinterpret_cast<uint32_t *>(misc), MISC_COUNT, st);
    if (e == hipSuccess) e = launch_fill_zero(at<float>(ws, L.grads), 8 * (size_t)L.N, st);
    if (e != hipSuccess) return GS2D_EHIP;

    std::vector<float> trace_host((size_t)opts->check_every);
    int done = 0, graph_k = 0, hit = -1;
    float last_loss = NAN;
    uint32_t sticky = 0;
    while (done < opts->iters) {
      const int k = std::min(opts->check_every, opts->iters - done);
      if (opts->use_graph) {
        if (graph_k != k) {
          if (G.x) (void)hipGraphExecDestroy(G.x), G.x = nullptr;
          if (G.g) (void)hipGraphDestroy(G.g), G.g = nullptr;
          if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return GS2D_EHIP;
          const hipError_t ce = enqueue_iterations(L, ws, target, xy, chol, rgb, m, v, step,
                                                   loss_trace, trace_len, opts->adam, k, st);
          hipError_t ee = hipStreamEndCapture(st, &G.g);
          if (ce != hipSuccess || ee != hipSuccess) return GS2D_EHIP;
          if (hipGraphInstantiate(&G.x, G.g, nullptr, nullptr, 0) != hipSuccess) return GS2D_EHIP;
          graph_k = k;
        }
        if (hipGraphLaunch(G.x, st) != hipSuccess) return GS2D_EHIP;
      } else {
        if (enqueue_iterations(L, ws, target, xy, chol, rgb, m, v, step, loss_trace, trace_len,
                               opts->adam, k, st) != hipSuccess)
          return GS2D_EHIP;
      }
      if (hipMemcpyAsync(trace_host.data(), loss_trace + step0 + done, sizeof(float) * k,
                         hipMemcpyDeviceToHost, st) != hipSuccess)
        return GS2D_EHIP;
      if (hipMemcpyAsync(&sticky, misc + MISC_STICKY, sizeof(uint32_t), hipMemcpyDeviceToHost,
                         st) != hipSuccess)
        return GS2D_EHIP;
      if (hipStreamSynchronize(st) != hipSuccess) return GS2D_EHIP;
      for (int i = 0; i < k; ++i) {
        last_loss = trace_host[i];
        if (hit < 0 && opts->psnr_target > 0.f && last_loss > 0.f &&
            10.0 * std::log10(1.0 / last_loss) >= opts->psnr_target)
          hit = done + i;
      }
      done += k;
      if (sticky & STATUS_OVERFLOW) break;
      if (hit >= 0) break;
    }
    int32_t n_culled = 0;
    (void)hipMemcpy(&n_culled, misc + MISC_N_CULLED, sizeof(int32_t), hipMemcpyDeviceToHost);
    if (stats) {
      stats->iters_run = done;
      stats->iter_hit_target = hit;
      stats->final_loss = last_loss;
      stats->final_psnr =
          (last_loss > 0.f) ? (float)(10.0 * std::log10(1.0 / last_loss)) : INFINITY;
      stats->status = sticky;
      stats->n_culled = n_culled;
      stats->seconds =
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return (sticky & STATUS_OVERFLOW) ? GS2D_EOVERFLOW : GS2D_OK;
  } catch (...) {
    return GS2D_EHIP;
  }
}
