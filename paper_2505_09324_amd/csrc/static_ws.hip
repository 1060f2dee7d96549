// gs2d_fit_frame_static: the fitting loop with its workspace in a
// file-scope device array instead of a caller buffer, for callers that
// cannot allocate device memory.  Each device the library runs on holds its
// own copy of the array until the process ends; its device address is
// looked up once per device and used for every kernel argument and clear.
#include <mutex>

#include "gs2d_internal.h"

namespace {

constexpr size_t STATIC_BYTES = (size_t)GS2D_STATIC_WORKSPACE_BYTES;
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[STATIC_BYTES];

std::mutex g_lock;
void *g_addr[MAX_DEVICES] = {};

// The device address of `scratch` on the current device (looked up on the
// first call on that device, with that device current).
int scratch_address(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return GS2D_EHIP;
  if (dev < 0 || dev >= MAX_DEVICES) return GS2D_EINVAL;
  std::lock_guard<std::mutex> g(g_lock);
  if (!g_addr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GS2D_EHIP;
    g_addr[dev] = p;
  }
  *out = g_addr[dev];
  return GS2D_OK;
}

}  // namespace

extern "C" int gs2d_fit_frame_static(const gs2d_shape *shape, const float *target, float *xy,
                                     float *chol, float *rgb, float *m, float *v, int32_t *step,
                                     float *loss_trace, int32_t trace_len,
                                     const gs2d_fit_opts *opts, gs2d_fit_stats *stats,
                                     void *stream) {
  try {
    gs2d::Layout L;
    if (!shape || !gs2d::make_layout(*shape, &L)) return GS2D_EINVAL;
    if (L.total > STATIC_BYTES) return GS2D_ENOSPACE;
    if (!target || !xy || !chol || !rgb || !m || !v || !step || !loss_trace || !opts)
      return GS2D_EINVAL;
    if (opts->iters < 0 || opts->check_every < 1 || opts->qat) return GS2D_EINVAL;
    if (!(opts->bin_skin >= 0.f && opts->bin_skin <= 64.f)) return GS2D_EINVAL;
    void *ws = nullptr;
    const int rc = scratch_address(&ws);
    if (rc != GS2D_OK) return rc;
    gs2d_fit_opts eager = *opts;
    eager.use_graph = 0;  // instantiating a graph may allocate
    const gs2d::FitArgs a{target, xy,        chol,         rgb,         m,  v,
                          step,   loss_trace, trace_len, ws,          opts->adam,
                          opts->active,        0,            0,           opts->bin_skin};
    return gs2d::fit_frame_run(nullptr, L, a, eager, stats, reinterpret_cast<hipStream_t>(stream));
  } catch (...) {
    return GS2D_EHIP;
  }
}
