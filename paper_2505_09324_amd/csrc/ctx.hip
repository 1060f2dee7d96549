// The fitting context: a per-device cache of instantiated hipGraphs for the
// chunks of fitting iterations that gs2d_fit_frame / gs2d_fit_batch replay.
// A video encoder calls the fitting loop once per frame with the same
// buffers (Sec. 3.2: every frame is fitted, P-frames warm-started from the
// previous one), so the capture and instantiation of a chunk happen once per
// sequence instead of once per frame.
#include <algorithm>
#include <new>

#include "gs2d_internal.h"

gs2d_ctx::~gs2d_ctx() {
  for (Entry &e : graphs)
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (capture) (void)hipStreamDestroy(capture);
  if (host_misc) (void)hipHostFree(host_misc);
}

hipError_t gs2d_ctx::graph_for(const gs2d::GraphKey &key,
                               const std::function<hipError_t(hipStream_t)> &enqueue,
                               hipGraphExec_t *out) {
  ++clock;
  for (Entry &e : graphs)
    if (e.key == key) {
      e.used = clock;
      *out = e.exec;
      return hipSuccess;
    }
  if (!capture) {
    hipError_t e = hipStreamCreateWithFlags(&capture, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  hipError_t e = hipStreamBeginCapture(capture, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  const hipError_t ce = enqueue(capture);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(capture, &g);
  if (ce != hipSuccess || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return ce != hipSuccess ? ce : e;
  }
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);  // the executable holds its own copy
  if (e != hipSuccess) return e;
  if (graphs.size() >= MAX_GRAPHS) {
    auto lru = std::min_element(graphs.begin(), graphs.end(),
                                [](const Entry &a, const Entry &b) { return a.used < b.used; });
    (void)hipGraphExecDestroy(lru->exec);
    graphs.erase(lru);
  }
  graphs.push_back(Entry{key, x, clock});
  ++captures;
  *out = x;
  return hipSuccess;
}

int gs2d_ctx_check(const gs2d_ctx *ctx) {
  if (!ctx) return GS2D_OK;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return GS2D_EHIP;
  return dev == ctx->device ? GS2D_OK : GS2D_EINVAL;
}

extern "C" int gs2d_ctx_create(gs2d_ctx **out, int32_t device) {
  try {
    if (!out) return GS2D_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) return GS2D_EHIP;
    if (device < 0 || device >= n) return GS2D_EINVAL;
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return GS2D_EHIP;
    if (cur != device && hipSetDevice(device) != hipSuccess) return GS2D_EHIP;
    gs2d_ctx *c = new (std::nothrow) gs2d_ctx;
    hipError_t e = c ? hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking)
                     : hipErrorOutOfMemory;
    if (e == hipSuccess)
      e = hipHostMalloc(reinterpret_cast<void **>(&c->host_misc),
                        gs2d_ctx::HOST_MISC_WORDS * sizeof(int32_t), hipHostMallocDefault);
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) {
      delete c;
      return GS2D_EHIP;
    }
    c->device = device;
    *out = c;
    return GS2D_OK;
  } catch (...) {
    return GS2D_EHIP;
  }
}

extern "C" void gs2d_ctx_destroy(gs2d_ctx *ctx) {
  try {
    delete ctx;
  } catch (...) {
  }
}

extern "C" int gs2d_ctx_stats(const gs2d_ctx *ctx, int32_t *cached, int64_t *captures) {
  if (!ctx) return GS2D_EINVAL;
  if (cached) *cached = (int32_t)ctx->graphs.size();
  if (captures) *captures = (int64_t)ctx->captures;
  return GS2D_OK;
}
