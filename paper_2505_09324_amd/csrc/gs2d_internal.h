// Internal definitions shared by the gs2d HIP translation units: workspace
// layout, kernel declarations and small device helpers.  Not part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <functional>
#include <vector>

#include "gs2d.h"

namespace gs2d {

// Slots of the small integer block at the end of the workspace.
enum MiscSlot : int {
  MISC_N_PAIRS = 0,   // min(total pairs, max_pairs)
  MISC_STATUS = 1,    // status bits of the last binning
  MISC_N_CULLED = 2,  // culled Gaussians of the last binning
  MISC_STICKY = 3,    // OR of MISC_STATUS over a fit call
  MISC_REBINS = 4,    // tile-list rebuilds in a fit call (lazy binning)
  MISC_STALE = 5,     // lazy binning: the lists must be rebuilt this iteration
  MISC_TICKET = 6,    // lazy rebuild: roles taken (k_bin_lazy_wide), 0 between launches
  MISC_EMITTED = 7,   // lazy rebuild: chunks emitted, 0 between launches
  MISC_FINISHED = 8,  // lazy rebuild: blocks done, 0 between launches
  MISC_STEP = 9,      // the fitting loop's last Adam step: its step count ...
  MISC_LAST_LOSS = 10,  // ... and the loss it recorded (FP32 bits)
  // lazy binning: the layout's signature (Layout::sig_lo, sig_hi) while the
  // workspace holds complete lazy lists of that layout, built from the
  // rectangles in brect; 0 once any other binning or a stalled rebuild has
  // written the lists.  A fitting call then starts from these lists instead
  // of rebuilding them.
  MISC_LISTS_LO = 12,
  MISC_LISTS_HI = 13,
  MISC_COUNT = 64
};

constexpr uint32_t STATUS_OVERFLOW = 1u;
constexpr uint32_t STATUS_CULLED = 2u;
constexpr uint32_t STATUS_STALLED = 4u;  // a lazy rebuild's bounded wait ran out (lists kept)

constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int SORT_BLOCK = 256;       // threads per sort block (4 waves)
constexpr int SORT_MAX_BLOCKS = 128;  // sort blocks (each owns one key chunk)
constexpr int SCAN_BLOCK = 1024;

// Byte offsets of every array inside one frame's workspace.
struct Layout {
  int W, H, N, T, max_pairs;
  int ppl;             // pixels per lane of the raster kernels (1, 2, 4)
  int TX, TY, n_tiles;
  int loss_parts;   // loss partials: one per raster wavefront (n_tiles * waves per tile)
  int sort_blocks;  // G: fixed chunks of the key array in the second pass
  int sort_passes;  // radix passes over the tile bits (1 or 2)
  bool wide;        // single pass whose digit is the whole tile index
  int digit_bits;   // bits of that digit (8..11), D = 2^digit_bits
  int D;
  size_t geom, rect, brect, counts, offsets, blocks, keys_a, keys_b, hist, tile_start, loss_part,
      grads, qparams, qws, misc, total;
  uint32_t sig_lo, sig_hi;  // non-zero 64-bit signature of the shape and the offsets above
  // the buffer holding the sorted keys after all passes
  size_t keys_sorted() const { return (sort_passes & 1) ? keys_b : keys_a; }
};

// Adam on one parameter (Kingma and Ba, as the fitting loop uses it): with
// bias corrections bc1 = 1 - b1^t, bc2 = 1 - b2^t,
//   m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;
//   theta <- theta - lr (m / bc1) / (sqrt(v / bc2) + eps).
// Shared by the standalone optimiser kernel and the fused
// optimiser-plus-projection kernel so both round identically.
__device__ inline float adam_update(float theta, float g, float *__restrict__ m,
                                    float *__restrict__ v, float lr, float b1, float b2, float eps,
                                    float bc1, float bc2) {
  const float mm = b1 * *m + (1.f - b1) * g;
  const float vv = b2 * *v + (1.f - b2) * g * g;
  *m = mm;
  *v = vv;
  return theta - lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
}

// Bias corrections of step t, evaluated in FP64 and rounded once.
__device__ inline void adam_bias(int t, float b1, float b2, float *bc1, float *bc2) {
  *bc1 = (float)(1.0 - pow((double)b1, (double)t));
  *bc2 = (float)(1.0 - pow((double)b2, (double)t));
}

// One thread's share of a block-wide FP64 sum of n floats (element i goes
// to thread i mod blockDim.x in 16-byte groups when p is 16-byte aligned):
// eight independent loads are in flight per thread.  The caller reduces the
// per-thread values across the block.
__device__ inline double thread_sum_parts(const float *__restrict__ p, int n) {
  const int nt = blockDim.x, t = threadIdx.x;
  double s = 0.0;
  int done = 0;
  if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
    const float4 *p4 = reinterpret_cast<const float4 *>(p);
    const int n4 = n >> 2;
    for (int i0 = t; i0 < n4; i0 += 8 * nt) {
      float4 v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = p4[min(i0 + j * nt, n4 - 1)];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (i0 + j * nt < n4) s += ((double)v[j].x + (double)v[j].y) + ((double)v[j].z + (double)v[j].w);
    }
    done = 4 * n4;
  }
  for (int i = done + t; i < n; i += nt) s += (double)p[i];
  return s;
}

// The optimiser step of the previous iteration, applied by the first
// binning kernel of the next one (the fitting loop's fused form): Adam over
// the 8 parameters of each Gaussian with step t = step[0], gradients cleared,
// and the previous iteration's loss partials reduced into trace[t - 1].
struct PendingAdam {
  float *xy, *chol, *rgb;
  float *g_xy, *g_chol, *g_rgb, *m, *v;
  const int32_t *step;
  gs2d_adam_cfg cfg;
  const float *loss_part;
  int n_part;
  float loss_scale;
  float *trace;
  int trace_len;
  const uint8_t *active;  // nullable: Gaussians with active[n] == 0 keep theta, m, v
};

// Returns false if the shape is outside the supported limits.
bool make_layout(const gs2d_shape &s, Layout *L);

// The arguments of one fitting call that end up in its kernels.
struct FitArgs {
  const float *target;
  float *xy, *chol, *rgb, *m, *v;
  int32_t *step;
  float *trace;
  int trace_len;
  void *ws;
  gs2d_adam_cfg cfg;
  const uint8_t *active;  // nullable: only flagged Gaussians are updated
  int qat_bits_chol, qat_bits_rgb;  // 0: plain fitting, else quantisation-aware
  float bin_skin;  // > 0: lazy binning with this margin (px), see launch_binning
};

template <typename T>
inline T *at(void *ws, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

// ---- kernels launched by the host code (defined in the .hip files) ----

// Binning (bin.hip).  Each enqueues on `st`.
// step_tick (nullable): a device counter incremented once by the binning.
// adam (nullable): apply that optimiser step to xy/chol/rgb first (the
// projection then reads the updated parameters).
// skin > 0 (single-pass path only): lazy binning.  The lists are built from
// every Gaussian's 3-sigma box grown by `skin` pixels, and rebuilt only when
// misc[MISC_STALE] is set: by the projection when some Gaussian's exact tile
// rectangle has left the rectangle its keys were built from (or it is
// culled and still has keys), or by launch_fit_begin when the workspace
// holds no complete lists of this layout (MISC_LISTS_LO/HI).  Otherwise the
// one kernel that emits and scatters returns at once and the lists of an
// earlier iteration, a superset of the exact ones in the same (tile, index)
// order, stay in use; the raster's exact per-pixel cutoff makes the render
// identical.  The fused raster clears the flag and stamps a rebuild's lists
// (launch_render_fused); exact binning clears the stamp.  The lazy path
// does not tick step_tick: its caller ticks it in the raster.
hipError_t launch_binning(const Layout &L, const float *xy, const float *chol, void *ws,
                          hipStream_t st, int *step_tick = nullptr,
                          const PendingAdam *adam = nullptr, float skin = 0.f);

// Stable LSD radix sort of keys on bits [16, 16 + 8*passes) with G sort
// blocks; misc[0] holds the key count; hist holds RADIX * G words.
// *sorted receives a or b.
hipError_t launch_radix_sort_tiles(uint32_t *a, uint32_t *b, const int *misc, int G, uint32_t *hist,
                                   int passes, hipStream_t st, const uint32_t **sorted);
// tile_start[t] for sorted keys; misc[0] holds the key count.
hipError_t launch_tile_ranges(const uint32_t *keys, const int *misc, int n_tiles, int *tile_start,
                              hipStream_t st);

// Raster (raster.hip).
hipError_t launch_render_fwd(const Layout &L, void *ws, const float *rgb, const float *target,
                             float *img, float *dl_dimg, hipStream_t st);
hipError_t launch_render_bwd(const Layout &L, void *ws, const float *rgb, const float *dl_dimg,
                             float *g_xy, float *g_chol, float *g_rgb, hipStream_t st);
// active (nullable): the backward skips Gaussians with active[n] == 0.
// lazy: the launch also clears misc[MISC_STALE] and, when it was set,
// stamps the rebuilt lists (FrameArgs::lazy_misc).
// tick (nullable): the launch also adds 1 to *tick (the step counter).
hipError_t launch_render_fused(const Layout &L, void *ws, const float *rgb, const float *target,
                               float *g_xy, float *g_chol, float *g_rgb, hipStream_t st,
                               const uint8_t *active = nullptr, bool lazy = false,
                               int32_t *tick = nullptr);
hipError_t launch_loss_reduce(const Layout &L, void *ws, float *loss, hipStream_t st);
hipError_t launch_count_pairs(const Layout &L, void *ws, unsigned long long *out, hipStream_t st);

// Optimiser (adam.hip).  step[0] must already hold this step's t (>= 1):
// either launch_step_tick or the binning's tick has run before.
// loss_part/loss_trace may be NULL; when given, the kernel also reduces the
// per-tile loss partials into loss_trace[t - 1], and with report also
// writes report[0] = t and report[1] = that loss (FP32 bits).
hipError_t launch_step_tick(int32_t *step, hipStream_t st);
hipError_t launch_adam(int N, float *xy, float *chol, float *rgb, float *g_xy, float *g_chol,
                       float *g_rgb, float *m, float *v, int32_t *step, const gs2d_adam_cfg &cfg,
                       const uint8_t *active, int zero_grads, const float *loss_part,
                       int n_loss_part, float loss_scale, float *loss_trace, int trace_len,
                       hipStream_t st, int32_t *report = nullptr);

hipError_t launch_fill_zero(float *p, size_t n, hipStream_t st);

// Quantisation (quant.hip): binary16 means, uniform min-max codes of the
// Cholesky vector and colour; codes, ranges and bits nullable; qws holds
// quantise_workspace_bytes(N).
hipError_t launch_quantise(int N, const float *xy, const float *chol, const float *rgb,
                           int bits_chol, int bits_rgb, float *q_xy, float *q_chol, float *q_rgb,
                           uint16_t *codes, float *ranges, double *bits, void *qws,
                           hipStream_t st);
size_t quantise_workspace_bytes(int N);
hipError_t launch_fill_zero_u32(uint32_t *p, size_t n, hipStream_t st);
// Start of a fitting call, in one launch: grads[0, n_grads) zeroed and misc
// reset for the call.  With lazy binning, if the stamp (MISC_LISTS_LO/HI)
// equals (sig_lo, sig_hi) the workspace's lists are complete lists of this
// layout and are kept (with their pair count, status and culled count; the
// call's sticky status starts from that status); else misc[MISC_STALE] = 1.
hipError_t launch_fit_begin(int32_t *misc, float *grads, size_t n_grads, bool lazy,
                            uint32_t sig_lo, uint32_t sig_hi, hipStream_t st);

// ---- device helpers ----

// FP32 operations evaluated exactly as written: each rounds once to nearest
// even and is never fused with a neighbouring operation into a multiply-add
// (these bodies are compiled with contraction off; the HIP _rn intrinsics
// alone do not stop a product from being contracted into a following sum).
// Every specified FP32 order whose result decides an integer (tile
// rectangles, gradient levels, selection and quantiser tests, target ranks)
// is written with them.
__device__ inline float f32_mul(float a, float b) {
#pragma clang fp contract(off)
  return a * b;
}
__device__ inline float f32_add(float a, float b) {
#pragma clang fp contract(off)
  return a + b;
}
__device__ inline float f32_sub(float a, float b) {
#pragma clang fp contract(off)
  return a - b;
}
// Correctly rounded square root (the library's sqrtf lowering, which
// corrects the hardware estimate; __fsqrt_rn is the uncorrected estimate).
__device__ inline float f32_sqrt(float a) { return __builtin_sqrtf(a); }

__device__ inline unsigned long long lanemask_lt() {
  const unsigned lane = __lane_id();
  return (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
}

// ---- host-side graph cache (the opaque gs2d_ctx of the C ABI) ----

// Words identifying one captured chunk of work: every pointer, size and
// hyper-parameter baked into its kernel arguments.
using GraphKey = std::vector<uint64_t>;

inline uint64_t key_word(const void *p) { return (uint64_t)reinterpret_cast<uintptr_t>(p); }
inline uint64_t key_word(float f) {
  uint32_t u;
  static_assert(sizeof(u) == sizeof(f), "float size");
  __builtin_memcpy(&u, &f, sizeof(u));
  return u;
}

}  // namespace gs2d

// Instantiated graphs of fitting chunks, keyed by GraphKey, captured on a
// stream of the context's own and launched on the caller's stream.  Host
// only; one context serves one host thread at a time.
struct gs2d_ctx {
  static constexpr size_t MAX_GRAPHS = 16;
  struct Entry {
    gs2d::GraphKey key;
    hipGraphExec_t exec;
    uint64_t used;
  };
  int device = 0;
  hipStream_t capture = nullptr;
  std::vector<Entry> graphs;
  uint64_t clock = 0;
  uint64_t captures = 0;  // graphs instantiated over the context's life
  // pinned host copy of a fitting call's status words (misc), so that the
  // read-back at the end of a call is an asynchronous copy; allocated with
  // the context (a call without a context copies to pageable memory)
  int32_t *host_misc = nullptr;
  static constexpr int HOST_MISC_WORDS = 16;

  // The executable for `key`: cached, or captured now by running `enqueue`
  // on the capture stream (the least recently used entry is dropped when
  // the cache is full; no cached graph is in flight then, since every
  // fitting call waits for its work before returning).
  hipError_t graph_for(const gs2d::GraphKey &key,
                       const std::function<hipError_t(hipStream_t)> &enqueue,
                       hipGraphExec_t *out);
  ~gs2d_ctx();
};

// Checks that `ctx` (nullable) belongs to the current device.
int gs2d_ctx_check(const gs2d_ctx *ctx);

namespace gs2d {
// The host side of gs2d_fit_frame on validated arguments (api.hip): chunks
// of iterations on `st`, replayed from ctx's graphs when opts.use_graph
// (ctx NULL: graphs kept for this call only), a read-back of the loss trace
// and status after each chunk.  Allocates no host or device memory when
// opts.use_graph is 0.
int fit_frame_run(gs2d_ctx *ctx, const Layout &L, const FitArgs &a, const gs2d_fit_opts &opts,
                  gs2d_fit_stats *stats, hipStream_t st);
}  // namespace gs2d
