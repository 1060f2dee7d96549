// Fused Adam update over all 8N Gaussian parameters (the optimisation step
// of the fitting loop), plus small fill kernels.
//
//   t = step[0]   (already incremented for this step, see below)
//   m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2
//   theta <- theta - lr_group * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)
//
// The step count lives in device memory so a captured graph can replay the
// update.  It is incremented before the Adam kernel runs, by a one-thread
// kernel for a standalone step, or by the single-block count scan of the
// binning inside the fitting loop, so the Adam kernel itself only reads it.
// Optionally the kernel clears the gradients after reading them (ready for
// the next backward pass's atomics), and block 0 reduces the per-tile loss
// partials of this iteration into loss_trace[t-1].
#include "gs2d_internal.h"

namespace gs2d {

__global__ void __launch_bounds__(256)
k_adam(int N, float *__restrict__ xy, float *__restrict__ chol, float *__restrict__ rgb,
       float *__restrict__ g_xy, float *__restrict__ g_chol, float *__restrict__ g_rgb,
       float *__restrict__ m, float *__restrict__ v, int32_t *__restrict__ step, float lr0,
       float lr1, float lr2, float b1, float b2, float eps, const uint8_t *__restrict__ active,
       int zero_grads, const float *__restrict__ loss_part, int n_part, float loss_scale,
       float *__restrict__ loss_trace, int trace_len, int32_t *__restrict__ report) {
  __shared__ double red[4];
  // every thread reads the step (advanced only by a separate kernel) and
  // derives the bias corrections itself: no barrier before the loads
  const int t = step[0];
  float bc1, bc2;
  adam_bias(t, b1, b2, &bc1, &bc2);
  const int total = 8 * N;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
    float *p, *g;
    float lr;
    int n;
    if (e < 2 * N) {
      p = xy + e;
      g = g_xy + e;
      lr = lr0;
      n = e >> 1;
    } else if (e < 5 * N) {
      const int i = e - 2 * N;
      p = chol + i;
      g = g_chol + i;
      lr = lr1;
      n = i / 3;
    } else {
      const int i = e - 5 * N;
      p = rgb + i;
      g = g_rgb + i;
      lr = lr2;
      n = i / 3;
    }
    const float gr = *g;
    if (zero_grads) *g = 0.f;
    if (active && active[n] == 0) continue;
    *p = adam_update(*p, gr, m + e, v + e, lr, b1, b2, eps, bc1, bc2);
  }
  if (loss_part && blockIdx.x == 0) {
    double s = 0.0;
    s = thread_sum_parts(loss_part, n_part);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      const float loss = (float)((red[0] + red[1] + red[2] + red[3]) * (double)loss_scale);
      if (t - 1 < trace_len) loss_trace[t - 1] = loss;
      if (report) {
        report[0] = t;
        report[1] = __float_as_int(loss);
      }
    }
  }
}

__global__ void k_step_tick(int32_t *__restrict__ step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) step[0] += 1;
}

hipError_t launch_step_tick(int32_t *step, hipStream_t st) {
  hipLaunchKernelGGL(k_step_tick, dim3(1), dim3(64), 0, st, step);
  return hipGetLastError();
}

__global__ void k_fill_zero(float *__restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

__global__ void k_fill_zero_u32(uint32_t *__restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// The start of a fitting call in one launch, and the n_grads gradient
// accumulators zeroed.  With lazy binning the lists in the workspace are
// kept when the stamp shows complete lists of this layout that did not
// overflow the pair capacity: then the words
// that describe them (pair count, status, culled count) and the stamp stay,
// and the call's sticky status starts from their status; otherwise
// misc[MISC_STALE] = 1 (rebuild at the first iteration).  Every other word
// is zeroed.
__global__ void k_fit_begin(int32_t *__restrict__ misc, float *__restrict__ grads, size_t n_grads,
                            int lazy, uint32_t sig_lo, uint32_t sig_hi) {
  const int i = (int)threadIdx.x;
  // lists truncated at the pair capacity are never kept
  const bool keep_lists = lazy && (uint32_t)misc[MISC_LISTS_LO] == sig_lo &&
                          (uint32_t)misc[MISC_LISTS_HI] == sig_hi &&
                          !(misc[MISC_STATUS] & (int)STATUS_OVERFLOW);
  if (blockIdx.x == 0 && i < MISC_COUNT && i != MISC_LISTS_LO && i != MISC_LISTS_HI &&
      i != MISC_N_PAIRS && i != MISC_STATUS && i != MISC_N_CULLED) {
    int v = 0;
    if (i == MISC_STALE) v = (lazy && !keep_lists) ? 1 : 0;
    if (i == MISC_STICKY) v = keep_lists ? misc[MISC_STATUS] : 0;
    misc[i] = v;
  }
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n_grads;
       i += (size_t)gridDim.x * blockDim.x)
    grads[i] = 0.f;
}

hipError_t launch_fit_begin(int32_t *misc, float *grads, size_t n_grads, bool lazy,
                            uint32_t sig_lo, uint32_t sig_hi, hipStream_t st) {
  static_assert(MISC_COUNT <= 256, "one block clears misc");
  size_t nb = (n_grads + 255) / 256;
  nb = nb < 1 ? 1 : (nb > 2048 ? 2048 : nb);
  hipLaunchKernelGGL(k_fit_begin, dim3((unsigned)nb), dim3(256), 0, st, misc, grads, n_grads,
                     lazy ? 1 : 0, sig_lo, sig_hi);
  return hipGetLastError();
}

static int adam_blocks(int N) {
  const int need = (8 * N + 255) / 256;
  return need < 1024 ? (need > 0 ? need : 1) : 1024;
}

hipError_t launch_adam(int N, float *xy, float *chol, float *rgb, float *g_xy, float *g_chol,
                       float *g_rgb, float *m, float *v, int32_t *step, const gs2d_adam_cfg &cfg,
                       const uint8_t *active, int zero_grads, const float *loss_part,
                       int n_loss_part, float loss_scale, float *loss_trace, int trace_len,
                       hipStream_t st, int32_t *report) {
  hipLaunchKernelGGL(k_adam, dim3(adam_blocks(N)), dim3(256), 0, st, N, xy, chol, rgb, g_xy, g_chol,
                     g_rgb, m, v, step, cfg.lr[0], cfg.lr[1], cfg.lr[2], cfg.beta1, cfg.beta2,
                     cfg.eps, active, zero_grads, loss_part, n_loss_part, loss_scale, loss_trace,
                     trace_len, report);
  return hipGetLastError();
}

hipError_t launch_fill_zero(float *p, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t nb = (n + 255) / 256;
  if (nb > 2048) nb = 2048;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)nb), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_fill_zero_u32(uint32_t *p, size_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  size_t nb = (n + 255) / 256;
  if (nb > 2048) nb = 2048;
  hipLaunchKernelGGL(k_fill_zero_u32, dim3((unsigned)nb), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace gs2d
