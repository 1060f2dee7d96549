// Post-training quantisation of a frame's Gaussians and the frame's bit
// count (the compression pipeline, Sec. 3.3.A / 3.3.B).  Distinct
// quantisers per attribute:
//   mean       IEEE binary16, round to nearest even (16 bits per coordinate);
//   Cholesky,  per component a uniform min-max quantiser with b bits over
//   colour     the frame's range: with lo, hi the component's extremes,
//              L = 2^b - 1, inv = L / (hi - lo) (0 if hi == lo),
//              step = (hi - lo) / L:
//                code = clamp(rint((x - lo) * inv), 0, L);  x^ = lo + code step
//              evaluated in FP32 in exactly this order without contraction,
//              so the codes are reproducible integer decisions.
// Bits of vanilla entropy coding: an ideal static coder for the frame's own
// code statistics, N * H per quantised component (H the empirical entropy,
// FP64), 16 bits per coordinate for the means, and lo, hi of every
// component (FP32) as side information.
//
// Kernels: per-block extremes of the six quantised components, one block
// that reduces them and derives inv and step, the encoder (one thread per
// Gaussian: binary16 means, codes, dequantised values, histogram counts by
// global atomics), and one block per component for its entropy.
#include <hip/hip_fp16.h>

#include <algorithm>

#include "gs2d_internal.h"

namespace gs2d {
namespace {

constexpr int QB = 256;          // threads per block
constexpr int Q_MAX_BLOCKS = 1024;
constexpr int Q_MAX_BITS = 12;
constexpr int Q_BINS = 1 << Q_MAX_BITS;

struct QLayout {
  size_t part, param, hist, total;
  int blocks;
};

QLayout q_layout(int N) {
  QLayout q;
  q.blocks = std::min((N + QB - 1) / QB, Q_MAX_BLOCKS);
  size_t o = 0;
  auto take = [&o](size_t b) {
    const size_t at = o;
    o = (o + b + 255) & ~(size_t)255;
    return at;
  };
  q.part = take((size_t)q.blocks * 12 * 4);  // per block: 6 x (min, max)
  q.param = take(6 * 4 * 4);                 // per component: lo, hi, inv, step
  q.hist = take((size_t)6 * Q_BINS * 4);
  q.total = o;
  return q;
}

__device__ inline float comp(const float *__restrict__ chol, const float *__restrict__ rgb, int n,
                             int c) {
  return c < 3 ? chol[3 * n + c] : rgb[3 * n + c - 3];
}

__global__ void __launch_bounds__(QB)
k_q_extremes(int N, const float *__restrict__ chol, const float *__restrict__ rgb,
             float *__restrict__ part) {
  __shared__ float red[QB / 64][12];
  float mn[6], mx[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) mn[c] = INFINITY, mx[c] = -INFINITY;
  for (int n = blockIdx.x * QB + threadIdx.x; n < N; n += gridDim.x * QB) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const float x = comp(chol, rgb, n, c);
      mn[c] = fminf(mn[c], x);
      mx[c] = fmaxf(mx[c], x);
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c)
    for (int o = 32; o > 0; o >>= 1) {
      mn[c] = fminf(mn[c], __shfl_xor(mn[c], o, 64));
      mx[c] = fmaxf(mx[c], __shfl_xor(mx[c], o, 64));
    }
  if ((threadIdx.x & 63) == 0)
    for (int c = 0; c < 6; ++c) red[threadIdx.x >> 6][2 * c] = mn[c], red[threadIdx.x >> 6][2 * c + 1] = mx[c];
  __syncthreads();
  if (threadIdx.x < 12) {
    float v = red[0][threadIdx.x];
    for (int w = 1; w < QB / 64; ++w)
      v = (threadIdx.x & 1) ? fmaxf(v, red[w][threadIdx.x]) : fminf(v, red[w][threadIdx.x]);
    part[blockIdx.x * 12 + threadIdx.x] = v;
  }
}

// One block: extremes over the block partials, then inv and step.
__global__ void k_q_params(int nblocks, const float *__restrict__ part, int bits_chol, int bits_rgb,
                           float *__restrict__ param, float *__restrict__ ranges) {
  __shared__ float ext[12];
  const int i = threadIdx.x;
  if (i < 12) {
    float v = part[i];
    for (int b = 1; b < nblocks; ++b)
      v = (i & 1) ? fmaxf(v, part[b * 12 + i]) : fminf(v, part[b * 12 + i]);
    ext[i] = v;
    if (ranges) ranges[i] = v;
  }
  __syncthreads();
  if (i < 6) {
    const float lo = ext[2 * i], hi = ext[2 * i + 1];
    const float L = (float)((1 << (i < 3 ? bits_chol : bits_rgb)) - 1);
    const float rng = f32_sub(hi, lo);
    param[4 * i] = lo;
    param[4 * i + 1] = hi;
    param[4 * i + 2] = rng == 0.f ? 0.f : __fdiv_rn(L, rng);
    param[4 * i + 3] = rng == 0.f ? 0.f : __fdiv_rn(rng, L);
  }
}

__global__ void __launch_bounds__(QB)
k_q_encode(int N, const float *__restrict__ xy, const float *__restrict__ chol,
           const float *__restrict__ rgb, int bits_chol, int bits_rgb,
           const float *__restrict__ param, float *__restrict__ q_xy, float *__restrict__ q_chol,
           float *__restrict__ q_rgb, uint16_t *__restrict__ codes, uint32_t *__restrict__ hist) {
  for (int n = blockIdx.x * QB + threadIdx.x; n < N; n += gridDim.x * QB) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const __half h = __float2half_rn(xy[2 * n + k]);
      q_xy[2 * n + k] = __half2float(h);
      if (codes) codes[8 * n + k] = __half_as_ushort(h);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const float lo = param[4 * c], inv = param[4 * c + 2], step = param[4 * c + 3];
      const float L = (float)((1 << (c < 3 ? bits_chol : bits_rgb)) - 1);
      const float t = f32_mul(f32_sub(comp(chol, rgb, n, c), lo), inv);
      const float code = fminf(fmaxf(rintf(t), 0.f), L);
      const float xh = f32_add(lo, f32_mul(code, step));
      if (c < 3) q_chol[3 * n + c] = xh;
      else q_rgb[3 * n + c - 3] = xh;
      if (codes) codes[8 * n + 2 + c] = (uint16_t)code;
      if (hist) atomicAdd(&hist[c * Q_BINS + (int)code], 1u);
    }
  }
}

// Block c: N * H of component c's histogram, in FP64.
__global__ void __launch_bounds__(QB)
k_q_entropy(int N, int bits_chol, int bits_rgb, const uint32_t *__restrict__ hist,
            double *__restrict__ bits) {
  __shared__ double red[QB / 64];
  const int c = blockIdx.x;
  const int nb = 1 << (c < 3 ? bits_chol : bits_rgb);
  const double inv_n = 1.0 / (double)N;
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += QB) {
    const uint32_t k = hist[c * Q_BINS + i];
    if (k) {
      const double p = (double)k * inv_n;
      s -= p * log2(p);
    }
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < QB / 64; ++w) t += red[w];
    bits[c] = t * (double)N;
  }
}

// bits[6] = 32 N (binary16 means) + sum of the six components + side info.
__global__ void k_q_total(int N, double *__restrict__ bits) {
  if (threadIdx.x == 0) {
    double t = 32.0 * (double)N + 6.0 * 64.0;
    for (int c = 0; c < 6; ++c) t += bits[c];
    bits[6] = t;
  }
}

}  // namespace

hipError_t launch_quantise(int N, const float *xy, const float *chol, const float *rgb,
                           int bits_chol, int bits_rgb, float *q_xy, float *q_chol, float *q_rgb,
                           uint16_t *codes, float *ranges, double *bits, void *qws,
                           hipStream_t st) {
  const QLayout q = q_layout(N);
  float *part = at<float>(qws, q.part), *param = at<float>(qws, q.param);
  uint32_t *hist = bits ? at<uint32_t>(qws, q.hist) : nullptr;
  hipLaunchKernelGGL(k_q_extremes, dim3(q.blocks), dim3(QB), 0, st, N, chol, rgb, part);
  hipLaunchKernelGGL(k_q_params, dim3(1), dim3(64), 0, st, q.blocks, part, bits_chol, bits_rgb,
                     param, ranges);
  if (hist) {
    hipError_t e = launch_fill_zero_u32(hist, (size_t)6 * Q_BINS, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_q_encode, dim3(q.blocks), dim3(QB), 0, st, N, xy, chol, rgb, bits_chol,
                     bits_rgb, param, q_xy, q_chol, q_rgb, codes, hist);
  if (bits) {
    hipLaunchKernelGGL(k_q_entropy, dim3(6), dim3(QB), 0, st, N, bits_chol, bits_rgb, hist, bits);
    hipLaunchKernelGGL(k_q_total, dim3(1), dim3(64), 0, st, N, bits);
  }
  return hipGetLastError();
}

size_t quantise_workspace_bytes(int N) { return q_layout(N).total; }

}  // namespace gs2d

using namespace gs2d;

extern "C" size_t gs2d_ptq_workspace_bytes(int32_t N) {
  return N < 1 ? 0 : quantise_workspace_bytes(N);
}

extern "C" int gs2d_ptq(int32_t N, const float *xy, const float *chol, const float *rgb,
                        const gs2d_quant_cfg *cfg, float *q_xy, float *q_chol, float *q_rgb,
                        uint16_t *codes, float *ranges, double *bits, void *ws, size_t ws_bytes,
                        void *stream) {
  try {
    if (N < 1 || !xy || !chol || !rgb || !cfg || !q_xy || !q_chol || !q_rgb) return GS2D_EINVAL;
    if (cfg->bits_chol < 1 || cfg->bits_chol > Q_MAX_BITS || cfg->bits_rgb < 1 ||
        cfg->bits_rgb > Q_MAX_BITS)
      return GS2D_EINVAL;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return GS2D_EINVAL;
    if (ws_bytes < quantise_workspace_bytes(N)) return GS2D_ENOSPACE;
    return launch_quantise(N, xy, chol, rgb, cfg->bits_chol, cfg->bits_rgb, q_xy, q_chol, q_rgb,
                           codes, ranges, bits, ws, reinterpret_cast<hipStream_t>(stream)) ==
                   hipSuccess
               ? GS2D_OK
               : GS2D_EHIP;
  } catch (...) {
    return GS2D_EHIP;
  }
}
