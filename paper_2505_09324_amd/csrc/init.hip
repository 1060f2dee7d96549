// Content-aware ROI initialisation (Sec. 3.2.A) in its synthetic-frame
// form: Gaussian centres are drawn inside the ROI with probability rising
// with the local image gradient, and uniformly outside it.
//
//  1. per pixel: Y = (R+G)+B; central differences (border: twice the
//     one-sided difference); mag = sqrt(gx*gx + gy*gy) in FP32 without
//     contraction; level q = floor(1024 mag).
//  2. inclusive prefix sums over the frame in raster order of
//     q*[roi] (int64), q (int64) and [roi] (int32).
//  3. per draw: ROI draws pick the first pixel whose running weight
//     sum_{roi} (q + b + 1) exceeds (pick mod Wt), b = Q // (10 R); outside
//     draws pick the (pick mod O)-th non-ROI pixel.  Scale, jitter and colour
//     follow; all integer decisions are exact.
#include <cmath>

#include "gs2d_internal.h"

namespace gs2d {

namespace {

constexpr int INIT_BLOCK = 256;
constexpr int INIT_PER_THREAD = 8;
constexpr int INIT_CHUNK = INIT_BLOCK * INIT_PER_THREAD;

struct InitLayout {
  size_t qm, qa, r, part, total;
  int n_chunks;
};

bool init_layout(int W, int H, InitLayout *L) {
  if (W < 1 || H < 1) return false;
  const long long HW = (long long)W * H;
  if (HW > (1LL << 28)) return false;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  L->n_chunks = (int)((HW + INIT_CHUNK - 1) / INIT_CHUNK);
  size_t o = 0;
  L->qm = o;
  o = al(o + HW * 8);
  L->qa = o;
  o = al(o + HW * 8);
  L->r = o;
  o = al(o + HW * 4);
  L->part = o;
  o = al(o + (size_t)L->n_chunks * 24 + 24);
  L->total = o;
  return true;
}

__device__ inline float luma_sum(const float *__restrict__ T, size_t HW, size_t p) {
  return f32_add(f32_add(T[p], T[HW + p]), T[2 * HW + p]);
}

__global__ void __launch_bounds__(INIT_BLOCK)
k_init_levels(int W, int H, const float *__restrict__ T, const uint8_t *__restrict__ mask,
              long long *__restrict__ qm, long long *__restrict__ qa, int *__restrict__ r) {
  const size_t HW = (size_t)W * H;
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < HW;
       p += (size_t)gridDim.x * blockDim.x) {
    const int y = (int)(p / W), x = (int)(p % W);
    float gx = 0.f, gy = 0.f;
    if (W > 1) {
      if (x == 0)
        gx = f32_mul(f32_sub(luma_sum(T, HW, p + 1), luma_sum(T, HW, p)), 2.0f);
      else if (x == W - 1)
        gx = f32_mul(f32_sub(luma_sum(T, HW, p), luma_sum(T, HW, p - 1)), 2.0f);
      else
        gx = f32_sub(luma_sum(T, HW, p + 1), luma_sum(T, HW, p - 1));
    }
    if (H > 1) {
      if (y == 0)
        gy = f32_mul(f32_sub(luma_sum(T, HW, p + W), luma_sum(T, HW, p)), 2.0f);
      else if (y == H - 1)
        gy = f32_mul(f32_sub(luma_sum(T, HW, p), luma_sum(T, HW, p - W)), 2.0f);
      else
        gy = f32_sub(luma_sum(T, HW, p + W), luma_sum(T, HW, p - W));
    }
    const float mag = f32_sqrt(f32_add(f32_mul(gx, gx), f32_mul(gy, gy)));
    const long long q = (long long)floorf(f32_mul(mag, 1024.0f));
    const int in = mask[p] != 0;
    qm[p] = in ? q : 0;
    qa[p] = q;
    r[p] = in;
  }
}

// Sum of each chunk of INIT_CHUNK pixels: part[c] = {sum qm, sum qa, sum r}.
__global__ void __launch_bounds__(INIT_BLOCK)
k_init_chunk_sums(size_t HW, const long long *__restrict__ qm, const long long *__restrict__ qa,
                  const int *__restrict__ r, long long *__restrict__ part) {
  __shared__ long long red[3][INIT_BLOCK / 64];
  const size_t base = (size_t)blockIdx.x * INIT_CHUNK;
  long long a = 0, b = 0, c = 0;
  for (int i = threadIdx.x; i < INIT_CHUNK; i += INIT_BLOCK) {
    const size_t p = base + i;
    if (p < HW) {
      a += qm[p];
      b += qa[p];
      c += r[p];
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
    c += __shfl_xor(c, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = b;
    red[2][threadIdx.x >> 6] = c;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    long long s = 0;
    for (int w = 0; w < INIT_BLOCK / 64; ++w) s += red[threadIdx.x][w];
    part[3 * (size_t)blockIdx.x + threadIdx.x] = s;
  }
}

// Exclusive scan of the chunk sums in place by one workgroup of SCAN_T
// threads (a few thousand chunks: each thread scans a contiguous run, then
// the run totals are scanned across the workgroup); the totals go to
// part[3*n .. 3*n+2].  Integer sums: the order does not matter.
constexpr int SCAN_T = 1024;
__global__ void __launch_bounds__(SCAN_T) k_init_scan_parts(int n, long long *__restrict__ part) {
  __shared__ long long run[3][SCAN_T];
  const int t = threadIdx.x;
  const int per = (n + SCAN_T - 1) / SCAN_T;
  const int beg = min(n, t * per), end = min(n, beg + per);
  long long s[3] = {0, 0, 0};
  for (int c = beg; c < end; ++c)
    for (int k = 0; k < 3; ++k) s[k] += part[3 * (size_t)c + k];
  for (int k = 0; k < 3; ++k) run[k][t] = s[k];
  __syncthreads();
  for (int o = 1; o < SCAN_T; o <<= 1) {  // inclusive Hillis-Steele scan of the run totals
    long long x[3];
    for (int k = 0; k < 3; ++k) x[k] = t >= o ? run[k][t - o] : 0;
    __syncthreads();
    for (int k = 0; k < 3; ++k) run[k][t] += x[k];
    __syncthreads();
  }
  long long acc[3];
  for (int k = 0; k < 3; ++k) acc[k] = run[k][t] - s[k];
  for (int c = beg; c < end; ++c)
    for (int k = 0; k < 3; ++k) {
      const long long v = part[3 * (size_t)c + k];
      part[3 * (size_t)c + k] = acc[k];
      acc[k] += v;
    }
  if (t == SCAN_T - 1)
    for (int k = 0; k < 3; ++k) part[3 * (size_t)n + k] = run[k][t];
}

// Inclusive scan inside each chunk plus the chunk's offset, in place.
__global__ void __launch_bounds__(INIT_BLOCK)
k_init_chunk_scan(size_t HW, long long *__restrict__ qm, long long *__restrict__ qa,
                  int *__restrict__ r, const long long *__restrict__ part) {
  __shared__ long long sa[INIT_BLOCK], sb[INIT_BLOCK], sc[INIT_BLOCK];
  const size_t base = (size_t)blockIdx.x * INIT_CHUNK + (size_t)threadIdx.x * INIT_PER_THREAD;
  long long a = 0, b = 0, c = 0;
  for (int i = 0; i < INIT_PER_THREAD; ++i) {
    const size_t p = base + i;
    if (p < HW) {
      a += qm[p];
      b += qa[p];
      c += r[p];
    }
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  sc[threadIdx.x] = c;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread sums
  for (int o = 1; o < INIT_BLOCK; o <<= 1) {
    long long xa = 0, xb = 0, xc = 0;
    if ((int)threadIdx.x >= o) {
      xa = sa[threadIdx.x - o];
      xb = sb[threadIdx.x - o];
      xc = sc[threadIdx.x - o];
    }
    __syncthreads();
    sa[threadIdx.x] += xa;
    sb[threadIdx.x] += xb;
    sc[threadIdx.x] += xc;
    __syncthreads();
  }
  long long ra = part[3 * (size_t)blockIdx.x + 0] + sa[threadIdx.x] - a;
  long long rb = part[3 * (size_t)blockIdx.x + 1] + sb[threadIdx.x] - b;
  long long rc = part[3 * (size_t)blockIdx.x + 2] + sc[threadIdx.x] - c;
  for (int i = 0; i < INIT_PER_THREAD; ++i) {
    const size_t p = base + i;
    if (p < HW) {
      ra += qm[p];
      rb += qa[p];
      rc += r[p];
      qm[p] = ra;
      qa[p] = rb;
      r[p] = (int)rc;
    }
  }
}

struct DrawArgs {
  int W, H, n_roi, n_out;
  const float *T;
  const long long *cq;  // cumulative q over the sampling region
  const int *cr;        // cumulative ROI indicator (or pixel count)
  bool roi_all, out_all;
  long long Q, R, O, b, Wt;
  double kappa;
};

__device__ inline long long cum_q(const DrawArgs &a, size_t p) { return a.cq[p]; }
__device__ inline long long cum_r(const DrawArgs &a, size_t p) {
  return a.roi_all ? (long long)p + 1 : (long long)a.cr[p];
}
__device__ inline long long cum_o(const DrawArgs &a, size_t p) {
  return a.out_all ? (long long)p + 1 : (long long)p + 1 - (long long)a.cr[p];
}

// First pixel p with f(p) > k; f is non-decreasing and f(HW-1) > k.
template <typename F>
__device__ inline size_t first_above(size_t HW, long long k, F f) {
  size_t lo = 0, hi = HW - 1;
  while (lo < hi) {
    const size_t mid = lo + (hi - lo) / 2;
    if (f(mid) > k)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

__device__ inline float clamp_scale(double s) {
  return (float)fmin(fmax(s, 0.5), 16.0);
}

__global__ void __launch_bounds__(256)
k_init_draw(DrawArgs a, const int64_t *__restrict__ pick_roi, const float *__restrict__ jit_roi,
            const int64_t *__restrict__ pick_out, const float *__restrict__ jit_out,
            float *__restrict__ xy, float *__restrict__ chol, float *__restrict__ rgb,
            int *__restrict__ picked) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = a.n_roi + a.n_out;
  if (i >= N) return;
  const size_t HW = (size_t)a.W * a.H;
  size_t p;
  float s;
  float jx, jy;
  if (i < a.n_roi) {
    const long long k = pick_roi[i] % a.Wt;
    const long long bb = a.b + 1;
    p = first_above(HW, k, [&](size_t t) { return cum_q(a, t) + bb * cum_r(a, t); });
    const long long w = (cum_q(a, p) - (p ? cum_q(a, p - 1) : 0)) + bb;
    s = clamp_scale(0.5 * sqrt((double)a.Wt / ((double)a.n_roi * (double)w)));
    jx = jit_roi[2 * i];
    jy = jit_roi[2 * i + 1];
  } else {
    const int j = i - a.n_roi;
    const long long k = pick_out[j] % a.O;
    p = first_above(HW, k, [&](size_t t) { return cum_o(a, t); });
    s = clamp_scale(0.5 * sqrt((double)a.O / (double)a.n_out));
    jx = jit_out[2 * j];
    jy = jit_out[2 * j + 1];
  }
  const int y = (int)(p / a.W), x = (int)(p % a.W);
  xy[2 * i] = f32_add(f32_add((float)x, 0.5f), jx);
  xy[2 * i + 1] = f32_add(f32_add((float)y, 0.5f), jy);
  chol[3 * i] = s;
  chol[3 * i + 1] = 0.f;
  chol[3 * i + 2] = s;
  for (int k = 0; k < 3; ++k) rgb[3 * i + k] = (float)((double)a.T[k * HW + p] * a.kappa);
  if (picked) picked[i] = (int)p;
}

}  // namespace

}  // namespace gs2d

using namespace gs2d;

extern "C" size_t gs2d_init_workspace_bytes(int32_t W, int32_t H) {
  InitLayout L;
  return init_layout(W, H, &L) ? L.total : 0;
}

extern "C" int gs2d_init_plain(int32_t W, int32_t H, const float *target, const uint8_t *roi_mask,
                               int32_t n_roi, const int64_t *pick_roi, const float *jit_roi,
                               int32_t n_out, const int64_t *pick_out, const float *jit_out,
                               float *xy, float *chol, float *rgb, int32_t *picked, void *ws,
                               size_t ws_bytes, void *stream) {
  try {
    InitLayout L;
    if (!init_layout(W, H, &L)) return GS2D_EINVAL;
    if (n_roi < 0 || n_out < 0 || n_roi + n_out < 1 || n_roi + (long long)n_out > 65536)
      return GS2D_EINVAL;
    if (!target || !roi_mask || !xy || !chol || !rgb || !ws) return GS2D_EINVAL;
    if ((n_roi > 0 && (!pick_roi || !jit_roi)) || (n_out > 0 && (!pick_out || !jit_out)))
      return GS2D_EINVAL;
    if (reinterpret_cast<uintptr_t>(ws) & 255) return GS2D_EINVAL;
    if (ws_bytes < L.total) return GS2D_ENOSPACE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const size_t HW = (size_t)W * H;
    long long *qm = at<long long>(ws, L.qm), *qa = at<long long>(ws, L.qa);
    int *r = at<int>(ws, L.r);
    long long *part = at<long long>(ws, L.part);
    hipLaunchKernelGGL(k_init_levels, dim3((unsigned)std::min<size_t>((HW + 255) / 256, 8192)),
                       dim3(256), 0, st, W, H, target, roi_mask, qm, qa, r);
    hipLaunchKernelGGL(k_init_chunk_sums, dim3(L.n_chunks), dim3(INIT_BLOCK), 0, st, HW, qm, qa, r,
                       part);
    hipLaunchKernelGGL(k_init_scan_parts, dim3(1), dim3(SCAN_T), 0, st, L.n_chunks, part);
    hipLaunchKernelGGL(k_init_chunk_scan, dim3(L.n_chunks), dim3(INIT_BLOCK), 0, st, HW, qm, qa, r,
                       part);
    // region totals decide the sampling regions: read them back (3 int64)
    long long tot[3];
    if (hipMemcpyAsync(tot, part + 3 * (size_t)L.n_chunks, sizeof(tot), hipMemcpyDeviceToHost, st) !=
        hipSuccess)
      return GS2D_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return GS2D_EHIP;
    DrawArgs a;
    a.W = W;
    a.H = H;
    a.n_roi = n_roi;
    a.n_out = n_out;
    a.T = target;
    a.R = tot[2];
    a.roi_all = (a.R == 0);
    if (a.roi_all) {
      a.R = (long long)HW;
      a.Q = tot[1];
      a.cq = qa;
    } else {
      a.Q = tot[0];
      a.cq = qm;
    }
    a.cr = r;
    a.O = (long long)HW - tot[2];
    a.out_all = (a.O == 0);
    if (a.out_all) a.O = (long long)HW;
    a.b = a.Q / (10 * a.R);
    a.Wt = a.Q + (a.b + 1) * a.R;
    a.kappa = 1.0 / (2.0 * M_PI * 0.25 * (1.0 - std::exp(-4.5)));
    const int N = n_roi + n_out;
    hipLaunchKernelGGL(k_init_draw, dim3((N + 255) / 256), dim3(256), 0, st, a, pick_roi, jit_roi,
                       pick_out, jit_out, xy, chol, rgb, picked);
    return hipGetLastError() == hipSuccess ? GS2D_OK : GS2D_EHIP;
  } catch (...) {
    return GS2D_EHIP;
  }
}
