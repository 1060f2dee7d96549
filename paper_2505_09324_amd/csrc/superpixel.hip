// Superpixel initialisation of the ROI Gaussians (Sec. 3.2.A, Fig. 2):
// K-means clustering of the ROI pixels in (x, y, colour) from K seed pixels,
// then one Gaussian per segment from the segment's centre, covariance and
// mean colour.
//
// Clustering (SLIC-style, one grid of cells of side S):
//   S = max(1, rint(sqrt(R / K))) (R ROI pixels, FP64, ties to even),
//   w = (m / S)^2 in FP32; pixel p joins the centre k minimising
//   D = ((dr^2 + dg^2) + db^2) + w (dx^2 + dy^2)  (FP32, this order, no
//   contraction; d = pixel - centre, pixel position = its centre) among the
//   centres whose cell floor(c / S) lies within one cell of the pixel's
//   cell x // S, ties to the lowest k.  Centres are exact means: positions
//   sum / n + 1/2 and colours sum / (n 65536) in FP64 from int64 sums of the
//   pixel indices and of the colours in 1/65536 units; an empty segment keeps
//   its centre.  After the last round each non-empty segment gives
//     mu = mean + 1/2,  L = chol(cov + I/12),
//     c' = colour sum / (2 pi l1 l3 (1 - e^-4.5))
//   (FP64, the order written in seg_gaussian, rounded to FP32 once), so the
//   Gaussian's rendered mass under the q <= 9 cutoff is the segment's colour
//   total; empty segments keep the caller's Gaussian.
//
// Kernels per round: zero the cell counts, count centres per cell, a chunked
// exclusive scan, scatter the centres into cell order, one thread per pixel
// for the assignment (about nine candidates), one wavefront per centre that
// sums the moments of the pixels labelled with it over its 3S x 3S window
// (every such pixel lies in it by the candidate rule), so no atomics touch
// the sums and they are deterministic.  S, the cell grid and w are computed on the
// device: the call never synchronises.
#include <climits>
#include <cmath>

#include "gs2d_internal.h"

namespace gs2d {
namespace {

constexpr int SP_BLOCK = 256;
constexpr int SP_MAX_K = 65536;
constexpr int SP_MAX_ITERS = 100;
constexpr double SP_COLOUR = 65536.0;
constexpr double SP_SCALE_2PI = 65536.0 * 2.0 * 3.14159265358979323846;
constexpr double SP_MASS = 0.98889100346175773;  // 1 - exp(-4.5)

// meta: R, roi_all, S, ncx, ncy, w (float bits)
enum { M_R = 0, M_ALL, M_S, M_NCX, M_NCY, M_W, M_N };

constexpr int SP_CHUNK = 4096;   // cells per block of the chunked scan (16 per thread)

struct SpLayout {
  size_t cen, cell, ends, part, sorted, sidx, labels, meta, total;
  int max_chunks;
};

bool sp_layout(int W, int H, int K, SpLayout *L) {
  if (W < 1 || H < 1 || K < 1 || K > SP_MAX_K) return false;
  const long long HW = (long long)W * H;
  if (HW > (1LL << 28)) return false;
  size_t o = 0;
  auto take = [&o](size_t b) {
    const size_t a = o;
    o = (o + b + 255) & ~(size_t)255;
    return a;
  };
  L->cen = take((size_t)2 * 5 * K * 4);        // two centre sets, SoA x y r g b
  L->cell = take((size_t)K * 4);               // cell of every centre this round
  L->ends = take((size_t)(HW + 1) * 4);        // per-cell counts -> cell ends
  L->max_chunks = (int)((HW + SP_CHUNK - 1) / SP_CHUNK);
  L->part = take((size_t)L->max_chunks * 4);   // chunk totals -> chunk offsets
  L->sorted = take((size_t)5 * K * 4);         // centres in cell order, SoA
  L->sidx = take((size_t)K * 4);               // their indices
  L->labels = take((size_t)HW * 4);
  L->meta = take(M_N * 4);
  L->total = o;
  return true;
}

__device__ inline long long colour_code(float v) { return (long long)rint((double)v * SP_COLOUR); }

__global__ void k_sp_zero_meta(int *__restrict__ meta) {
  if (threadIdx.x < M_N) meta[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(SP_BLOCK)
k_sp_count_roi(size_t HW, const uint8_t *__restrict__ mask, int *__restrict__ meta) {
  __shared__ int red[SP_BLOCK / 64];
  int c = 0;
  for (size_t p = blockIdx.x * (size_t)SP_BLOCK + threadIdx.x; p < HW;
       p += (size_t)gridDim.x * SP_BLOCK)
    c += mask[p] != 0;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int v = 0; v < SP_BLOCK / 64; ++v) t += red[v];
    if (t) atomicAdd(&meta[M_R], t);
  }
}

__global__ void k_sp_setup(int W, int H, int K, float m, int *__restrict__ meta) {
  if (threadIdx.x != 0) return;
  long long R = meta[M_R];
  const int all = R == 0;
  if (all) R = (long long)W * H;
  const int S = max(1, (int)rint(sqrt((double)R / (double)K)));
  const float r = __fdiv_rn(m, (float)S);
  const float w = f32_mul(r, r);
  meta[M_ALL] = all;
  meta[M_S] = S;
  meta[M_NCX] = (W + S - 1) / S;
  meta[M_NCY] = (H + S - 1) / S;
  meta[M_W] = __float_as_int(w);
}

__global__ void __launch_bounds__(SP_BLOCK)
k_sp_seed(int W, int H, int K, const float *__restrict__ T, const int32_t *__restrict__ seeds,
          float *__restrict__ cen) {
  const int k = blockIdx.x * SP_BLOCK + threadIdx.x;
  if (k >= K) return;
  const size_t HW = (size_t)W * H;
  const int p = min(max(seeds[k], 0), (int)(HW - 1));
  cen[k] = (float)(p % W) + 0.5f;
  cen[K + k] = (float)(p / W) + 0.5f;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    cen[(2 + c) * K + k] = (float)((double)colour_code(T[c * HW + p]) / SP_COLOUR);
}

__global__ void __launch_bounds__(SP_BLOCK)
k_sp_zero_cells(const int *__restrict__ meta, int *__restrict__ ends) {
  const int n = meta[M_NCX] * meta[M_NCY] + 1;
  for (int i = blockIdx.x * SP_BLOCK + threadIdx.x; i < n; i += gridDim.x * SP_BLOCK) ends[i] = 0;
}

__global__ void __launch_bounds__(SP_BLOCK)
k_sp_cells(int K, const float *__restrict__ cen, const int *__restrict__ meta,
           int *__restrict__ cell, int *__restrict__ ends) {
  const int k = blockIdx.x * SP_BLOCK + threadIdx.x;
  if (k >= K) return;
  const float fS = (float)meta[M_S];
  const int ncx = meta[M_NCX], ncy = meta[M_NCY];
  // centres are means of pixel centres, so these lie inside the grid; the
  // clamp only keeps the index in range
  const int cx = min(max((int)floorf(__fdiv_rn(cen[k], fS)), 0), ncx - 1);
  const int cy = min(max((int)floorf(__fdiv_rn(cen[K + k], fS)), 0), ncy - 1);
  const int c = cy * ncx + cx;
  cell[k] = c;
  atomicAdd(&ends[c], 1);
}

// Exclusive scan of the ncells counts in place, in chunks of SP_CHUNK cells:
// chunk totals, one block that turns them into chunk offsets, then each
// chunk's own scan plus its offset.  Blocks past the last chunk return.
__device__ inline int block_excl_scan(int v, int *red, int *total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) red[wid] = x;
  __syncthreads();
  int off = 0, all = 0;
  for (int w = 0; w < SP_BLOCK / 64; ++w) {
    if (w < wid) off += red[w];
    all += red[w];
  }
  __syncthreads();
  *total = all;
  return off + x - v;
}

__global__ void __launch_bounds__(SP_BLOCK)
k_sp_scan_sums(const int *__restrict__ meta, const int *__restrict__ ends, int *__restrict__ part) {
  __shared__ int red[SP_BLOCK / 64];
  const int n = meta[M_NCX] * meta[M_NCY];
  const int b0 = blockIdx.x * SP_CHUNK;
  if (b0 >= n) return;
  constexpr int PER = SP_CHUNK / SP_BLOCK;
  const int e0 = b0 + threadIdx.x * PER;
  int s = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j)
    if (e0 + j < n) s += ends[e0 + j];
  int total;
  block_excl_scan(s, red, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ void __launch_bounds__(SP_BLOCK)
k_sp_scan_top(const int *__restrict__ meta, int *__restrict__ part) {
  __shared__ int red[SP_BLOCK / 64];
  const int n = (meta[M_NCX] * meta[M_NCY] + SP_CHUNK - 1) / SP_CHUNK;
  const int per = (n + SP_BLOCK - 1) / SP_BLOCK;
  const int b = threadIdx.x * per, e = min(b + per, n);
  int s = 0;
  for (int i = b; i < e; ++i) s += part[i];
  int total;
  int run = block_excl_scan(s, red, &total);
  for (int i = b; i < e; ++i) {
    const int c = part[i];
    part[i] = run;
    run += c;
  }
}

__global__ void __launch_bounds__(SP_BLOCK)
k_sp_scan_apply(const int *__restrict__ meta, int *__restrict__ ends,
                const int *__restrict__ part) {
  __shared__ int red[SP_BLOCK / 64];
  const int n = meta[M_NCX] * meta[M_NCY];
  const int b0 = blockIdx.x * SP_CHUNK;
  if (b0 >= n) return;
  constexpr int PER = SP_CHUNK / SP_BLOCK;
  const int e0 = b0 + threadIdx.x * PER;
  int v[PER];
  int s = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    v[j] = e0 + j < n ? ends[e0 + j] : 0;
    s += v[j];
  }
  int total;
  int run = part[blockIdx.x] + block_excl_scan(s, red, &total);
#pragma unroll
  for (int j = 0; j < PER; ++j)
    if (e0 + j < n) {
      ends[e0 + j] = run;
      run += v[j];
    }
}

// After this, cell c holds slots [c ? ends[c-1] : 0, ends[c]).
__global__ void __launch_bounds__(SP_BLOCK)
k_sp_scatter(int K, const float *__restrict__ cen, const int *__restrict__ cell,
             int *__restrict__ ends, float *__restrict__ sorted, int *__restrict__ sidx) {
  const int k = blockIdx.x * SP_BLOCK + threadIdx.x;
  if (k >= K) return;
  const int pos = atomicAdd(&ends[cell[k]], 1);
#pragma unroll
  for (int a = 0; a < 5; ++a) sorted[a * K + pos] = cen[a * K + k];
  sidx[pos] = k;
}

__global__ void __launch_bounds__(SP_BLOCK)
k_sp_assign(int W, int H, int K, const float *__restrict__ T, const uint8_t *__restrict__ mask,
            const int *__restrict__ meta, const int *__restrict__ ends,
            const float *__restrict__ sorted, const int *__restrict__ sidx,
            int32_t *__restrict__ labels) {
  const size_t HW = (size_t)W * H;
  const int S = meta[M_S], ncx = meta[M_NCX], ncy = meta[M_NCY], all = meta[M_ALL];
  const float w = __int_as_float(meta[M_W]);
  for (size_t p = blockIdx.x * (size_t)SP_BLOCK + threadIdx.x; p < HW;
       p += (size_t)gridDim.x * SP_BLOCK) {
    int best_k = -1;
    if (all || mask[p]) {
      const int x = (int)(p % W), y = (int)(p / W);
      const float px = (float)x + 0.5f, py = (float)y + 0.5f;
      const float r = T[p], g = T[HW + p], bl = T[2 * HW + p];
      const int gx = x / S, gy = y / S;
      float best = INFINITY;
      best_k = INT_MAX;
      for (int cy = max(gy - 1, 0); cy <= min(gy + 1, ncy - 1); ++cy)
        for (int cx = max(gx - 1, 0); cx <= min(gx + 1, ncx - 1); ++cx) {
          const int c = cy * ncx + cx;
          const int e = ends[c];
          for (int i = c ? ends[c - 1] : 0; i < e; ++i) {
            const float dr = f32_sub(r, sorted[2 * K + i]);
            const float dg = f32_sub(g, sorted[3 * K + i]);
            const float db = f32_sub(bl, sorted[4 * K + i]);
            const float dx = f32_sub(px, sorted[i]);
            const float dy = f32_sub(py, sorted[K + i]);
            const float dcol = f32_add(f32_add(f32_mul(dr, dr), f32_mul(dg, dg)), f32_mul(db, db));
            const float dpos = f32_add(f32_mul(dx, dx), f32_mul(dy, dy));
            const float D = f32_add(dcol, f32_mul(w, dpos));
            const int k = sidx[i];
            if (D < best || (D == best && k < best_k)) best = D, best_k = k;
          }
        }
      if (best_k == INT_MAX) best_k = -1;
    }
    labels[p] = best_k;
  }
}

// Segment Gaussian from exact moments s = n, Sx, Sy, Sxx, Sxy, Syy, Sr, Sg, Sb.
__device__ void seg_gaussian(const long long *s, float *xy, float *chol, float *rgb) {
#pragma clang fp contract(off)
  const double n = (double)s[0];
  const double ex = (double)s[1] / n, ey = (double)s[2] / n;
  const double vxx = ((double)s[3] / n - ex * ex) + 1.0 / 12.0;
  const double vxy = (double)s[4] / n - ex * ey;
  const double vyy = ((double)s[5] / n - ey * ey) + 1.0 / 12.0;
  const double l1 = sqrt(vxx);
  const double l2 = vxy / l1;
  const double l3 = sqrt(vyy - l2 * l2);
  const double den = ((SP_SCALE_2PI * l1) * l3) * SP_MASS;
  xy[0] = (float)(ex + 0.5);
  xy[1] = (float)(ey + 0.5);
  chol[0] = (float)l1;
  chol[1] = (float)l2;
  chol[2] = (float)l3;
#pragma unroll
  for (int c = 0; c < 3; ++c) rgb[c] = (float)((double)s[6 + c] / den);
}

__device__ void seg_centre(const long long *s, int K, int k, float *dst) {
#pragma clang fp contract(off)
  const double n = (double)s[0];
  dst[k] = (float)((double)s[1] / n + 0.5);
  dst[K + k] = (float)((double)s[2] / n + 0.5);
#pragma unroll
  for (int c = 0; c < 3; ++c) dst[(2 + c) * K + k] = (float)((double)s[6 + c] / (n * SP_COLOUR));
}

// Wavefront k (four per block): moments of the pixels labelled k in its
// window; new centre; on the last round also the segment Gaussian.
constexpr int SP_GATHER_WAVES = SP_BLOCK / 64;

__global__ void __launch_bounds__(SP_BLOCK)
k_sp_gather(int W, int H, int K, const float *__restrict__ T, const int *__restrict__ meta,
            const int *__restrict__ cell, const int32_t *__restrict__ labels,
            const float *__restrict__ src, float *__restrict__ dst, int last,
            float *__restrict__ xy, float *__restrict__ chol, float *__restrict__ rgb) {
  const int k = blockIdx.x * SP_GATHER_WAVES + (threadIdx.x >> 6);
  if (k >= K) return;  // whole wavefronts; the kernel has no barrier
  const int lane = threadIdx.x & 63;
  const size_t HW = (size_t)W * H;
  const int S = meta[M_S], ncx = meta[M_NCX];
  const int ckx = cell[k] % ncx, cky = cell[k] / ncx;
  const int x0 = max((ckx - 1) * S, 0), x1 = min((ckx + 2) * S, W);
  const int y0 = max((cky - 1) * S, 0), y1 = min((cky + 2) * S, H);
  const int ww = x1 - x0;
  const long long area = (long long)ww * (y1 - y0);
  long long s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (long long i = lane; i < area; i += 64) {
    const int x = x0 + (int)(i % ww), y = y0 + (int)(i / ww);
    const size_t p = (size_t)y * W + x;
    if (labels[p] != k) continue;
    s[0] += 1;
    s[1] += x;
    s[2] += y;
    s[3] += (long long)x * x;
    s[4] += (long long)x * y;
    s[5] += (long long)y * y;
#pragma unroll
    for (int c = 0; c < 3; ++c) s[6 + c] += colour_code(T[c * HW + p]);
  }
#pragma unroll
  for (int j = 0; j < 9; ++j)
    for (int o = 32; o > 0; o >>= 1) s[j] += __shfl_xor(s[j], o, 64);
  if (lane != 0) return;
  if (s[0] == 0) {
#pragma unroll
    for (int a = 0; a < 5; ++a) dst[a * K + k] = src[a * K + k];
    return;
  }
  seg_centre(s, K, k, dst);
  if (last) seg_gaussian(s, xy + 2 * k, chol + 3 * k, rgb + 3 * k);
}

unsigned grid_for(size_t n) { return (unsigned)std::min<size_t>((n + SP_BLOCK - 1) / SP_BLOCK, 8192); }

}  // namespace
}  // namespace gs2d

using namespace gs2d;

extern "C" size_t gs2d_superpixel_workspace_bytes(int32_t W, int32_t H, int32_t K) {
  SpLayout L;
  return sp_layout(W, H, K, &L) ? L.total : 0;
}

extern "C" int gs2d_init_superpixel(int32_t W, int32_t H, const float *target,
                                    const uint8_t *roi_mask, int32_t K, const int32_t *seeds,
                                    int32_t iters, float compactness, float *xy, float *chol,
                                    float *rgb, int32_t *labels, float *centres, void *ws,
                                    size_t ws_bytes, void *stream) {
  try {
    SpLayout L;
    if (!sp_layout(W, H, K, &L)) return GS2D_EINVAL;
    if (iters < 1 || iters > SP_MAX_ITERS || !(compactness > 0.f) || !std::isfinite(compactness))
      return GS2D_EINVAL;
    if (!target || !roi_mask || !seeds || !xy || !chol || !rgb || !ws) return GS2D_EINVAL;
    if (reinterpret_cast<uintptr_t>(ws) & 255) return GS2D_EINVAL;
    if (ws_bytes < L.total) return GS2D_ENOSPACE;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const size_t HW = (size_t)W * H;
    float *cen = at<float>(ws, L.cen);
    int *cell = at<int>(ws, L.cell), *ends = at<int>(ws, L.ends), *sidx = at<int>(ws, L.sidx);
    int *part = at<int>(ws, L.part);
    float *sorted = at<float>(ws, L.sorted);
    int32_t *lab = labels ? labels : at<int32_t>(ws, L.labels);
    int *meta = at<int>(ws, L.meta);
    const unsigned gk = (unsigned)((K + SP_BLOCK - 1) / SP_BLOCK);
    hipLaunchKernelGGL(k_sp_zero_meta, dim3(1), dim3(64), 0, st, meta);
    hipLaunchKernelGGL(k_sp_count_roi, dim3(std::min(grid_for(HW), 1024u)), dim3(SP_BLOCK), 0, st,
                       HW, roi_mask, meta);
    hipLaunchKernelGGL(k_sp_setup, dim3(1), dim3(64), 0, st, W, H, K, compactness, meta);
    hipLaunchKernelGGL(k_sp_seed, dim3(gk), dim3(SP_BLOCK), 0, st, W, H, K, target, seeds, cen);
    for (int it = 0; it < iters; ++it) {
      float *src = cen + (size_t)(it & 1) * 5 * K, *dst = cen + (size_t)((it + 1) & 1) * 5 * K;
      hipLaunchKernelGGL(k_sp_zero_cells, dim3(grid_for(HW + 1)), dim3(SP_BLOCK), 0, st, meta,
                         ends);
      hipLaunchKernelGGL(k_sp_cells, dim3(gk), dim3(SP_BLOCK), 0, st, K, src, meta, cell, ends);
      hipLaunchKernelGGL(k_sp_scan_sums, dim3(L.max_chunks), dim3(SP_BLOCK), 0, st, meta, ends,
                         part);
      hipLaunchKernelGGL(k_sp_scan_top, dim3(1), dim3(SP_BLOCK), 0, st, meta, part);
      hipLaunchKernelGGL(k_sp_scan_apply, dim3(L.max_chunks), dim3(SP_BLOCK), 0, st, meta, ends,
                         part);
      hipLaunchKernelGGL(k_sp_scatter, dim3(gk), dim3(SP_BLOCK), 0, st, K, src, cell, ends, sorted,
                         sidx);
      hipLaunchKernelGGL(k_sp_assign, dim3(grid_for(HW)), dim3(SP_BLOCK), 0, st, W, H, K, target,
                         roi_mask, meta, ends, sorted, sidx, lab);
      hipLaunchKernelGGL(k_sp_gather, dim3((K + SP_GATHER_WAVES - 1) / SP_GATHER_WAVES),
                         dim3(SP_BLOCK), 0, st, W, H, K, target, meta, cell,
                         lab, src, dst, (int)(it == iters - 1), xy, chol, rgb);
    }
    if (centres) {
      const size_t bytes = (size_t)5 * K * sizeof(float);
      if (hipMemcpyAsync(centres, cen + (size_t)((iters - 1) & 1) * 5 * K, bytes,
                         hipMemcpyDeviceToDevice, st) != hipSuccess ||
          hipMemcpyAsync(centres + (size_t)5 * K, cen + (size_t)(iters & 1) * 5 * K, bytes,
                         hipMemcpyDeviceToDevice, st) != hipSuccess)
        return GS2D_EHIP;
    }
    return hipGetLastError() == hipSuccess ? GS2D_OK : GS2D_EHIP;
  } catch (...) {
    return GS2D_EHIP;
  }
}
