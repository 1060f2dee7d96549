// Tile rasteriser for Eq. 2 (accumulated summation, Sec. 3.1) and its
// backward pass.
//
// One workgroup per TILE x TILE screen tile.  Each wavefront owns a sub-block
// 8 pixels wide and 8*PPL pixels tall: lane (lx, ly) = (lane & 7, lane >> 3)
// handles the PPL vertically adjacent pixels (x0 + lx, y0 + ly*PPL + k),
// which share d_x, u1 = d_x / l1 and u1^2.  The tile's Gaussian list is
// staged through LDS in chunks; while staging, each Gaussian's 3-sigma box
// and then its cutoff ellipse are tested against every sub-block, and each
// wavefront compacts the chunk into its own list of the Gaussians that can
// reach its sub-block's pixels.
//
// Per (pixel, Gaussian), with d = (x+1/2, y+1/2) - mu and u = L^-1 d:
//   u1 = d1 / l1;  u2 = (d2 - l2 u1) / l3;  q = u1^2 + u2^2
//   w = exp(-q/2) if q <= 9 else 0;  C += c' w
// Backward, with g = dL/dC at the pixel, s = (g . c') w, v = L^-T u:
//   dL/dmu += s v;  dL/dl1 += s v1 u1;  dL/dl2 += s v2 u1;  dL/dl3 += s v2 u2;
//   dL/dc' += g w.
// The eight per-lane sums of one Gaussian are reduced across the wavefront
// by a transposing butterfly (each exchange halves the values a lane
// carries), added into an LDS accumulator shared by the tile's wavefronts,
// and flushed with one global atomic per (tile, Gaussian, parameter).
#include "raster_tile.h"

namespace gs2d {

// ----------------------------------------------------------------- forward --
template <int TILE, int PPL>
__global__ void __launch_bounds__((Cfg<TILE, PPL>::NT)) GS2D_RASTER_OCCUPANCY
k_render_fwd(FrameArgs f, const float *__restrict__ target, float *__restrict__ img,
             float *__restrict__ dl_dimg, float *__restrict__ loss_part, float grad_scale) {
  using C = Cfg<TILE, PPL>;
  __shared__ Smem<C::NW> S;
  const int tile = blockIdx.x;
  const int tx = tile % f.TX, ty = tile / f.TX;
  const int beg = f.tile_start[tile], end = f.tile_start[tile + 1];
  int px, py0;
  pixel_of_thread<TILE, PPL>(tx, ty, &px, &py0);
  const float pxc = (float)px + 0.5f, pyc0 = (float)py0 + 0.5f;
  const unsigned inside = inside_mask<PPL>(f, px, py0);
  float acc[PPL][3] = {};
  for (int c = beg; c < end; c += CH) {
    const int cnt = min(CH, end - c);
    __syncthreads();
    stage_chunk<TILE, PPL>(S, f.keys, c, cnt, tx, ty, f.W, f.H, f.geom, f.rgb);
    __syncthreads();
    const int len = compact_chunk<C::NW>(S, cnt);
    __syncthreads();
    fwd_chunk<C::NW, PPL, false>(S, len, pxc, pyc0, inside, acc);
  }
  float l = 0.f;
  const size_t HW = (size_t)f.W * f.H;
#pragma unroll
  for (int r = 0; r < PPL; ++r) {
    if (!((inside >> r) & 1u)) continue;
    const size_t p = (size_t)(py0 + r) * f.W + px;
    if (img) {
      img[p] = acc[r][0];
      img[HW + p] = acc[r][1];
      img[2 * HW + p] = acc[r][2];
    }
    if (target) {
      const float r0 = acc[r][0] - target[p], r1 = acc[r][1] - target[HW + p],
                  r2 = acc[r][2] - target[2 * HW + p];
      l += r0 * r0 + r1 * r1 + r2 * r2;
      if (dl_dimg) {
        dl_dimg[p] = r0 * grad_scale;
        dl_dimg[HW + p] = r1 * grad_scale;
        dl_dimg[2 * HW + p] = r2 * grad_scale;
      }
    }
  }
  if (loss_part) wave_loss(l, loss_part + tile * C::NW + (threadIdx.x >> 6));
}

// ---------------------------------------------------------------- backward --
template <int TILE, int PPL>
__global__ void __launch_bounds__((Cfg<TILE, PPL>::NT)) GS2D_RASTER_OCCUPANCY
k_render_bwd(FrameArgs f, const float *__restrict__ dl_dimg, float *__restrict__ g_xy,
             float *__restrict__ g_chol, float *__restrict__ g_rgb) {
  using C = Cfg<TILE, PPL>;
  __shared__ Smem<C::NW> S;
  __shared__ float acc[CH * 8];
  const int tile = blockIdx.x;
  const int tx = tile % f.TX, ty = tile / f.TX;
  const int beg = f.tile_start[tile], end = f.tile_start[tile + 1];
  if (beg >= end) return;
  int px, py0;
  pixel_of_thread<TILE, PPL>(tx, ty, &px, &py0);
  const float pxc = (float)px + 0.5f, pyc0 = (float)py0 + 0.5f;
  const unsigned inside = inside_mask<PPL>(f, px, py0);
  float g[PPL][3];
  const size_t HW = (size_t)f.W * f.H;
#pragma unroll
  for (int r = 0; r < PPL; ++r) {
    g[r][0] = g[r][1] = g[r][2] = 0.f;
    if ((inside >> r) & 1u) {
      const size_t p = (size_t)(py0 + r) * f.W + px;
      g[r][0] = dl_dimg[p];
      g[r][1] = dl_dimg[HW + p];
      g[r][2] = dl_dimg[2 * HW + p];
    }
  }
  for (int c = beg; c < end; c += CH) {
    const int cnt = min(CH, end - c);
    __syncthreads();
    stage_chunk<TILE, PPL>(S, f.keys, c, cnt, tx, ty, f.W, f.H, f.geom, f.rgb);
    for (int i = threadIdx.x; i < CH * 8; i += C::NT) acc[i] = 0.f;
    __syncthreads();
    const int len = compact_chunk<C::NW>(S, cnt);
    __syncthreads();
    bwd_chunk<C::NW, PPL, false>(S, acc, len, pxc, pyc0, g);
    __syncthreads();
    flush_grads<C::NT, C::NW>(S, acc, cnt, g_xy, g_chol, g_rgb);
  }
}

// ------------------------------------------- fused forward + loss + backward --
template <int TILE, int PPL>
__global__ void __launch_bounds__((Cfg<TILE, PPL>::NT)) GS2D_RASTER_OCCUPANCY
k_render_fused(FrameArgs f, const float *__restrict__ target, float *__restrict__ loss_part,
               float grad_scale, float *__restrict__ g_xy, float *__restrict__ g_chol,
               float *__restrict__ g_rgb) {
  using C = Cfg<TILE, PPL>;
  __shared__ Smem<C::NW> S;
  __shared__ float acc[CH * 8];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (f.lazy_misc && f.lazy_misc[MISC_STALE]) {
      const bool ok = !(f.lazy_misc[MISC_STICKY] & (int)STATUS_STALLED);
      f.lazy_misc[MISC_LISTS_LO] = ok ? (int)f.sig_lo : 0;
      f.lazy_misc[MISC_LISTS_HI] = ok ? (int)f.sig_hi : 0;
      f.lazy_misc[MISC_STALE] = 0;
    }
    if (f.tick) *f.tick += 1;
  }
  fused_tile<TILE, PPL, true, true>(S, acc, f, (int)blockIdx.x, target,
                                    loss_part + blockIdx.x * C::NW, grad_scale, g_xy, g_chol,
                                    g_rgb);
}

// ------------------------------------------------- in-cutoff pair counting --
// Number of (pixel, Gaussian) pairs with q <= 9 inside the frame: the terms
// Eq. 2 actually sums (the algorithmic work of one render).
template <int TILE>
__global__ void __launch_bounds__((Cfg<TILE, 1>::NT))
k_count_pairs(FrameArgs f, unsigned long long *__restrict__ out) {
  using C = Cfg<TILE, 1>;
  __shared__ Smem<C::NW> S;
  const int tile = blockIdx.x;
  const int tx = tile % f.TX, ty = tile / f.TX;
  const int beg = f.tile_start[tile], end = f.tile_start[tile + 1];
  int px, py;
  pixel_of_thread<TILE, 1>(tx, ty, &px, &py);
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const bool inside = px < f.W && py < f.H;
  const int w = threadIdx.x >> 6;
  unsigned int n = 0;
  for (int c = beg; c < end; c += CH) {
    const int cnt = min(CH, end - c);
    __syncthreads();
    stage_chunk<TILE, 1>(S, f.keys, c, cnt, tx, ty, f.W, f.H, f.geom, nullptr);
    __syncthreads();
    const int len = compact_chunk<C::NW>(S, cnt);
    __syncthreads();
    for (int k = 0; k < len; ++k) {
      const int j = S.list[w][k];
      const float4 A = S.A[j], B = S.B[j];
      const float u1 = (pxc - A.x) * A.z;
      const float u2 = ((pyc - A.y) - A.w * u1) * B.x;
      n += (inside && u1 * u1 + u2 * u2 <= CUTOFF_QS) ? 1u : 0u;
    }
  }
  for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
  if ((threadIdx.x & 63) == 0 && n) atomicAdd(out, (unsigned long long)n);
}

// ------------------------------------------------------------- loss reduce --
__global__ void __launch_bounds__(1024)
k_loss_reduce(const float *__restrict__ part, int n, float scale, float *__restrict__ out) {
  __shared__ double red[16];
  double s = 0.0;
  s = thread_sum_parts(part, n);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w];
    *out = (float)(t * (double)scale);
  }
}

// ------------------------------------------------------------------ launch --
static FrameArgs frame_args(const Layout &L, void *ws, const float *rgb) {
  FrameArgs f;
  f.W = L.W;
  f.H = L.H;
  f.TX = L.TX;
  f.geom = at<const float4>(ws, L.geom);
  f.keys = at<const uint32_t>(ws, L.keys_sorted());
  f.tile_start = at<const int>(ws, L.tile_start);
  f.rgb = rgb;
  f.active = nullptr;
  f.lazy_misc = nullptr;
  f.sig_lo = f.sig_hi = 0;
  f.tick = nullptr;
  return f;
}

static float grad_scale(const Layout &L) { return (float)(2.0 / (3.0 * L.W * (double)L.H)); }

// (tile, pixels per lane) variants that are compiled.
#define GS2D_VARIANTS(X) X(8, 1) X(16, 1) X(16, 2) X(32, 1) X(32, 2) X(32, 4)

hipError_t launch_render_fwd(const Layout &L, void *ws, const float *rgb, const float *target,
                             float *img, float *dl_dimg, hipStream_t st) {
  FrameArgs f = frame_args(L, ws, rgb);
  float *lp = target ? at<float>(ws, L.loss_part) : nullptr;
  bool done = false;
#define CALL(TT, PP)                                                                       \
  if (!done && L.T == TT && L.ppl == PP) {                                                 \
    hipLaunchKernelGGL((k_render_fwd<TT, PP>), dim3(L.n_tiles), dim3(Cfg<TT, PP>::NT), 0, st, \
                       f, target, img, dl_dimg, lp, grad_scale(L));                        \
    done = true;                                                                           \
  }
  GS2D_VARIANTS(CALL)
#undef CALL
  return done ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t launch_render_bwd(const Layout &L, void *ws, const float *rgb, const float *dl_dimg,
                             float *g_xy, float *g_chol, float *g_rgb, hipStream_t st) {
  FrameArgs f = frame_args(L, ws, rgb);
  bool done = false;
#define CALL(TT, PP)                                                                       \
  if (!done && L.T == TT && L.ppl == PP) {                                                 \
    hipLaunchKernelGGL((k_render_bwd<TT, PP>), dim3(L.n_tiles), dim3(Cfg<TT, PP>::NT), 0, st, \
                       f, dl_dimg, g_xy, g_chol, g_rgb);                                   \
    done = true;                                                                           \
  }
  GS2D_VARIANTS(CALL)
#undef CALL
  return done ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t launch_render_fused(const Layout &L, void *ws, const float *rgb, const float *target,
                               float *g_xy, float *g_chol, float *g_rgb, hipStream_t st,
                               const uint8_t *active, bool lazy, int32_t *tick) {
  FrameArgs f = frame_args(L, ws, rgb);
  f.active = active;
  if (lazy) {
    f.lazy_misc = at<int>(ws, L.misc);
    f.sig_lo = L.sig_lo;
    f.sig_hi = L.sig_hi;
  }
  f.tick = tick;
  float *lp = at<float>(ws, L.loss_part);
  bool done = false;
#define CALL(TT, PP)                                                                           \
  if (!done && L.T == TT && L.ppl == PP) {                                                     \
    hipLaunchKernelGGL((k_render_fused<TT, PP>), dim3(L.n_tiles), dim3(Cfg<TT, PP>::NT), 0, st, \
                       f, target, lp, grad_scale(L), g_xy, g_chol, g_rgb);                     \
    done = true;                                                                               \
  }
  GS2D_VARIANTS(CALL)
#undef CALL
  return done ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t launch_count_pairs(const Layout &L, void *ws, unsigned long long *out, hipStream_t st) {
  FrameArgs f = frame_args(L, ws, nullptr);
  hipError_t e = launch_fill_zero_u32(reinterpret_cast<uint32_t *>(out), 2, st);
  if (e != hipSuccess) return e;
  switch (L.T) {
    case 8: hipLaunchKernelGGL(k_count_pairs<8>, dim3(L.n_tiles), dim3(64), 0, st, f, out); break;
    case 16: hipLaunchKernelGGL(k_count_pairs<16>, dim3(L.n_tiles), dim3(256), 0, st, f, out); break;
    case 32: hipLaunchKernelGGL(k_count_pairs<32>, dim3(L.n_tiles), dim3(1024), 0, st, f, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_loss_reduce(const Layout &L, void *ws, float *loss, hipStream_t st) {
  hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(1024), 0, st, at<const float>(ws, L.loss_part),
                     L.loss_parts, (float)(1.0 / (3.0 * L.W * (double)L.H)), loss);
  return hipGetLastError();
}

}  // namespace gs2d
