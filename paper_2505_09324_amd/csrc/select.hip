// P-frame selective optimisation (Sec. 3.2.C): the pixels whose value
// changed by more than a threshold since the reference frame, and the
// reference Gaussians that influence one of them (the pixel lies inside the
// Gaussian's 3-sigma cutoff).  Only those Gaussians are optimised in the
// P-frame.
//
// The reference frame's tile lists (gs2d_project_bin on the reference
// Gaussians) are the pixel-to-Gaussian mapping: a Gaussian influences a
// pixel only if its 3-sigma box meets the pixel's tile.  One workgroup per
// tile: each lane evaluates the change test on its pixels; a tile without a
// changed pixel stops there.  Otherwise the tile's Gaussians are staged (raw
// mean and Cholesky vector, a box test against every sub-block), each
// wavefront walks its list and, for every Gaussian with q <= 9 at one of its
// changed pixels, one lane marks it active.  Both decisions are integer
// results of floating-point tests, taken in FP32 with a fixed order and no
// contraction:
//   changed = |I_t - I_{t-1}| > tau on some channel
//   dx = (x + 1/2) - mx;  dy = (y + 1/2) - my;  u1 = dx / l1;
//   u2 = (dy - l2 u1) / l3;  q = u1 u1 + u2 u2;  influences = q <= 9.
#include <algorithm>

#include "raster_tile.h"

namespace gs2d {
namespace {

template <int NW>
struct SelSmem {
  float4 A[CH];  // mx, my, l1, l2
  float l3[CH];
  uint16_t mask[CH];
  uint16_t id[CH];
  uint16_t list[NW][CH];
};

__device__ inline bool changed_px(const float *__restrict__ a, const float *__restrict__ b,
                                  size_t p, size_t HW, float tau) {
  const float d0 = f32_sub(a[p], b[p]);
  const float d1 = f32_sub(a[HW + p], b[HW + p]);
  const float d2 = f32_sub(a[2 * HW + p], b[2 * HW + p]);
  return fabsf(d0) > tau || fabsf(d1) > tau || fabsf(d2) > tau;
}

template <int TILE, int PPL>
__global__ void __launch_bounds__((Cfg<TILE, PPL>::NT))
k_select(int W, int H, int TX, const uint32_t *__restrict__ keys,
         const int *__restrict__ tile_start, const float *__restrict__ xy,
         const float *__restrict__ chol, const float *__restrict__ frame,
         const float *__restrict__ prev, float tau, uint8_t *__restrict__ active,
         int *__restrict__ n_changed) {
  using C = Cfg<TILE, PPL>;
  __shared__ SelSmem<C::NW> S;
  const int tile = blockIdx.x;
  const int tx = tile % TX, ty = tile / TX;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int px, py0;
  pixel_of_thread<TILE, PPL>(tx, ty, &px, &py0);
  const size_t HW = (size_t)W * H;
  unsigned ch = 0;
#pragma unroll
  for (int r = 0; r < PPL; ++r)
    if (px < W && py0 + r < H && changed_px(frame, prev, (size_t)(py0 + r) * W + px, HW, tau))
      ch |= 1u << r;
  const unsigned long long wch = __ballot(ch != 0);
  if (n_changed) {
    int cnt = __popc(ch);
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if (lane == 0 && cnt) atomicAdd(n_changed, cnt);
  }
  if (!__syncthreads_or(ch != 0)) return;  // the tile has no changed pixel
  const int beg = tile_start[tile], end = tile_start[tile + 1];
  const float pxc = (float)px + 0.5f, pyc0 = (float)py0 + 0.5f;
  const float xlast = (float)W - 0.5f, ylast = (float)H - 0.5f;
  for (int c = beg; c < end; c += CH) {
    const int cnt = min(CH, end - c);
    __syncthreads();
    for (int j = threadIdx.x; j < cnt; j += C::NT) {
      const int id = (int)(keys[c + j] & 0xFFFFu);
      const float mx = xy[2 * id], my = xy[2 * id + 1];
      const float l1 = chol[3 * id], l2 = chol[3 * id + 1], l3 = chol[3 * id + 2];
      S.A[j] = make_float4(mx, my, l1, l2);
      S.l3[j] = l3;
      S.id[j] = (uint16_t)id;
      // box of the q <= 9 ellipse, widened well beyond rounding: a superset
      const float rx = 3.0f * fabsf(l1) * 1.001f + 0.01f;
      const float ry = 3.0f * sqrtf(l2 * l2 + l3 * l3) * 1.001f + 0.01f;
      uint32_t m = 0;
      for (int b = 0; b < C::NW; ++b) {
        const float X0 = (float)(tx * TILE + (b % C::SBX) * 8) + 0.5f;
        const float Y0 = (float)(ty * TILE + (b / C::SBX) * C::SBH) + 0.5f;
        const float X1 = fminf(X0 + 7.0f, xlast), Y1 = fminf(Y0 + (float)(C::SBH - 1), ylast);
        // NaN geometry never reaches here: culled Gaussians have no tiles
        if (mx - rx <= X1 && mx + rx >= X0 && my - ry <= Y1 && my + ry >= Y0) m |= 1u << b;
      }
      S.mask[j] = (uint16_t)m;
    }
    __syncthreads();
    if (!wch) continue;  // no changed pixel in this wavefront's sub-block
    const unsigned long long lt = lanemask_lt();
    int len = 0;
    for (int j0 = 0; j0 < cnt; j0 += 64) {
      const int j = j0 + lane;
      const bool hit = (j < cnt) && ((S.mask[j] >> w) & 1u);
      const unsigned long long bal = __ballot(hit);
      if (hit) S.list[w][len + __popcll(bal & lt)] = (uint16_t)j;
      len += __popcll(bal);
    }
    for (int k = 0; k < len; ++k) {
      const int j = S.list[w][k];
      const float4 A = S.A[j];
      const float l3 = S.l3[j];
      const float u1 = __fdiv_rn(f32_sub(pxc, A.x), A.z);
      const float t = f32_mul(A.w, u1);
      const float u1s = f32_mul(u1, u1);
      bool hit = false;
#pragma unroll
      for (int r = 0; r < PPL; ++r) {
        const float dy = f32_sub(pyc0 + (float)r, A.y);
        const float u2 = __fdiv_rn(f32_sub(dy, t), l3);
        const float q = f32_add(u1s, f32_mul(u2, u2));
        hit |= ((ch >> r) & 1u) && q <= 9.0f;
      }
      if (__ballot(hit) && lane == 0) active[S.id[j]] = 1;
    }
  }
}

__global__ void k_fill_u8(uint8_t *__restrict__ p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void k_zero_counts(int *__restrict__ c) {
  if (threadIdx.x < 2) c[threadIdx.x] = 0;
}

__global__ void __launch_bounds__(256)
k_count_active(const uint8_t *__restrict__ active, int n, int *__restrict__ out) {
  int s = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    s += active[i] != 0;
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0 && s) atomicAdd(out, s);
}

}  // namespace
}  // namespace gs2d

using namespace gs2d;

extern "C" int gs2d_select_changed(const gs2d_shape *shape, void *ws, size_t ws_bytes,
                                   const float *xy, const float *chol, const float *frame,
                                   const float *prev, float tau, uint8_t *active,
                                   int32_t *counts, void *stream) {
  try {
    Layout L;
    if (!shape || !make_layout(*shape, &L)) return GS2D_EINVAL;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return GS2D_EINVAL;
    if (ws_bytes < L.total) return GS2D_ENOSPACE;
    if (!xy || !chol || !frame || !prev || !active) return GS2D_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int nb = std::min((L.N + 255) / 256, 1024);
    hipLaunchKernelGGL(k_fill_u8, dim3(nb), dim3(256), 0, st, active, L.N);
    if (counts) hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(64), 0, st, counts);
    const uint32_t *keys = at<const uint32_t>(ws, L.keys_sorted());
    const int *ts = at<const int>(ws, L.tile_start);
    bool done = false;
#define CASE(TT, PP)                                                                          \
  if (!done && L.T == TT && L.ppl == PP) {                                                    \
    hipLaunchKernelGGL((k_select<TT, PP>), dim3(L.n_tiles), dim3(Cfg<TT, PP>::NT), 0, st, L.W, \
                       L.H, L.TX, keys, ts, xy, chol, frame, prev, tau, active, counts);       \
    done = true;                                                                              \
  }
    CASE(8, 1) CASE(16, 1) CASE(16, 2) CASE(32, 1) CASE(32, 2) CASE(32, 4)
#undef CASE
    if (!done) return GS2D_EINVAL;
    if (counts)
      hipLaunchKernelGGL(k_count_active, dim3(nb), dim3(256), 0, st, active, L.N, counts + 1);
    return hipGetLastError() == hipSuccess ? GS2D_OK : GS2D_EHIP;
  } catch (...) {
    return GS2D_EHIP;
  }
}
