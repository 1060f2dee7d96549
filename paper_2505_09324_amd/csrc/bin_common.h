// Device-side building blocks of projection and tile binning, shared by the
// one-frame kernels (bin.hip) and the batched ones (batch.hip).
#pragma once

#include "gs2d_internal.h"

namespace gs2d {

constexpr int SCAN_PER = 64;  // max elements per scan thread: 64 * 1024 = 65536

// Projection of Gaussian n (index into xy/chol and the outputs).
// counts[n] = number of tiles met, or -1 for a culled Gaussian (the scan
// turns -1 into 0 and counts the culls).  geom[n] = {mx, my, 1/l1, l2, 1/l3,
// rx, ry, 0}; rect[n] = {tx0, ty0, tx1, ty1}.  The box/rectangle arithmetic
// uses the _rn intrinsics so that no multiply and add are contracted: the
// tile decision must match its FP32 specification exactly.
__device__ inline void project_gaussian(int n, int TX, int TY, float inv_tile,
                                        const float *__restrict__ xy,
                                        const float *__restrict__ chol, float4 *__restrict__ geom,
                                        int4 *__restrict__ rect, int *__restrict__ counts) {
  const float mx = xy[2 * n + 0], my = xy[2 * n + 1];
  const float l1 = chol[3 * n + 0], l2 = chol[3 * n + 1], l3 = chol[3 * n + 2];
  const float tiny = 6.103515625e-05f;  // 2^-14
  const bool finite = isfinite(mx) && isfinite(my) && isfinite(l1) && isfinite(l2) && isfinite(l3);
  if (!finite || !(fabsf(l1) >= tiny) || !(fabsf(l3) >= tiny)) {
    counts[n] = -1;
    rect[n] = make_int4(0, 0, -1, -1);
    geom[2 * n + 0] = make_float4(0.f, 0.f, 0.f, 0.f);
    geom[2 * n + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  const float a = __fmul_rn(l2, l2);
  const float b = __fmul_rn(l3, l3);
  const float s = __fadd_rn(a, b);
  const float r = __fsqrt_rn(s);
  const float ry = __fmul_rn(3.0f, r);
  const float rx = __fmul_rn(3.0f, fabsf(l1));
  const float xlo = __fsub_rn(mx, rx), xhi = __fadd_rn(mx, rx);
  const float ylo = __fsub_rn(my, ry), yhi = __fadd_rn(my, ry);
  // division by a power of two == multiplication by its exact reciprocal
  const float fx0 = floorf(__fmul_rn(xlo, inv_tile)), fx1 = floorf(__fmul_rn(xhi, inv_tile));
  const float fy0 = floorf(__fmul_rn(ylo, inv_tile)), fy1 = floorf(__fmul_rn(yhi, inv_tile));
  const float lastx = (float)(TX - 1), lasty = (float)(TY - 1);
  int cnt = 0;
  int4 rc = make_int4(0, 0, -1, -1);
  if (!(fx1 < 0.f || fx0 > lastx || fy1 < 0.f || fy0 > lasty)) {
    rc.x = (int)fmaxf(fx0, 0.f);
    rc.z = (int)fminf(fx1, lastx);
    rc.y = (int)fmaxf(fy0, 0.f);
    rc.w = (int)fminf(fy1, lasty);
    cnt = (rc.z - rc.x + 1) * (rc.w - rc.y + 1);
  }
  counts[n] = cnt;
  rect[n] = rc;
  geom[2 * n + 0] = make_float4(mx, my, __fdiv_rn(1.0f, l1), l2);
  geom[2 * n + 1] = make_float4(__fdiv_rn(1.0f, l3), rx, ry, 0.f);
}

// ------------------------------------------------------------ block scan --
// Exclusive scan of one 64-bit value per thread across a block of NT
// threads.  `lds` holds NT/64 entries.  Returns the exclusive prefix and the
// block total.
template <int NT>
__device__ inline long long block_exclusive_scan(long long v, long long *total, long long *lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int NW = NT / 64;
  long long x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    long long y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[w] = x;
  __syncthreads();
  if (w == 0) {
    long long s = (lane < NW) ? lds[lane] : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      long long y = __shfl_up(s, o, 64);
      if (lane >= o) s += y;
    }
    if (lane < NW) lds[lane] = s;
  }
  __syncthreads();
  const long long before = (w > 0) ? lds[w - 1] : 0;
  *total = lds[NW - 1];
  __syncthreads();
  return before + x - v;
}

// Chunk of the key array owned by sort block b (a multiple of SORT_BLOCK).
__device__ inline void sort_chunk(int n, int G, int b, int *beg, int *end) {
  int chunk = (n + G - 1) / G;
  chunk = (chunk + SORT_BLOCK - 1) / SORT_BLOCK * SORT_BLOCK;
  *beg = min(n, b * chunk);
  *end = min(n, *beg + chunk);
}

}  // namespace gs2d
