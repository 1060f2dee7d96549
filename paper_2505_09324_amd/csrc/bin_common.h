// Device-side building blocks of projection and tile binning, shared by the
// one-frame kernels (bin.hip) and the batched ones (batch.hip).
#pragma once

#include "gs2d_internal.h"

namespace gs2d {

constexpr int BIN_BLOCK = 256;  // threads of the projection / emission blocks
// Radix digit-offset scan: SORT_MAX_BLOCKS * RADIX entries over SCAN_BLOCK
// threads, at most this many per thread (kept in 32-bit registers).
constexpr int RADIX_SCAN_PER = (SORT_MAX_BLOCKS * RADIX + SCAN_BLOCK - 1) / SCAN_BLOCK;
static_assert(RADIX_SCAN_PER * (SCAN_BLOCK / 64) <= 64 * 8, "wave-total table too small");

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


// Exclusive scan of one int per thread over a block of NT threads; `lds`
// holds NT/64 ints.  Returns the prefix; *total receives the block sum.
template <int NT>
__device__ inline int block_exclusive_scan_i32(int v, int *total, int *lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int NW = NT / 64;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[w] = x;
  __syncthreads();
  if (w == 0) {
    int s = (lane < NW) ? lds[lane] : 0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(s, o, 64);
      if (lane >= o) s += y;
    }
    if (lane < NW) lds[lane] = s;
  }
  __syncthreads();
  const int before = (w > 0) ? lds[w - 1] : 0;
  *total = lds[NW - 1];
  __syncthreads();
  return before + x - v;
}

// Projection of the block's Gaussians [base, base + BIN_BLOCK) of an array
// of N, plus the block's sum of tile counts and of culled Gaussians.
__device__ inline void project_block(int base, int N, int TX, int TY, float inv_tile,
                                     const float *__restrict__ xy, const float *__restrict__ chol,
                                     float4 *__restrict__ geom, int4 *__restrict__ rect,
                                     int *__restrict__ counts, int *__restrict__ bsum,
                                     int *__restrict__ bcull) {
  __shared__ int red[2][BIN_BLOCK / 64];
  const int n = base + (int)threadIdx.x;
  int c = 0, cull = 0;
  if (n < N) {
    project_gaussian(n, TX, TY, inv_tile, xy, chol, geom, rect, counts);
    const int v = counts[n];
    c = v > 0 ? v : 0;
    cull = v < 0;
  }
  for (int o = 32; o > 0; o >>= 1) {
    c += __shfl_xor(c, o, 64);
    cull += __shfl_xor(cull, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = c;
    red[1][threadIdx.x >> 6] = cull;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int a = 0, b = 0;
    for (int w = 0; w < BIN_BLOCK / 64; ++w) {
      a += red[0][w];
      b += red[1][w];
    }
    *bsum = a;
    *bcull = b;
  }
}

// Key emission of the block's Gaussians [base, base + BIN_BLOCK): each
// Gaussian's first key slot is block_off (the exclusive prefix of all
// earlier blocks) plus the block-local exclusive prefix of the counts;
// slots at or beyond `cap` are dropped.  offsets[n] receives the clamped
// first slot; keys are (tile << 16) | n, row-major over the rectangle.
__device__ inline void emit_block(int base, int N, int TX, long long block_off, int cap,
                                  const int4 *__restrict__ rect, const int *__restrict__ counts,
                                  int *__restrict__ offsets, uint32_t *__restrict__ keys) {
  __shared__ int lds[BIN_BLOCK / 64];
  const int n = base + (int)threadIdx.x;
  int c = 0;
  if (n < N) {
    const int v = counts[n];
    c = v > 0 ? v : 0;
  }
  int tot;
  const int local = block_exclusive_scan_i32<BIN_BLOCK>(c, &tot, lds);
  if (n >= N) return;
  const long long start = block_off + local;
  const int beg = (int)min(start, (long long)cap);
  const int end = (int)min(start + c, (long long)cap);
  offsets[n] = beg;
  if (end <= beg) return;
  const int4 rc = rect[n];
  int k = beg;
  for (int ty = rc.y; ty <= rc.w && k < end; ++ty)
    for (int tx = rc.x; tx <= rc.z && k < end; ++tx, ++k)
      keys[k] = ((uint32_t)(ty * TX + tx) << 16) | (uint32_t)n;
}

// Exclusive scan of up to BIN_BLOCK per-block sums (one block of BIN_BLOCK
// threads): boff[b] for b < nb; returns the totals in *pairs and *culled
// (valid in every thread).
__device__ inline void scan_block_sums(int nb, const int *__restrict__ bsum,
                                       const int *__restrict__ bcull, long long *__restrict__ boff,
                                       long long *pairs, int *culled) {
  __shared__ long long lds[BIN_BLOCK / 64];
  __shared__ int cl[BIN_BLOCK / 64];
  const int b = threadIdx.x;
  const long long v = (b < nb) ? bsum[b] : 0;
  int c = (b < nb) ? bcull[b] : 0;
  long long total;
  const long long ex = block_exclusive_scan<BIN_BLOCK>(v, &total, lds);
  if (b < nb) boff[b] = ex;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) cl[threadIdx.x >> 6] = c;
  __syncthreads();
  int cs = 0;
  for (int w = 0; w < BIN_BLOCK / 64; ++w) cs += cl[w];
  *pairs = total;
  *culled = cs;
}

// In-place exclusive scan of `total` <= RADIX_SCAN_PER * SCAN_BLOCK 32-bit
// entries by one block of SCAN_BLOCK threads.  Entry e = k * SCAN_BLOCK + t
// lives in register k of thread t, so every load and store of a wavefront
// touches 64 consecutive words.  Each register column is scanned inside the
// wavefronts, the (column, wavefront) totals are scanned by one wavefront in
// (column, wavefront) order, and every thread adds its base back.
__device__ inline void scan_u32_block(uint32_t *__restrict__ a, int total) {
  constexpr int NW = SCAN_BLOCK / 64;
  constexpr int NTOT = RADIX_SCAN_PER * NW;  // <= 512
  __shared__ uint32_t tot[NTOT];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  uint32_t v[RADIX_SCAN_PER], inc[RADIX_SCAN_PER];
#pragma unroll
  for (int k = 0; k < RADIX_SCAN_PER; ++k) {
    const int e = k * SCAN_BLOCK + t;
    v[k] = (e < total) ? a[e] : 0u;
  }
#pragma unroll
  for (int k = 0; k < RADIX_SCAN_PER; ++k) {
    uint32_t x = v[k];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    inc[k] = x;
    if (lane == 63) tot[k * NW + w] = x;
  }
  __syncthreads();
  if (w == 0) {
    // lane l scans entries [8l, 8l + 8) of the (column, wavefront) totals
    uint32_t loc[8], s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = lane * 8 + j;
      loc[j] = (i < NTOT) ? tot[i] : 0u;
      s += loc[j];
    }
    uint32_t x = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    uint32_t run = x - s;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = lane * 8 + j;
      if (i < NTOT) tot[i] = run;
      run += loc[j];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < RADIX_SCAN_PER; ++k) {
    const int e = k * SCAN_BLOCK + t;
    if (e < total) a[e] = tot[k * NW + w] + inc[k] - v[k];
  }
}

// Chunk of the key array owned by sort block b (a multiple of SORT_BLOCK).
__device__ inline void sort_chunk(int n, int G, int b, int *beg, int *end) {
  int chunk = (n + G - 1) / G;
  chunk = (chunk + SORT_BLOCK - 1) / SORT_BLOCK * SORT_BLOCK;
  *beg = min(n, b * chunk);
  *end = min(n, *beg + chunk);
}

}  // namespace gs2d
