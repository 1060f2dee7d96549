// Device-side building blocks of projection and tile binning, shared by the
// one-frame kernels (bin.hip) and the batched ones (batch.hip).
#pragma once

#include "gs2d_internal.h"

namespace gs2d {

constexpr int BIN_BLOCK = 256;  // threads of the projection / emission blocks
static_assert(BIN_BLOCK * BIN_BLOCK >= 65536, "emission scans at most BIN_BLOCK block sums");
static_assert(SORT_BLOCK == RADIX, "scatter threads map one-to-one onto digits");

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

// Grid-stride clear of n4 uint4 words (one call per thread of a grid).
__device__ inline void clear_u4(uint4 *__restrict__ p, long long n4) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Keys per sort chunk when n keys are split over G chunks: a multiple of
// SORT_BLOCK, never zero.
__device__ inline int chunk_len(int n, int G) {
  const int c = (n + G - 1) / G;
  return max(SORT_BLOCK, (c + SORT_BLOCK - 1) / SORT_BLOCK * SORT_BLOCK);
}

// Chunk [beg, end) of the key array owned by sort block b.
__device__ inline void sort_chunk(int n, int G, int b, int *beg, int *end) {
  const int chunk = chunk_len(n, G);
  *beg = min(n, b * chunk);
  *end = min(n, *beg + chunk);
}

// One block of BIN_BLOCK threads: the exclusive prefix of entry b among the
// nb <= BIN_BLOCK per-block pair counts, their total and the total of the
// culled counts (valid in every thread).
__device__ inline void block_sum_prefix(int nb, int b, const int *__restrict__ bsum,
                                        const int *__restrict__ bcull, long long *prefix,
                                        long long *total, int *culled) {
  __shared__ long long lds[BIN_BLOCK / 64];
  __shared__ long long pre_b;
  __shared__ int cl[BIN_BLOCK / 64];
  const int t = threadIdx.x;
  const long long v = (t < nb) ? bsum[t] : 0;
  int c = (t < nb) ? bcull[t] : 0;
  long long tot;
  const long long ex = block_exclusive_scan<BIN_BLOCK>(v, &tot, lds);
  if (t == b) pre_b = ex;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((t & 63) == 0) cl[t >> 6] = c;
  __syncthreads();
  int cs = 0;
  for (int w = 0; w < BIN_BLOCK / 64; ++w) cs += cl[w];
  *prefix = pre_b;
  *total = tot;
  *culled = cs;
}

// Key emission of the block's Gaussians [base, base + BIN_BLOCK): each
// Gaussian's first key slot is block_off (the exclusive prefix of all
// earlier blocks) plus the block-local exclusive prefix of the counts;
// slots at or beyond n_keys (= min(total, capacity)) are dropped.
// offsets[n] receives the clamped first slot; keys are (tile << 16) | n,
// row-major over the rectangle.  Every emitted key also counts into
// hist0[chunk * RADIX + (tile & 0xFF)] (chunk = slot / chunk_len(n_keys, G):
// the first radix pass's per-chunk histogram) and into tile_count[tile].
__device__ inline void emit_block(int base, int N, int TX, long long block_off, int n_keys, int G,
                                  const int4 *__restrict__ rect, const int *__restrict__ counts,
                                  int *__restrict__ offsets, uint32_t *__restrict__ keys,
                                  uint32_t *__restrict__ hist0, uint32_t *__restrict__ tile_count) {
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
  const int beg = (int)min(start, (long long)n_keys);
  const int end = (int)min(start + c, (long long)n_keys);
  offsets[n] = beg;
  if (end <= beg) return;
  const int chunk = chunk_len(n_keys, G);
  int ck = beg / chunk;
  int next = (ck + 1) * chunk;
  const int4 rc = rect[n];
  int k = beg;
  for (int ty = rc.y; ty <= rc.w && k < end; ++ty)
    for (int tx = rc.x; tx <= rc.z && k < end; ++tx, ++k) {
      const uint32_t tile = (uint32_t)(ty * TX + tx);
      keys[k] = (tile << 16) | (uint32_t)n;
      if (k == next) {
        ++ck;
        next += chunk;
      }
      atomicAdd(&hist0[ck * RADIX + (tile & (RADIX - 1))], 1u);
      atomicAdd(&tile_count[tile], 1u);
    }
}

// Per-chunk histogram of one radix pass, block-major: hist[b * RADIX + d] =
// keys of digit d in chunk b (zero for an empty chunk).
__device__ inline void chunk_histogram(const uint32_t *__restrict__ keys, int n, int G, int b,
                                       int shift, uint32_t *__restrict__ hist) {
  __shared__ uint32_t h[RADIX];
  h[threadIdx.x] = 0;
  __syncthreads();
  int beg, end;
  sort_chunk(n, G, b, &beg, &end);
  for (int i = beg + threadIdx.x; i < end; i += SORT_BLOCK)
    atomicAdd(&h[(keys[i] >> shift) & (RADIX - 1)], 1u);
  __syncthreads();
  hist[b * RADIX + threadIdx.x] = h[threadIdx.x];
}

// Digit offsets of chunk b for one radix pass, by one block of SORT_BLOCK
// threads: off[d] = (keys of every digit < d in all chunks) + (keys of digit
// d in the chunks before b), from the block-major histogram of `rows`
// non-empty chunks.  Each wavefront sums every fourth row with one 16-byte
// load per lane (a row is 1 KiB), so the rows are read coalesced and
// in parallel; the partial sums meet in LDS.  Ends with a barrier.
__device__ inline void chunk_digit_offsets(const uint32_t *__restrict__ hist, int rows, int b,
                                           uint32_t *__restrict__ off) {
  constexpr int NW = SORT_BLOCK / 64;
  __shared__ uint32_t ptot[NW][RADIX];
  __shared__ uint32_t ppre[NW][RADIX];
  __shared__ int lds[NW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint4 *h4 = reinterpret_cast<const uint4 *>(hist);
  uint4 tot = make_uint4(0u, 0u, 0u, 0u), pre = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll 4
  for (int r = w; r < rows; r += NW) {
    const uint4 h = h4[r * (RADIX / 4) + lane];
    tot.x += h.x;
    tot.y += h.y;
    tot.z += h.z;
    tot.w += h.w;
    if (r < b) {
      pre.x += h.x;
      pre.y += h.y;
      pre.z += h.z;
      pre.w += h.w;
    }
  }
  reinterpret_cast<uint4 *>(ptot[w])[lane] = tot;
  reinterpret_cast<uint4 *>(ppre[w])[lane] = pre;
  __syncthreads();
  const int d = threadIdx.x;
  uint32_t T = 0, P = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    T += ptot[k][d];
    P += ppre[k][d];
  }
  int all;
  const int ex = block_exclusive_scan_i32<SORT_BLOCK>((int)T, &all, lds);
  off[d] = (uint32_t)ex + P;
  __syncthreads();
}

// Stable scatter of chunk b of one radix pass (keys in[0, n) sorted on the
// digit at `shift`, G chunks): in input order, each key goes to
// off[digit] + (earlier keys of the same digit in this chunk).  With
// hist_next, every key also counts into the next pass's per-chunk
// histogram at its output slot.
template <bool NEXT>
__device__ inline void scatter_chunk(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                     int n, int G, int b, int shift,
                                     const uint32_t *__restrict__ hist,
                                     uint32_t *__restrict__ hist_next) {
  constexpr int NW = SORT_BLOCK / 64;
  __shared__ uint32_t off[RADIX];
  __shared__ uint32_t wcnt[NW][RADIX];
  __shared__ uint32_t wpre[NW][RADIX];
  const int chunk = chunk_len(n, G);
  const int beg = min(n, b * chunk), end = min(n, beg + chunk);
  if (beg >= end) return;  // uniform over the block
  const int tid = threadIdx.x, w = tid >> 6;
#pragma unroll
  for (int k = 0; k < NW; ++k) wcnt[k][tid] = 0;
  chunk_digit_offsets(hist, (n + chunk - 1) / chunk, b, off);
  const unsigned long long lt = lanemask_lt();
  for (int base = beg; base < end; base += SORT_BLOCK) {
    const int i = base + tid;
    const bool valid = i < end;
    const uint32_t key = valid ? in[i] : 0u;
    const uint32_t d = (key >> shift) & (RADIX - 1);
    // lanes of this wave holding the same digit
    unsigned long long match = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < RADIX_BITS; ++bit) {
      const bool on = (d >> bit) & 1u;
      const unsigned long long bal = __ballot(on);
      match &= on ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(match & lt);
    if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(match);
    __syncthreads();
    {
      uint32_t s = 0;
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        wpre[k][tid] = s;
        s += wcnt[k][tid];
      }
      wcnt[0][tid] = s;  // reuse row 0 as the sub-tile total of digit tid
    }
    __syncthreads();
    if (valid) {
      const uint32_t p = off[d] + wpre[w][d] + rank;
      out[p] = key;
      if (NEXT)
        atomicAdd(&hist_next[(p / (uint32_t)chunk) * RADIX + ((key >> (shift + RADIX_BITS)) & (RADIX - 1))],
                  1u);
    }
    __syncthreads();
    off[tid] += wcnt[0][tid];
#pragma unroll
    for (int k = 0; k < NW; ++k) wcnt[k][tid] = 0;
    __syncthreads();
  }
}

// One block of SORT_BLOCK threads: tile_start[t] = sum of tile_count[0, t)
// for t in [0, n_tiles] (the first slot of every tile's run in the sorted
// key array).  Rounds of 8 consecutive counts per thread.
__device__ inline void tile_starts(const uint32_t *__restrict__ tile_count, int n_tiles,
                                   int *__restrict__ tile_start) {
  constexpr int PER = 8;
  __shared__ int lds[SORT_BLOCK / 64];
  int carry = 0;
  for (int base = 0; base < n_tiles; base += SORT_BLOCK * PER) {
    const int t0 = base + (int)threadIdx.x * PER;
    int v[PER], s = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      v[j] = (t0 + j < n_tiles) ? (int)tile_count[t0 + j] : 0;
      s += v[j];
    }
    int round_total;
    int run = carry + block_exclusive_scan_i32<SORT_BLOCK>(s, &round_total, lds);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      if (t0 + j < n_tiles) tile_start[t0 + j] = run;
      run += v[j];
    }
    carry += round_total;
  }
  if (threadIdx.x == 0) tile_start[n_tiles] = carry;
}

// Bucket of a tile's pair count for the launch order: four buckets per
// power of two, bucket 0 for the largest counts.
__device__ inline int count_bucket(uint32_t c) {
  const uint32_t x = c + 1u;  // >= 1
  const int k = 31 - __clz((int)x);
  const int f = k >= 2 ? (int)((x >> (k - 2)) & 3u) : (int)((x << (2 - k)) & 3u);
  return 127 - (4 * k + f);
}

// One block of SORT_BLOCK threads: order[0, n_tiles) = the tiles by
// decreasing pair count (bucketed as above; any order inside a bucket).
// The raster processes tiles in this order, so the longest tiles start
// first and short ones fill the end of the launch.
__device__ inline void tile_order_by_count(const uint32_t *__restrict__ tile_count, int n_tiles,
                                           int *__restrict__ order) {
  constexpr int NBK = 128;
  static_assert(NBK <= SORT_BLOCK, "one bucket per thread");
  __shared__ int bk[NBK];
  __shared__ int lds[SORT_BLOCK / 64];
  if (threadIdx.x < NBK) bk[threadIdx.x] = 0;
  __syncthreads();
  for (int t = threadIdx.x; t < n_tiles; t += SORT_BLOCK) atomicAdd(&bk[count_bucket(tile_count[t])], 1);
  __syncthreads();
  const int v = (threadIdx.x < NBK) ? bk[threadIdx.x] : 0;
  int all;
  const int ex = block_exclusive_scan_i32<SORT_BLOCK>(v, &all, lds);
  if (threadIdx.x < NBK) bk[threadIdx.x] = ex;
  __syncthreads();
  for (int t = threadIdx.x; t < n_tiles; t += SORT_BLOCK)
    order[atomicAdd(&bk[count_bucket(tile_count[t])], 1)] = t;
}

}  // namespace gs2d
