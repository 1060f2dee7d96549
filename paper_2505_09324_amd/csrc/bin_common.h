// Device-side building blocks of projection and tile binning, shared by the
// one-frame kernels (bin.hip) and the batched ones (batch.hip).
#pragma once

#include "gs2d_internal.h"

namespace gs2d {

constexpr int BIN_BLOCK = 256;  // threads of the projection / emission blocks
static_assert(BIN_BLOCK * BIN_BLOCK >= 65536, "emission scans at most BIN_BLOCK block sums");
static_assert(SORT_BLOCK == RADIX, "scatter threads map one-to-one onto digits");

// Single-pass binning (frames of at most WIDE_MAX_TILES tiles): the whole
// tile index is one radix digit.
constexpr int WIDE_BLOCK = 1024;      // threads of its emission blocks (one chunk each)
constexpr int WIDE_PROJ = 256;        // threads of its projection blocks
constexpr int WIDE_GROUP = WIDE_BLOCK / WIDE_PROJ;  // projection blocks per chunk
constexpr int WIDE_MAX_TILES = 2048;  // largest digit range (11 bits)
constexpr int WIDE_SCATTER = 512;     // threads of its scatter blocks
constexpr int WIDE_SPLIT = 4;         // scatter blocks per emission chunk
static_assert(WIDE_BLOCK * 64 >= 65536, "at most 64 emission blocks per frame");
// Histogram area of the single-pass path (words): the chunk rows (chunk b at
// b * D), then from WIDE_PART_ROWS the cumulative part rows (chunk b, row r
// at WIDE_PART_ROWS + (b * (WIDE_SPLIT - 1) + r) * D).
constexpr size_t WIDE_PART_ROWS = (size_t)64 * WIDE_MAX_TILES;
constexpr size_t WIDE_HIST_WORDS = (size_t)64 * WIDE_MAX_TILES * WIDE_SPLIT;
// Workspace bytes of the binning histograms: the radix path's per-block
// rows or the single-pass path's chunk and cumulative part rows, whichever
// is larger.
constexpr size_t RADIX_HIST_BYTES = (size_t)RADIX * 256 * 4 * 2;
constexpr size_t HIST_BYTES =
    WIDE_HIST_WORDS * 4 > RADIX_HIST_BYTES ? WIDE_HIST_WORDS * 4 : RADIX_HIST_BYTES;

// Projection of Gaussian n (index into xy/chol and the outputs).
// counts[n] = number of tiles met, or -1 for a culled Gaussian (the scan
// turns -1 into 0 and counts the culls).  geom[n] = {mx, my, 1/l1, l2, 1/l3,
// rx, ry, 0}; rect[n] = {tx0, ty0, tx1, ty1}.  The box/rectangle arithmetic
// uses the contraction-free f32_* operations (each rounded once, no fused
// multiply-add): the tile decision must match its FP32 specification exactly.
// Tile rectangle {tx0, ty0, tx1, ty1} of the pixel box [xlo, xhi] x [ylo,
// yhi] clipped to the frame's TX x TY tiles; {0, 0, -1, -1} when the box
// misses the frame.  floor of (edge / T) in FP32, division by the power of
// two T as multiplication by its exact reciprocal.
__device__ inline int4 tile_rect(float xlo, float xhi, float ylo, float yhi, float inv_tile, int TX,
                                 int TY) {
  const float fx0 = floorf(f32_mul(xlo, inv_tile)), fx1 = floorf(f32_mul(xhi, inv_tile));
  const float fy0 = floorf(f32_mul(ylo, inv_tile)), fy1 = floorf(f32_mul(yhi, inv_tile));
  const float lastx = (float)(TX - 1), lasty = (float)(TY - 1);
  int4 rc = make_int4(0, 0, -1, -1);
  if (!(fx1 < 0.f || fx0 > lastx || fy1 < 0.f || fy0 > lasty)) {
    rc.x = (int)fmaxf(fx0, 0.f);
    rc.z = (int)fminf(fx1, lastx);
    rc.y = (int)fmaxf(fy0, 0.f);
    rc.w = (int)fminf(fy1, lasty);
  }
  return rc;
}

__device__ inline bool rect_empty(int4 r) { return r.z < r.x || r.w < r.y; }

// With LAZY (lazy binning, see launch_binning): rect[n] and counts[n] take
// the rectangle of the box grown by `skin` pixels on every side (what a
// rebuild bins), and *stale is set when the exact rectangle is not inside
// brect[n] (the rectangle the current lists were built from) or when the
// Gaussian is culled while brect[n] is not empty (its keys would render the
// zeroed geometry).
template <bool LAZY = false>
__device__ inline int project_values(int n, int TX, int TY, float inv_tile, float mx, float my,
                                     float l1, float l2, float l3, float4 *__restrict__ geom,
                                     int4 *__restrict__ rect, int *__restrict__ counts,
                                     float skin = 0.f, const int4 *__restrict__ brect = nullptr,
                                     bool *stale = nullptr) {
  const float tiny = 6.103515625e-05f;  // 2^-14
  const bool finite = isfinite(mx) && isfinite(my) && isfinite(l1) && isfinite(l2) && isfinite(l3);
  if (!finite || !(fabsf(l1) >= tiny) || !(fabsf(l3) >= tiny)) {
    counts[n] = -1;
    rect[n] = make_int4(0, 0, -1, -1);
    geom[2 * n + 0] = make_float4(0.f, 0.f, 0.f, 0.f);
    geom[2 * n + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (LAZY && !rect_empty(brect[n])) *stale = true;
    return -1;
  }
  const float a = f32_mul(l2, l2);
  const float b = f32_mul(l3, l3);
  const float s = f32_add(a, b);
  const float r = f32_sqrt(s);
  const float ry = f32_mul(3.0f, r);
  const float rx = f32_mul(3.0f, fabsf(l1));
  const float xlo = f32_sub(mx, rx), xhi = f32_add(mx, rx);
  const float ylo = f32_sub(my, ry), yhi = f32_add(my, ry);
  int4 rc = tile_rect(xlo, xhi, ylo, yhi, inv_tile, TX, TY);
  if (LAZY) {
    const int4 bq = brect[n];
    if (!rect_empty(rc) &&
        (rect_empty(bq) || rc.x < bq.x || rc.y < bq.y || rc.z > bq.z || rc.w > bq.w))
      *stale = true;
    rc = tile_rect(f32_sub(xlo, skin), f32_add(xhi, skin), f32_sub(ylo, skin), f32_add(yhi, skin),
                   inv_tile, TX, TY);
  }
  const int cnt = rect_empty(rc) ? 0 : (rc.z - rc.x + 1) * (rc.w - rc.y + 1);
  counts[n] = cnt;
  rect[n] = rc;
  geom[2 * n + 0] = make_float4(mx, my, __fdiv_rn(1.0f, l1), l2);
  geom[2 * n + 1] = make_float4(__fdiv_rn(1.0f, l3), rx, ry, 0.f);
  return cnt;
}

__device__ inline int project_gaussian(int n, int TX, int TY, float inv_tile,
                                       const float *__restrict__ xy, const float *__restrict__ chol,
                                       float4 *__restrict__ geom, int4 *__restrict__ rect,
                                       int *__restrict__ counts) {
  return project_values(n, TX, TY, inv_tile, xy[2 * n + 0], xy[2 * n + 1], chol[3 * n + 0],
                        chol[3 * n + 1], chol[3 * n + 2], geom, rect, counts);
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

// Block sums of the tile counts (v > 0) and of the culled Gaussians
// (v < 0) of one value per thread, written by thread 0.
template <int NT>
__device__ inline void block_count_sums(int v, int *__restrict__ bsum, int *__restrict__ bcull) {
  __shared__ int red[2][NT / 64];
  int c = v > 0 ? v : 0, cull = v < 0;
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
    for (int w = 0; w < NT / 64; ++w) {
      a += red[0][w];
      b += red[1][w];
    }
    *bsum = a;
    *bcull = b;
  }
}

// Projection of the block's Gaussians [base, base + NT) of an array of N,
// plus the block's sum of tile counts and of culled Gaussians.
template <int NT = BIN_BLOCK>
__device__ inline void project_block(int base, int N, int TX, int TY, float inv_tile,
                                     const float *__restrict__ xy, const float *__restrict__ chol,
                                     float4 *__restrict__ geom, int4 *__restrict__ rect,
                                     int *__restrict__ counts, int *__restrict__ bsum,
                                     int *__restrict__ bcull) {
  const int n = base + (int)threadIdx.x;
  int v = 0;
  if (n < N) v = project_gaussian(n, TX, TY, inv_tile, xy, chol, geom, rect, counts);
  block_count_sums<NT>(v, bsum, bcull);
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

// One block of NT threads: the exclusive prefix of entry b among the
// nb <= NT per-block pair counts, their total and the total of the culled
// counts (valid in every thread).
template <int NT = BIN_BLOCK>
__device__ inline void block_sum_prefix(int nb, int b, const int *__restrict__ bsum,
                                        const int *__restrict__ bcull, long long *prefix,
                                        long long *total, int *culled) {
  __shared__ long long lds[NT / 64];
  __shared__ long long pre_b;
  __shared__ int cl[NT / 64];
  const int t = threadIdx.x;
  const long long v = (t < nb) ? bsum[t] : 0;
  int c = (t < nb) ? bcull[t] : 0;
  long long tot;
  const long long ex = block_exclusive_scan<NT>(v, &tot, lds);
  if (t == b) pre_b = ex;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((t & 63) == 0) cl[t >> 6] = c;
  __syncthreads();
  int cs = 0;
  for (int w = 0; w < NT / 64; ++w) cs += cl[w];
  *prefix = pre_b;
  *total = tot;
  *culled = cs;
}

// One block of NT threads: the exclusive prefixes at entries g * b and
// min(g * (b + 1), nbp) of the nbp <= NT per-block pair counts (the first
// and one-past-last key slot of chunk b, which spans g projection blocks),
// their total and the total of the culled counts (valid in every thread).
template <int NT>
__device__ inline void chunk_bounds(int nbp, int b, int g, const int *__restrict__ bsum,
                                    const int *__restrict__ bcull, long long *lo, long long *hi,
                                    long long *total, int *culled) {
  __shared__ long long lds[NT / 64];
  __shared__ long long s_lo, s_hi;
  __shared__ int cl[NT / 64];
  const int t = threadIdx.x;
  const long long v = (t < nbp) ? bsum[t] : 0;
  int c = (t < nbp) ? bcull[t] : 0;
  long long tot;
  const long long ex = block_exclusive_scan<NT>(v, &tot, lds);
  const int i0 = g * b, i1 = min(g * (b + 1), nbp);
  if (t == i0) s_lo = ex;
  if (t == i1) s_hi = ex;
  if (t == 0 && i1 >= nbp) s_hi = tot;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((t & 63) == 0) cl[t >> 6] = c;
  __syncthreads();
  int cs = 0;
  for (int w = 0; w < NT / 64; ++w) cs += cl[w];
  *lo = s_lo;
  *hi = s_hi;
  *total = tot;
  *culled = cs;
}

// Key emission of the block's Gaussians [base, base + BIN_BLOCK): each
// Gaussian's first key slot is block_off (the exclusive prefix of all
// earlier blocks) plus the block-local exclusive prefix of the counts;
// slots at or beyond n_keys (= min(total, capacity)) are dropped.
// offsets[n] receives the clamped first slot; keys are (tile << 16) | n,
// row-major over the rectangle.  The block's keys form one chunk of the
// first radix pass: hist_row[d] receives how many of them have low tile
// byte d (counted in LDS, written with plain stores).
__device__ inline void emit_block(int base, int N, int TX, long long block_off, int n_keys,
                                  const int4 *__restrict__ rect, const int *__restrict__ counts,
                                  int *__restrict__ offsets, uint32_t *__restrict__ keys,
                                  uint32_t *__restrict__ hist_row) {
  static_assert(BIN_BLOCK == RADIX, "one histogram bin per thread");
  __shared__ int lds[BIN_BLOCK / 64];
  __shared__ uint32_t h[RADIX];
  h[threadIdx.x] = 0;
  const int n = base + (int)threadIdx.x;
  int c = 0;
  if (n < N) {
    const int v = counts[n];
    c = v > 0 ? v : 0;
  }
  int tot;
  const int local = block_exclusive_scan_i32<BIN_BLOCK>(c, &tot, lds);  // ends with a barrier
  if (n < N) {
    const long long start = block_off + local;
    const int beg = (int)min(start, (long long)n_keys);
    const int end = (int)min(start + c, (long long)n_keys);
    offsets[n] = beg;
    if (end > beg) {
      const int4 rc = rect[n];
      int k = beg;
      for (int ty = rc.y; ty <= rc.w && k < end; ++ty)
        for (int tx = rc.x; tx <= rc.z && k < end; ++tx, ++k) {
          const uint32_t tile = (uint32_t)(ty * TX + tx);
          keys[k] = (tile << 16) | (uint32_t)n;
          atomicAdd(&h[tile & (RADIX - 1)], 1u);
        }
    }
  }
  __syncthreads();
  hist_row[threadIdx.x] = h[threadIdx.x];
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

// Stable scatter of chunk b = keys in[beg, end) for one radix pass (keys
// sorted on the digit at `shift`; `rows` chunks in order, block-major
// histogram): in input order, each key goes to off[digit] + (earlier keys
// of the same digit in this chunk).
__device__ inline void scatter_chunk(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                     int beg, int end, int rows, int b, int shift,
                                     const uint32_t *__restrict__ hist) {
  constexpr int NW = SORT_BLOCK / 64;
  __shared__ uint32_t off[RADIX];
  __shared__ uint32_t wcnt[NW][RADIX];
  __shared__ uint32_t wpre[NW][RADIX];
  if (beg >= end) return;  // uniform over the block
  const int tid = threadIdx.x, w = tid >> 6;
#pragma unroll
  for (int k = 0; k < NW; ++k) wcnt[k][tid] = 0;
  chunk_digit_offsets(hist, rows, b, off);
  const unsigned long long lt = lanemask_lt();
  // the chunk's keys are loaded into registers KPT sub-tiles at a time, all
  // loads issued together (indices clamped into the chunk)
  constexpr int KPT = 8;
  for (int gbase = beg; gbase < end; gbase += KPT * SORT_BLOCK) {
    uint32_t kreg[KPT];
#pragma unroll
    for (int j = 0; j < KPT; ++j) kreg[j] = in[min(gbase + j * SORT_BLOCK + tid, end - 1)];
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const int base = gbase + j * SORT_BLOCK;
      if (base >= end) break;  // uniform over the block
      const bool valid = base + tid < end;
      const uint32_t key = kreg[j];
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
      if (valid) out[off[d] + wpre[w][d] + rank] = key;
      __syncthreads();
      off[tid] += wcnt[0][tid];
#pragma unroll
      for (int k = 0; k < NW; ++k) wcnt[k][tid] = 0;
      __syncthreads();
    }
  }
}

// tile_start[t] = first index i with tile(keys[i]) >= t, for t in
// [0, n_tiles], over sorted keys[0, n); grid-stride over i.
__device__ inline void tile_ranges(const uint32_t *__restrict__ keys, int n, int n_tiles,
                                   int *__restrict__ tile_start) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x) {
    const int cur = (i < n) ? (int)(keys[i] >> 16) : n_tiles;
    const int prev = (i > 0) ? (int)(keys[i - 1] >> 16) : -1;
    for (int t = prev + 1; t <= cur && t <= n_tiles; ++t) tile_start[t] = i;
  }
}

// ------------------------------------------------------ single-pass path --
// Key emission as emit_block, by blocks of WIDE_BLOCK threads; the block's
// keys are one chunk of the single radix pass whose digit is the whole tile
// index: hist_row[t] (t < D) receives how many of them fall in tile t, and
// part_rows[r * D + t] how many of them fall in tile t within the chunk's
// first r + 1 scatter parts (the split the scatter uses: WIDE_SPLIT parts
// of q = ceil(keys / WIDE_SPLIT) keys), for r < WIDE_SPLIT - 1.  NT threads
// each take WIDE_BLOCK / NT adjacent Gaussians (the keys do not depend on
// it).  E: the block's LDS (EmitLds).
struct EmitLds {
  int lds[WIDE_BLOCK / 64];
  uint32_t hp[WIDE_SPLIT][WIDE_MAX_TILES];
};

template <int NT = WIDE_BLOCK>
__device__ __forceinline__ void emit_block_wide(int base, int N, int TX, long long block_off,
                                       long long block_end, int n_keys, int D,
                                       const int4 *__restrict__ rect,
                                       const int *__restrict__ counts, int *__restrict__ offsets,
                                       uint32_t *__restrict__ keys,
                                       uint32_t *__restrict__ hist_row,
                                       uint32_t *__restrict__ part_rows, EmitLds &E) {
  // one LDS count per key, into its part's histogram; the chunk row is the
  // sum of the parts
  constexpr int G = WIDE_BLOCK / NT;  // adjacent Gaussians per thread
  static_assert(G * NT == WIDE_BLOCK && G <= 2, "one or two Gaussians per thread");
  int *lds = E.lds;
  uint32_t(*hp)[WIDE_MAX_TILES] = E.hp;
  for (int d = threadIdx.x; d < D; d += NT) {
#pragma unroll
    for (int r = 0; r < WIDE_SPLIT; ++r) hp[r][d] = 0;
  }
  const int cbeg = (int)min(block_off, (long long)n_keys);
  const int cend = (int)min(block_end, (long long)n_keys);
  const int q = (cend - cbeg + WIDE_SPLIT - 1) / WIDE_SPLIT;  // >= 1 when a key exists
  const int n0 = base + G * (int)threadIdx.x;
  int c[G], csum = 0;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    c[g] = 0;
    if (n0 + g < N) {
      const int v = counts[n0 + g];
      c[g] = v > 0 ? v : 0;
    }
    csum += c[g];
  }
  int tot;
  int local = block_exclusive_scan_i32<NT>(csum, &tot, lds);  // ends with a barrier
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int n = n0 + g;
    if (n < N) {
      const long long start = block_off + local;
      const int beg = (int)min(start, (long long)n_keys);
      const int end = (int)min(start + c[g], (long long)n_keys);
      offsets[n] = beg;
      if (end > beg) {
        const int4 rc = rect[n];
        int k = beg;
        for (int ty = rc.y; ty <= rc.w && k < end; ++ty)
          for (int tx = rc.x; tx <= rc.z && k < end; ++tx, ++k) {
            const uint32_t tile = (uint32_t)(ty * TX + tx);
            keys[k] = (tile << 16) | (uint32_t)n;
            atomicAdd(&hp[(k - cbeg) / q][tile], 1u);  // part < WIDE_SPLIT: k < cbeg + WIDE_SPLIT q
          }
      }
    }
    local += c[g];
  }
  __syncthreads();
  for (int d = threadIdx.x; d < D; d += NT) {
    uint32_t acc = 0;
#pragma unroll
    for (int r = 0; r < WIDE_SPLIT - 1; ++r) {
      acc += hp[r][d];
      part_rows[(size_t)r * D + d] = acc;
    }
    hist_row[d] = acc + hp[WIDE_SPLIT - 1][d];
  }
}

// Stable scatter of part `part` (of WIDE_SPLIT equal parts) of chunk b (the
// keys emission block b wrote; its bounds from the nbp projection-block
// sums) on the whole tile index (D = 2^bits >= n_tiles digits) by one block
// of WIDE_SCATTER threads, from the `nb` histogram rows (row r = chunk r, D
// words each) and, for part > 0, the chunk's cumulative part row part - 1
// (its earlier parts' keys per tile).
// Each key goes to (keys of lower tiles in all chunks) + (keys of its tile
// in earlier chunks) + (earlier keys of its tile in this chunk).  Block 0
// also writes tile_start[0, n_tiles] (the per-tile totals' exclusive
// prefix; n at the end).  Ranking inside a sub-tile of WIDE_SCATTER keys:
// every lane ORs its lane bit into a per-(wavefront, tile) 64-bit mask in
// LDS; its own wavefront's mask gives its rank among equal tiles (lanes
// below it) and the other wavefronts' masks the count of its tile in
// earlier wavefronts; only the masks that were set are cleared.  The
// histogram loads are issued before the chunk bounds are
// known so that their latency overlaps the block-sum prefix.
// LDS of one scatter block (scatter_chunk_wide).
struct ScatterLds {
  uint32_t off[WIDE_MAX_TILES];
  unsigned long long wmask[WIDE_SCATTER / 64][WIDE_MAX_TILES];
  uint4 fold[2][WIDE_SCATTER];
  int lds[WIDE_SCATTER / 64];
};

__device__ __forceinline__ void scatter_chunk_wide(const uint32_t *__restrict__ in,
                                          uint32_t *__restrict__ out, int nb, int nbp, int b,
                                          int part, int D,
                                          int bits, int n, int n_tiles,
                                          const int *__restrict__ bsum,
                                          const int *__restrict__ bcull,
                                          const uint32_t *__restrict__ hist,
                                          int *__restrict__ tile_start, ScatterLds &L) {
  constexpr int NT = WIDE_SCATTER, NW = NT / 64, RB = 16;
  static_assert(NT * 4 == WIDE_MAX_TILES, "one uint4 column of digits per thread at most");
  uint32_t *off = L.off;
  unsigned long long(*wmask)[WIDE_MAX_TILES] = L.wmask;
  uint4(*fold)[NT] = L.fold;
  int *lds = L.lds;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  {
    uint4 *t4 = reinterpret_cast<uint4 *>(&wmask[0][0]);
    for (int i = tid; i < NW * WIDE_MAX_TILES / 2; i += NT) t4[i] = make_uint4(0u, 0u, 0u, 0u);
  }
  // digit totals and the prefix over earlier chunks: thread t owns digits
  // [4 cq, 4 cq + 4) of column cq = t % C (C = D / 4 uint4 columns) over the
  // rows r = t / C, t / C + K, ... (K = NT / C row groups)
  const int C = D / 4, K = NT / C;
  const int cq = tid % C, r0 = tid / C;
  const uint4 *h4 = reinterpret_cast<const uint4 *>(hist);
  uint4 h[RB];
#pragma unroll
  for (int j = 0; j < RB; ++j) h[j] = h4[(size_t)min(r0 + j * K, nb - 1) * C + cq];
  uint4 early = make_uint4(0u, 0u, 0u, 0u);  // this chunk's earlier parts, per digit
  if (part > 0 && r0 == 0)
    early = reinterpret_cast<const uint4 *>(
        hist + WIDE_PART_ROWS + ((size_t)b * (WIDE_SPLIT - 1) + part - 1) * D)[cq];
  long long pre_keys, end_keys, total;
  int culled;
  chunk_bounds<NT>(nbp, b, WIDE_GROUP, bsum, bcull, &pre_keys, &end_keys, &total, &culled);
  const int cbeg = (int)min(pre_keys, (long long)n);
  const int cend = (int)min(end_keys, (long long)n);
  const int q = (cend - cbeg + WIDE_SPLIT - 1) / WIDE_SPLIT;
  const int beg = min(cbeg + part * q, cend), end = min(beg + q, cend);
  const bool first = b == 0 && part == 0;  // writes tile_start
  if (beg >= end && !first) return;  // uniform over the block
  // the chunk's keys into registers (KPT sub-tiles, loads issued together)
  constexpr int KPT = 16;
  uint32_t kreg[KPT];
#pragma unroll
  for (int j = 0; j < KPT; ++j) kreg[j] = (beg < end) ? in[min(beg + j * NT + tid, end - 1)] : 0u;
  uint4 tot = make_uint4(0u, 0u, 0u, 0u), pre = make_uint4(0u, 0u, 0u, 0u);
  for (int rb = r0;;) {
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      const int r = rb + j * K;
      const uint32_t in_rows = r < nb ? 1u : 0u, earlier = r < b ? 1u : 0u;
      tot.x += in_rows * h[j].x;
      tot.y += in_rows * h[j].y;
      tot.z += in_rows * h[j].z;
      tot.w += in_rows * h[j].w;
      pre.x += earlier * h[j].x;
      pre.y += earlier * h[j].y;
      pre.z += earlier * h[j].z;
      pre.w += earlier * h[j].w;
    }
    rb += RB * K;
    if (rb >= nb) break;
#pragma unroll
    for (int j = 0; j < RB; ++j) h[j] = h4[(size_t)min(rb + j * K, nb - 1) * C + cq];
  }
  // fold the K row groups of each column (C * K = NT)
  if (K > 1) {
    fold[0][tid] = tot;
    fold[1][tid] = pre;
    __syncthreads();
    if (r0 == 0) {
      for (int k = 1; k < K; ++k) {
        const uint4 a = fold[0][k * C + cq], p = fold[1][k * C + cq];
        tot.x += a.x;
        tot.y += a.y;
        tot.z += a.z;
        tot.w += a.w;
        pre.x += p.x;
        pre.y += p.y;
        pre.z += p.z;
        pre.w += p.w;
      }
    }
  }
  // threads with r0 == 0 (tid < C) hold digits [4 tid, 4 tid + 4); the
  // block scan runs over all NT threads with zeros beyond C
  const uint32_t tsum = (r0 == 0) ? (tot.x + tot.y + tot.z + tot.w) : 0u;
  int all;
  const uint32_t ex = (uint32_t)block_exclusive_scan_i32<NT>((int)tsum, &all, lds);
  if (r0 == 0) {
    const uint32_t b0 = ex, b1 = b0 + tot.x, b2 = b1 + tot.y, b3 = b2 + tot.z;
    const int d = 4 * cq;
    off[d + 0] = b0 + pre.x + early.x;
    off[d + 1] = b1 + pre.y + early.y;
    off[d + 2] = b2 + pre.z + early.z;
    off[d + 3] = b3 + pre.w + early.w;
    if (first) {
      if (d + 0 < n_tiles) tile_start[d + 0] = (int)b0;
      if (d + 1 < n_tiles) tile_start[d + 1] = (int)b1;
      if (d + 2 < n_tiles) tile_start[d + 2] = (int)b2;
      if (d + 3 < n_tiles) tile_start[d + 3] = (int)b3;
    }
  }
  if (first && tid == 0) tile_start[n_tiles] = n;
  __syncthreads();
  const unsigned long long lt = lanemask_lt();
  const unsigned long long me = 1ull << lane;
  for (int gbase = beg; gbase < end; gbase += KPT * NT) {
    if (gbase != beg) {
#pragma unroll
      for (int j = 0; j < KPT; ++j) kreg[j] = in[min(gbase + j * NT + tid, end - 1)];
    }
#pragma unroll
    for (int j = 0; j < KPT; ++j) {
      const int base = gbase + j * NT;
      if (base >= end) break;  // uniform over the block
      const bool valid = base + tid < end;
      const uint32_t key = kreg[j];
      const uint32_t d = key >> 16;
      if (valid) atomicOr(&wmask[w][d], me);
      __syncthreads();
      uint32_t before = 0, after = 0, rank = 0, cnt = 0;
      if (valid) {
#pragma unroll
        for (int k = 0; k < NW; ++k) {
          const unsigned long long m = wmask[k][d];
          const uint32_t c = (uint32_t)__popcll(m);
          before += (k < w) ? c : 0u;
          after += (k > w) ? c : 0u;
          if (k == w) {
            rank = (uint32_t)__popcll(m & lt);
            cnt = c;
          }
        }
        out[off[d] + before + rank] = key;
      }
      __syncthreads();
      // the lowest lane of the last wavefront holding tile d advances its
      // offset; the lowest lane of each wavefront clears its mask
      if (valid && rank == 0) {
        if (after == 0) off[d] += before + cnt;
        wmask[w][d] = 0ull;
      }
      __syncthreads();
    }
  }
}

}  // namespace gs2d
