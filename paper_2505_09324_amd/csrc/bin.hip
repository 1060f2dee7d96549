// Projection and tile binning for the tile-based rasteriser of Eq. 2.
//
// Per iteration:  project (one thread per Gaussian)  ->  exclusive scan of
// tile counts (one block)  ->  key emission  ->  stable LSD radix sort of the
// keys on their tile bits (8-bit digits; histogram, digit-offset scan,
// stable scatter)  ->  per-tile ranges.
//
// Keys are (tile << 16) | gaussian_index.  Keys are emitted in ascending
// Gaussian order and the sort is stable on the tile bits, so the result is
// ascending in (tile, index): unique, hence bit-exact between runs.
//
// The box/rectangle arithmetic uses the _rn intrinsics so that no multiply
// and add are contracted: the tile decision must match its FP32
// specification exactly.
#include "bin_common.h"

namespace gs2d {

// ---------------------------------------------------------------- project --
// One thread per Gaussian; each block also writes the sum of its tile counts
// and of its culled Gaussians (bsum/bcull[block]).
__global__ void __launch_bounds__(BIN_BLOCK)
k_project(int N, int TX, int TY, float inv_tile, const float *__restrict__ xy,
          const float *__restrict__ chol, float4 *__restrict__ geom, int4 *__restrict__ rect,
          int *__restrict__ counts, int *__restrict__ bsum, int *__restrict__ bcull) {
  project_block(blockIdx.x * BIN_BLOCK, N, TX, TY, inv_tile, xy, chol, geom, rect, counts,
                bsum + blockIdx.x, bcull + blockIdx.x);
}

// ---------------------------------------------------------- block sum scan --
// One block: exclusive scan of the per-block pair counts (boff), total pair
// count n_pairs = min(total, max_pairs) and offsets[N], status bits, culled
// count.  When `tick` is given its value is incremented once (the fitting
// loop's step counter, read by the optimiser later in the same iteration).
__global__ void __launch_bounds__(BIN_BLOCK)
k_scan_blocks(int N, int nb, int max_pairs, const int *__restrict__ bsum,
              const int *__restrict__ bcull, long long *__restrict__ boff,
              int *__restrict__ offsets, int *__restrict__ misc, int *__restrict__ tick) {
  long long total;
  int culled;
  scan_block_sums(nb, bsum, bcull, boff, &total, &culled);
  if (threadIdx.x == 0) {
    const int np = (int)min(total, (long long)max_pairs);
    offsets[N] = np;
    const uint32_t st = (total > (long long)max_pairs ? STATUS_OVERFLOW : 0u) |
                        (culled > 0 ? STATUS_CULLED : 0u);
    misc[MISC_N_PAIRS] = np;
    misc[MISC_STATUS] = (int)st;
    misc[MISC_N_CULLED] = culled;
    misc[MISC_STICKY] |= (int)st;
    if (tick) tick[0] += 1;
  }
}

// ------------------------------------------------------------- emit keys --
__global__ void __launch_bounds__(BIN_BLOCK)
k_emit_keys(int N, int TX, int max_pairs, const int4 *__restrict__ rect,
            const int *__restrict__ counts, const long long *__restrict__ boff,
            int *__restrict__ offsets, uint32_t *__restrict__ keys) {
  emit_block(blockIdx.x * BIN_BLOCK, N, TX, boff[blockIdx.x], max_pairs, rect, counts, offsets,
             keys);
}

// ------------------------------------------------------------ radix sort --
// Pass histogram: hist[d * G + b] = keys of digit d in chunk b.
__global__ void __launch_bounds__(SORT_BLOCK)
k_radix_hist(const uint32_t *__restrict__ keys, const int *__restrict__ misc, int shift, int G,
             uint32_t *__restrict__ hist) {
  __shared__ uint32_t h[RADIX];
  const int b = blockIdx.x;
  h[threadIdx.x] = 0;
  __syncthreads();
  int beg, end;
  sort_chunk(misc[MISC_N_PAIRS], G, b, &beg, &end);
  for (int i = beg + threadIdx.x; i < end; i += SORT_BLOCK)
    atomicAdd(&h[(keys[i] >> shift) & (RADIX - 1)], 1u);
  __syncthreads();
  hist[threadIdx.x * G + b] = h[threadIdx.x];
}

// Exclusive scan of the G*RADIX histogram in (digit, block) order, in place.
__global__ void __launch_bounds__(SCAN_BLOCK)
k_radix_scan(uint32_t *__restrict__ hist, int total_entries) {
  scan_u32_block(hist, total_entries);
}

// Stable scatter of chunk b: in input order, each key goes to
// off[digit] + (earlier keys of the same digit in this chunk).
__global__ void __launch_bounds__(SORT_BLOCK)
k_radix_scatter(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                const int *__restrict__ misc, int shift, int G, const uint32_t *__restrict__ hist) {
  constexpr int NW = SORT_BLOCK / 64;
  __shared__ uint32_t off[RADIX];
  __shared__ uint32_t wcnt[NW][RADIX];
  __shared__ uint32_t wpre[NW][RADIX];
  const int b = blockIdx.x, tid = threadIdx.x, w = tid >> 6;
  off[tid] = hist[tid * G + b];
#pragma unroll
  for (int k = 0; k < NW; ++k) wcnt[k][tid] = 0;
  __syncthreads();
  int beg, end;
  sort_chunk(misc[MISC_N_PAIRS], G, b, &beg, &end);
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
    if (valid) out[off[d] + wpre[w][d] + rank] = key;
    __syncthreads();
    off[tid] += wcnt[0][tid];
#pragma unroll
    for (int k = 0; k < NW; ++k) wcnt[k][tid] = 0;
    __syncthreads();
  }
}

// --------------------------------------------------------------- ranges --
// tile_start[t] = first index i with tile(keys[i]) >= t, for t in [0, n_tiles].
__global__ void __launch_bounds__(256)
k_tile_ranges(const uint32_t *__restrict__ keys, const int *__restrict__ misc, int n_tiles,
              int *__restrict__ tile_start) {
  const int n = misc[MISC_N_PAIRS];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += gridDim.x * blockDim.x) {
    const int cur = (i < n) ? (int)(keys[i] >> 16) : n_tiles;
    const int prev = (i > 0) ? (int)(keys[i - 1] >> 16) : -1;
    for (int t = prev + 1; t <= cur && t <= n_tiles; ++t) tile_start[t] = i;
  }
}

hipError_t launch_binning(const Layout &L, const float *xy, const float *chol, void *ws,
                          hipStream_t st, int *step_tick) {
  float4 *geom = at<float4>(ws, L.geom);
  int *counts = at<int>(ws, L.counts);
  int *offsets = at<int>(ws, L.offsets);
  int *misc = at<int>(ws, L.misc);
  int4 *rect = at<int4>(ws, L.rect);
  int *bsum = at<int>(ws, L.blocks);
  int *bcull = bsum + 256;
  long long *boff = at<long long>(ws, L.blocks + 2048);
  const int nb = (L.N + BIN_BLOCK - 1) / BIN_BLOCK;
  hipLaunchKernelGGL(k_project, dim3(nb), dim3(BIN_BLOCK), 0, st, L.N, L.TX, L.TY,
                     1.0f / (float)L.T, xy, chol, geom, rect, counts, bsum, bcull);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(BIN_BLOCK), 0, st, L.N, nb, L.max_pairs, bsum,
                     bcull, boff, offsets, misc, step_tick);
  uint32_t *ka = at<uint32_t>(ws, L.keys_a), *kb = at<uint32_t>(ws, L.keys_b);
  hipLaunchKernelGGL(k_emit_keys, dim3(nb), dim3(BIN_BLOCK), 0, st, L.N, L.TX, L.max_pairs, rect,
                     counts, boff, offsets, ka);
  uint32_t *hist = at<uint32_t>(ws, L.hist);
  uint32_t *src = ka, *dst = kb;
  for (int p = 0; p < L.sort_passes; ++p) {
    const int shift = 16 + RADIX_BITS * p;
    hipLaunchKernelGGL(k_radix_hist, dim3(L.sort_blocks), dim3(SORT_BLOCK), 0, st, src, misc, shift,
                       L.sort_blocks, hist);
    hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(SCAN_BLOCK), 0, st, hist, L.sort_blocks * RADIX);
    hipLaunchKernelGGL(k_radix_scatter, dim3(L.sort_blocks), dim3(SORT_BLOCK), 0, st, src, dst, misc,
                       shift, L.sort_blocks, hist);
    uint32_t *t = src;
    src = dst;
    dst = t;
  }
  hipLaunchKernelGGL(k_tile_ranges, dim3(512), dim3(256), 0, st, src, misc, L.n_tiles,
                     at<int>(ws, L.tile_start));
  return hipGetLastError();
}

hipError_t launch_radix_sort_tiles(uint32_t *a, uint32_t *b, const int *misc, int G, uint32_t *hist,
                                   int passes, hipStream_t st, const uint32_t **sorted) {
  uint32_t *src = a, *dst = b;
  for (int p = 0; p < passes; ++p) {
    const int shift = 16 + RADIX_BITS * p;
    hipLaunchKernelGGL(k_radix_hist, dim3(G), dim3(SORT_BLOCK), 0, st, src, misc, shift, G, hist);
    hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(SCAN_BLOCK), 0, st, hist, G * RADIX);
    hipLaunchKernelGGL(k_radix_scatter, dim3(G), dim3(SORT_BLOCK), 0, st, src, dst, misc, shift, G,
                       hist);
    uint32_t *t = src;
    src = dst;
    dst = t;
  }
  *sorted = src;
  return hipGetLastError();
}

hipError_t launch_tile_ranges(const uint32_t *keys, const int *misc, int n_tiles, int *tile_start,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_tile_ranges, dim3(256), dim3(256), 0, st, keys, misc, n_tiles, tile_start);
  return hipGetLastError();
}

}  // namespace gs2d
