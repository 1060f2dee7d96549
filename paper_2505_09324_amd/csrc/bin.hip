// Projection and tile binning for the tile-based rasteriser of Eq. 2.
//
// Per iteration, four launches:
//   project   one thread per Gaussian: box, tile rectangle, tile count, and
//             per-block sums; also clears the histograms below;
//   emit      every block scans the (<= 256) block sums for its own prefix,
//             writes its Gaussians' keys, and counts them into the first
//             radix pass's per-chunk digit histogram and into per-tile
//             counts (integer atomics: order-independent, exact);
//   scatter   one launch per 8-bit digit pass of the stable LSD radix sort
//             on the tile bits: each block derives its chunk's digit
//             offsets from the histogram rows itself, scatters stably, and
//             (all passes but the last) counts its keys into the next
//             pass's histogram at their output slots; the last pass carries
//             one extra block that turns the per-tile counts into tile
//             ranges and into the raster's tile order (largest lists
//             first).
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
// and of its culled Gaussians (bsum/bcull[block]) and clears its share of
// the n4 uint4 words at `zero` (histograms and tile counts).
__global__ void __launch_bounds__(BIN_BLOCK)
k_project(int N, int TX, int TY, float inv_tile, const float *__restrict__ xy,
          const float *__restrict__ chol, float4 *__restrict__ geom, int4 *__restrict__ rect,
          int *__restrict__ counts, int *__restrict__ bsum, int *__restrict__ bcull,
          uint4 *__restrict__ zero, long long n4) {
  project_block(blockIdx.x * BIN_BLOCK, N, TX, TY, inv_tile, xy, chol, geom, rect, counts,
                bsum + blockIdx.x, bcull + blockIdx.x);
  clear_u4(zero, n4);
}

// ------------------------------------------------------------- emit keys --
// Block b: prefix of its pair count among all nb blocks, then key emission.
// Block 0 also publishes the pair count n_pairs = min(total, max_pairs),
// offsets[N], the status bits and the culled count; when `tick` is given its
// value is incremented once (the fitting loop's step counter, read by the
// optimiser later in the same iteration).
__global__ void __launch_bounds__(BIN_BLOCK)
k_emit_keys(int N, int TX, int nb, int max_pairs, int G, const int4 *__restrict__ rect,
            const int *__restrict__ counts, const int *__restrict__ bsum,
            const int *__restrict__ bcull, int *__restrict__ offsets, uint32_t *__restrict__ keys,
            uint32_t *__restrict__ hist0, uint32_t *__restrict__ tile_count,
            int *__restrict__ misc, int *__restrict__ tick) {
  long long pre, total;
  int culled;
  block_sum_prefix(nb, blockIdx.x, bsum, bcull, &pre, &total, &culled);
  const int np = (int)min(total, (long long)max_pairs);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    offsets[N] = np;
    const uint32_t st = (total > (long long)max_pairs ? STATUS_OVERFLOW : 0u) |
                        (culled > 0 ? STATUS_CULLED : 0u);
    misc[MISC_N_PAIRS] = np;
    misc[MISC_STATUS] = (int)st;
    misc[MISC_N_CULLED] = culled;
    misc[MISC_STICKY] |= (int)st;
    if (tick) tick[0] += 1;
  }
  emit_block(blockIdx.x * BIN_BLOCK, N, TX, pre, np, G, rect, counts, offsets, keys, hist0,
             tile_count);
}

// ------------------------------------------------------------ radix sort --
// Per-chunk histogram of one pass (used when no earlier kernel counted it).
__global__ void __launch_bounds__(SORT_BLOCK)
k_radix_hist(const uint32_t *__restrict__ keys, const int *__restrict__ misc, int shift, int G,
             uint32_t *__restrict__ hist) {
  chunk_histogram(keys, misc[MISC_N_PAIRS], G, blockIdx.x, shift, hist);
}

// Blocks [0, G): stable scatter of one chunk (NEXT: also count the next
// pass's histogram).  LAST: block G computes tile_start and the tile order
// from tile_count.
template <bool NEXT, bool LAST>
__global__ void __launch_bounds__(SORT_BLOCK)
k_radix_scatter(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                const int *__restrict__ misc, int shift, int G, const uint32_t *__restrict__ hist,
                uint32_t *__restrict__ hist_next, const uint32_t *__restrict__ tile_count,
                int n_tiles, int *__restrict__ tile_start, int *__restrict__ tile_order) {
  if (LAST && (int)blockIdx.x == G) {
    tile_starts(tile_count, n_tiles, tile_start);
    __syncthreads();
    tile_order_by_count(tile_count, n_tiles, tile_order);
    return;
  }
  scatter_chunk<NEXT>(in, out, misc[MISC_N_PAIRS], G, blockIdx.x, shift, hist, hist_next);
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
  int *bcull = bsum + BIN_BLOCK;
  uint32_t *hist0 = at<uint32_t>(ws, L.hist);
  uint32_t *hist1 = hist0 + (size_t)RADIX * L.sort_blocks;
  uint32_t *tcount = at<uint32_t>(ws, L.tile_count);
  int *tstart = at<int>(ws, L.tile_start);
  int *torder = at<int>(ws, L.tile_order);
  const long long n4 = (long long)(L.tile_count + 4 * (size_t)L.tile_count_words - L.hist) / 16;
  const int nb = (L.N + BIN_BLOCK - 1) / BIN_BLOCK;
  const int G = L.sort_blocks;
  hipLaunchKernelGGL(k_project, dim3(nb), dim3(BIN_BLOCK), 0, st, L.N, L.TX, L.TY,
                     1.0f / (float)L.T, xy, chol, geom, rect, counts, bsum, bcull,
                     at<uint4>(ws, L.hist), n4);
  uint32_t *ka = at<uint32_t>(ws, L.keys_a), *kb = at<uint32_t>(ws, L.keys_b);
  hipLaunchKernelGGL(k_emit_keys, dim3(nb), dim3(BIN_BLOCK), 0, st, L.N, L.TX, nb, L.max_pairs, G,
                     rect, counts, bsum, bcull, offsets, ka, hist0, tcount, misc, step_tick);
  if (L.sort_passes == 1) {
    hipLaunchKernelGGL((k_radix_scatter<false, true>), dim3(G + 1), dim3(SORT_BLOCK), 0, st, ka,
                       kb, misc, 16, G, hist0, nullptr, tcount, L.n_tiles, tstart, torder);
  } else {
    hipLaunchKernelGGL((k_radix_scatter<true, false>), dim3(G), dim3(SORT_BLOCK), 0, st, ka, kb,
                       misc, 16, G, hist0, hist1, nullptr, 0, nullptr, nullptr);
    hipLaunchKernelGGL((k_radix_scatter<false, true>), dim3(G + 1), dim3(SORT_BLOCK), 0, st, kb,
                       ka, misc, 16 + RADIX_BITS, G, hist1, nullptr, tcount, L.n_tiles, tstart, torder);
  }
  return hipGetLastError();
}

hipError_t launch_radix_sort_tiles(uint32_t *a, uint32_t *b, const int *misc, int G, uint32_t *hist,
                                   int passes, hipStream_t st, const uint32_t **sorted) {
  uint32_t *src = a, *dst = b;
  for (int p = 0; p < passes; ++p) {
    const int shift = 16 + RADIX_BITS * p;
    hipLaunchKernelGGL(k_radix_hist, dim3(G), dim3(SORT_BLOCK), 0, st, src, misc, shift, G, hist);
    hipLaunchKernelGGL((k_radix_scatter<false, false>), dim3(G), dim3(SORT_BLOCK), 0, st, src, dst,
                       misc, shift, G, hist, nullptr, nullptr, 0, nullptr, nullptr);
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
