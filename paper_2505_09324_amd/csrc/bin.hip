// Projection and tile binning for the tile-based rasteriser of Eq. 2.
//
// Frames of at most 2048 tiles take a single radix pass whose digit is the
// whole tile index:
//   project   (1024-thread blocks) box, tile rectangle, count, block sums;
//   emit      every block scans the (<= 64) block sums for its prefix,
//             writes its keys and their per-tile histogram row (LDS);
//   scatter   block b stably scatters emission block b's keys; it derives
//             its per-tile offsets from the histogram rows, and block 0
//             writes tile_start from the per-tile totals.
// Larger frames use two 8-bit passes:
//   project   one thread per Gaussian: box, tile rectangle, tile count, and
//             per-block sums;
//   emit      every block scans the (<= 256) block sums for its own prefix
//             and writes its Gaussians' keys; its keys are one chunk of the
//             first radix pass, whose digit histogram it counts in LDS;
//   scatter   stable scatter of each emission block's chunk on the low tile
//             byte, digit offsets computed inside the block from the
//             histogram rows;
//   [hist, scatter]  the second pass (high tile byte) when there are more
//             than 256 tiles, over fixed chunks;
//   ranges    tile_start from the sorted keys.
// No kernel uses global atomics or a single-block serial scan.
//
// Keys are (tile << 16) | gaussian_index.  Keys are emitted in ascending
// Gaussian order and the sort is stable on the tile bits, so the result is
// ascending in (tile, index): unique, hence bit-exact between runs.
//
// The box/rectangle arithmetic uses the contraction-free f32_* operations
// (each rounded once, no fused multiply-add): the tile decision must match
// its FP32 specification exactly.
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

// ------------------------------------------------------------- emit keys --
// Block b: prefix of its pair count among all nb blocks, then key emission
// and the first pass's histogram row b.  Block 0 also publishes the pair
// count n_pairs = min(total, max_pairs), offsets[N], the status bits and the
// culled count; when `tick` is given its value is incremented once (the
// fitting loop's step counter, read by the optimiser later in the same
// iteration).
__global__ void __launch_bounds__(BIN_BLOCK)
k_emit_keys(int N, int TX, int nb, int max_pairs, const int4 *__restrict__ rect,
            const int *__restrict__ counts, const int *__restrict__ bsum,
            const int *__restrict__ bcull, int *__restrict__ offsets, uint32_t *__restrict__ keys,
            uint32_t *__restrict__ hist, int *__restrict__ misc, int *__restrict__ tick) {
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
    misc[MISC_LISTS_LO] = misc[MISC_LISTS_HI] = 0;  // no longer lazy lists
    if (tick) tick[0] += 1;
  }
  emit_block(blockIdx.x * BIN_BLOCK, N, TX, pre, np, rect, counts, offsets, keys,
             hist + (size_t)blockIdx.x * RADIX);
}

// ------------------------------------------------------- single-pass path --
// Lazy binning (skin > 0): one flag per wavefront whose Gaussians made the
// lists stale.
__device__ inline void flag_stale(bool stale, int *__restrict__ misc) {
  if (__ballot(stale) && (threadIdx.x & 63) == 0) atomicOr(&misc[MISC_STALE], 1);
}

__global__ void __launch_bounds__(WIDE_PROJ)
k_project_wide(int N, int TX, int TY, float inv_tile, const float *__restrict__ xy,
               const float *__restrict__ chol, float4 *__restrict__ geom, int4 *__restrict__ rect,
               int *__restrict__ counts, int *__restrict__ bsum, int *__restrict__ bcull,
               float skin, const int4 *__restrict__ brect, int *__restrict__ misc) {
  if (skin > 0.f) {
    const int n = blockIdx.x * WIDE_PROJ + (int)threadIdx.x;
    int v = 0;
    bool stale = false;
    if (n < N)
      v = project_values<true>(n, TX, TY, inv_tile, xy[2 * n], xy[2 * n + 1], chol[3 * n],
                               chol[3 * n + 1], chol[3 * n + 2], geom, rect, counts, skin, brect,
                               &stale);
    flag_stale(stale, misc);
    block_count_sums<WIDE_PROJ>(v, bsum + blockIdx.x, bcull + blockIdx.x);
    return;
  }
  project_block<WIDE_PROJ>(blockIdx.x * WIDE_PROJ, N, TX, TY, inv_tile, xy, chol, geom, rect,
                           counts, bsum + blockIdx.x, bcull + blockIdx.x);
}

// The previous iteration's optimiser step fused with the projection: one
// thread per Gaussian applies Adam to its 8 parameters (gradients cleared)
// and projects the updated Gaussian from its registers.  One extra block
// (blockIdx.x == gridDim.x - 1) reduces the previous iteration's loss
// partials into the trace.  Every thread reads the step (written only by
// the later emission kernel) and derives the bias corrections itself, so
// its parameter, gradient and moment loads wait for no barrier.
__global__ void __launch_bounds__(WIDE_PROJ)
k_adam_project_wide(int N, int TX, int TY, float inv_tile, PendingAdam a,
                    float4 *__restrict__ geom, int4 *__restrict__ rect, int *__restrict__ counts,
                    int *__restrict__ bsum, int *__restrict__ bcull, float skin,
                    const int4 *__restrict__ brect, int *__restrict__ misc) {
  __shared__ double red[WIDE_PROJ / 64];
  const int s_t = a.step[0];
  if (blockIdx.x == gridDim.x - 1) {  // the loss of the previous iteration
    double s = 0.0;
    s = thread_sum_parts(a.loss_part, a.n_part);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0 && s_t - 1 < a.trace_len) {
      double tot = 0.0;
      for (int w = 0; w < WIDE_PROJ / 64; ++w) tot += red[w];
      a.trace[s_t - 1] = (float)(tot * (double)a.loss_scale);
    }
    return;
  }
  const float b1 = a.cfg.beta1, b2 = a.cfg.beta2, eps = a.cfg.eps;
  float bc1, bc2;
  adam_bias(s_t, b1, b2, &bc1, &bc2);
  const int n = blockIdx.x * WIDE_PROJ + threadIdx.x;
  int v = 0;
  bool stale = false;
  if (n < N) {
    const size_t N2 = 2 * (size_t)N, N5 = 5 * (size_t)N;
    // an inactive Gaussian keeps its parameters and moments (its gradient
    // is still cleared)
    const bool upd = !a.active || a.active[n];
    float p[8];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const size_t i = 2 * (size_t)n + c;
      const float g = a.g_xy[i];
      a.g_xy[i] = 0.f;
      p[c] = a.xy[i];
      if (upd) {
        p[c] = adam_update(p[c], g, a.m + i, a.v + i, a.cfg.lr[0], b1, b2, eps, bc1, bc2);
        a.xy[i] = p[c];
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const size_t i = 3 * (size_t)n + c;
      const float g = a.g_chol[i];
      a.g_chol[i] = 0.f;
      p[2 + c] = a.chol[i];
      if (upd) {
        p[2 + c] = adam_update(p[2 + c], g, a.m + N2 + i, a.v + N2 + i, a.cfg.lr[1], b1, b2, eps,
                               bc1, bc2);
        a.chol[i] = p[2 + c];
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const size_t i = 3 * (size_t)n + c;
      const float g = a.g_rgb[i];
      a.g_rgb[i] = 0.f;
      if (upd)
        a.rgb[i] = adam_update(a.rgb[i], g, a.m + N5 + i, a.v + N5 + i, a.cfg.lr[2], b1, b2, eps,
                               bc1, bc2);
    }
    if (skin > 0.f)
      v = project_values<true>(n, TX, TY, inv_tile, p[0], p[1], p[2], p[3], p[4], geom, rect,
                               counts, skin, brect, &stale);
    else
      v = project_values(n, TX, TY, inv_tile, p[0], p[1], p[2], p[3], p[4], geom, rect, counts);
  }
  if (skin > 0.f) flag_stale(stale, misc);
  block_count_sums<WIDE_PROJ>(v, bsum + blockIdx.x, bcull + blockIdx.x);
}

// Exact (non-lazy) emission of the single-pass path: block 0 also clears
// the lazy lists' stamp, since these lists replace them.
__global__ void __launch_bounds__(WIDE_BLOCK)
k_emit_wide(int N, int TX, int nbp, int max_pairs, int D, const int4 *__restrict__ rect,
            const int *__restrict__ counts, const int *__restrict__ bsum,
            const int *__restrict__ bcull, int *__restrict__ offsets, uint32_t *__restrict__ keys,
            uint32_t *__restrict__ hist, int *__restrict__ misc, int *__restrict__ tick) {
  __shared__ EmitLds E;
  long long pre, end_keys, total;
  int culled;
  chunk_bounds<WIDE_BLOCK>(nbp, blockIdx.x, WIDE_GROUP, bsum, bcull, &pre, &end_keys, &total,
                           &culled);
  const int np = (int)min(total, (long long)max_pairs);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    offsets[N] = np;
    const uint32_t st = (total > (long long)max_pairs ? STATUS_OVERFLOW : 0u) |
                        (culled > 0 ? STATUS_CULLED : 0u);
    misc[MISC_N_PAIRS] = np;
    misc[MISC_STATUS] = (int)st;
    misc[MISC_N_CULLED] = culled;
    misc[MISC_STICKY] |= (int)st;
    misc[MISC_LISTS_LO] = misc[MISC_LISTS_HI] = 0;  // no longer lazy lists
    if (tick) tick[0] += 1;
  }
  emit_block_wide(blockIdx.x * WIDE_BLOCK, N, TX, pre, end_keys, np, D, rect, counts, offsets,
                  keys, hist + (size_t)blockIdx.x * D,
                  hist + WIDE_PART_ROWS + (size_t)blockIdx.x * (WIDE_SPLIT - 1) * D, E);
}

__global__ void __launch_bounds__(WIDE_SCATTER)
k_scatter_wide(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
               const int *__restrict__ misc, int nb, int nbp, int D, int bits, int n_tiles,
               const int *__restrict__ bsum, const int *__restrict__ bcull,
               const uint32_t *__restrict__ hist, int *__restrict__ tile_start) {
  __shared__ ScatterLds L;
  scatter_chunk_wide(in, out, nb, nbp, blockIdx.x / WIDE_SPLIT, blockIdx.x % WIDE_SPLIT, D, bits,
                     misc[MISC_N_PAIRS], n_tiles, bsum, bcull, hist, tile_start, L);
}

// Lazy binning's emission and scatter in one launch.  While the lists stay
// valid (misc[MISC_STALE] == 0) every block returns at once.  For a rebuild
// the blocks take roles in the order they start, by ticket: the first nbw
// emit one chunk each (k_emit_wide's work), the others each scatter one part
// of a chunk (k_scatter_wide's) once every chunk is emitted; blocks have
// the scatter's WIDE_SCATTER threads, an emission block taking two
// Gaussians per thread (the registers of 1024-thread blocks would not hold
// the scatter's key and histogram tiles).  A role is only
// ever held by a running block and emission waits for nothing, so the
// scatter's wait ends however many blocks are resident at once; it is also
// bounded (about 0.5 s), after which the block records STATUS_STALLED and
// skips its part, leaving the previous lists in place.  An emission block's
// writes are released device-wide (every wavefront's stores completed, a
// barrier, then one thread's release fence) before its chunk is counted, and a scatter block acquires them (one
// thread's acquire fence, then a barrier).  The last block to
// finish returns the three counters to zero.  It does not tick the step
// (the caller's raster does, so that the early return is a single load);
// the raster also stamps the rebuilt lists as complete (MISC_LISTS_LO/HI)
// unless a wait ran out.
__global__ void __launch_bounds__(WIDE_SCATTER)
k_bin_lazy_wide(int N, int TX, int nbp, int nbw, int max_pairs, int D, int bits, int n_tiles,
                const int4 *__restrict__ rect, const int *__restrict__ counts,
                const int *__restrict__ bsum, const int *__restrict__ bcull,
                int *__restrict__ offsets, uint32_t *__restrict__ ka, uint32_t *__restrict__ kb,
                uint32_t *__restrict__ hist, int *__restrict__ misc,
                int4 *__restrict__ brect, int *__restrict__ tile_start) {
  constexpr size_t RAW = sizeof(ScatterLds) > sizeof(EmitLds) ? sizeof(ScatterLds) : sizeof(EmitLds);
  __shared__ __align__(16) unsigned char raw[RAW];
  __shared__ unsigned s_ticket;
  __shared__ int s_go;
  const int tid = (int)threadIdx.x;
  if (misc[MISC_STALE] == 0) return;  // uniform over the grid
  unsigned *ctr = reinterpret_cast<unsigned *>(misc);
  if (tid == 0) s_ticket = atomicAdd(ctr + MISC_TICKET, 1u);
  __syncthreads();
  const int t = (int)s_ticket;
  if (t < nbw) {  // emission of chunk t
    for (int n = t * WIDE_BLOCK + tid; n < min(N, (t + 1) * WIDE_BLOCK); n += WIDE_SCATTER)
      brect[n] = rect[n];
    long long pre, end_keys, total;
    int culled;
    chunk_bounds<WIDE_SCATTER>(nbp, t, WIDE_GROUP, bsum, bcull, &pre, &end_keys, &total, &culled);
    const int np = (int)min(total, (long long)max_pairs);
    if (t == 0 && tid == 0) {
      offsets[N] = np;
      const uint32_t st = (total > (long long)max_pairs ? STATUS_OVERFLOW : 0u) |
                          (culled > 0 ? STATUS_CULLED : 0u);
      misc[MISC_N_PAIRS] = np;
      misc[MISC_STATUS] = (int)st;
      misc[MISC_N_CULLED] = culled;
      misc[MISC_STICKY] |= (int)st;
      misc[MISC_REBINS] += 1;
    }
    emit_block_wide<WIDE_SCATTER>(t * WIDE_BLOCK, N, TX, pre, end_keys, np, D, rect, counts,
                                  offsets, ka,
                    hist + (size_t)t * D, hist + WIDE_PART_ROWS + (size_t)t * (WIDE_SPLIT - 1) * D,
                    *reinterpret_cast<EmitLds *>(raw));
    // every wavefront's stores have completed before the barrier, so the
    // one-thread release after it covers them without relying on the order
    // in which the compute unit issues different wavefronts' requests
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (tid == 0) {
      __threadfence();  // release the block's writes (after the barrier: cumulative)
      atomicAdd(ctr + MISC_EMITTED, 1u);
    }
  } else {  // scatter of part (t - nbw) % WIDE_SPLIT of chunk (t - nbw) / WIDE_SPLIT
    if (tid == 0) {
      int go = 1;
      for (unsigned spin = 0;
           __hip_atomic_load(ctr + MISC_EMITTED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
           (unsigned)nbw;) {
        __builtin_amdgcn_s_sleep(2);
        if (++spin == (1u << 22)) {
          go = 0;
          atomicOr(misc + MISC_STICKY, (int)STATUS_STALLED);
          break;
        }
      }
      __threadfence();  // acquire the emitted keys and histograms (for the block: the barrier)
      s_go = go;
    }
    __syncthreads();
    if (s_go) {
      const int s = t - nbw;
      scatter_chunk_wide(ka, kb, nbw, nbp, s / WIDE_SPLIT, s % WIDE_SPLIT, D, bits,
                         misc[MISC_N_PAIRS], n_tiles, bsum, bcull, hist, tile_start,
                         *reinterpret_cast<ScatterLds *>(raw));
    }
  }
  if (tid == 0 && atomicAdd(ctr + MISC_FINISHED, 1u) == gridDim.x - 1) {
    atomicExch(ctr + MISC_TICKET, 0u);
    atomicExch(ctr + MISC_EMITTED, 0u);
    atomicExch(ctr + MISC_FINISHED, 0u);
  }
}

// ------------------------------------------------------------ radix sort --
// First pass: block b scatters the keys emission block b wrote (its range
// recomputed from the block sums), on the low tile byte.
__global__ void __launch_bounds__(SORT_BLOCK)
k_scatter_first(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                const int *__restrict__ misc, int nb, const int *__restrict__ bsum,
                const int *__restrict__ bcull, const uint32_t *__restrict__ hist) {
  long long pre, total;
  int culled;
  block_sum_prefix(nb, blockIdx.x, bsum, bcull, &pre, &total, &culled);
  const long long n = misc[MISC_N_PAIRS];
  const int beg = (int)min(pre, n), end = (int)min(pre + bsum[blockIdx.x], n);
  scatter_chunk(in, out, beg, end, nb, blockIdx.x, 16, hist);
}

// Later passes over G fixed chunks: per-chunk histogram, then scatter.
__global__ void __launch_bounds__(SORT_BLOCK)
k_radix_hist(const uint32_t *__restrict__ keys, const int *__restrict__ misc, int shift, int G,
             uint32_t *__restrict__ hist) {
  chunk_histogram(keys, misc[MISC_N_PAIRS], G, blockIdx.x, shift, hist);
}

__global__ void __launch_bounds__(SORT_BLOCK)
k_radix_scatter(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                const int *__restrict__ misc, int shift, int G, const uint32_t *__restrict__ hist) {
  const int n = misc[MISC_N_PAIRS];
  const int chunk = chunk_len(n, G);
  int beg, end;
  sort_chunk(n, G, blockIdx.x, &beg, &end);
  scatter_chunk(in, out, beg, end, (n + chunk - 1) / chunk, blockIdx.x, shift, hist);
}

// --------------------------------------------------------------- ranges --
__global__ void __launch_bounds__(256)
k_tile_ranges(const uint32_t *__restrict__ keys, const int *__restrict__ misc, int n_tiles,
              int *__restrict__ tile_start) {
  tile_ranges(keys, misc[MISC_N_PAIRS], n_tiles, tile_start);
}

hipError_t launch_binning(const Layout &L, const float *xy, const float *chol, void *ws,
                          hipStream_t st, int *step_tick, const PendingAdam *adam, float skin) {
  float4 *geom = at<float4>(ws, L.geom);
  int *counts = at<int>(ws, L.counts);
  int *offsets = at<int>(ws, L.offsets);
  int *misc = at<int>(ws, L.misc);
  int4 *rect = at<int4>(ws, L.rect);
  int *bsum = at<int>(ws, L.blocks);
  int *bcull = bsum + BIN_BLOCK;
  uint32_t *hist = at<uint32_t>(ws, L.hist);
  uint32_t *ka = at<uint32_t>(ws, L.keys_a), *kb = at<uint32_t>(ws, L.keys_b);
  if (L.wide) {
    const int nbw = (L.N + WIDE_BLOCK - 1) / WIDE_BLOCK;  // chunks
    const int nbp = (L.N + WIDE_PROJ - 1) / WIDE_PROJ;    // projection blocks
    const int lazy = skin > 0.f ? 1 : 0;
    int4 *brect = at<int4>(ws, L.brect);
    if (adam)
      hipLaunchKernelGGL(k_adam_project_wide, dim3(nbp + 1), dim3(WIDE_PROJ), 0, st, L.N, L.TX, L.TY,
                         1.0f / (float)L.T, *adam, geom, rect, counts, bsum, bcull, skin, brect,
                         misc);
    else
      hipLaunchKernelGGL(k_project_wide, dim3(nbp), dim3(WIDE_PROJ), 0, st, L.N, L.TX, L.TY,
                         1.0f / (float)L.T, xy, chol, geom, rect, counts, bsum, bcull, skin, brect,
                         misc);
    if (lazy) {
      hipLaunchKernelGGL(k_bin_lazy_wide, dim3(nbw * (1 + WIDE_SPLIT)), dim3(WIDE_SCATTER), 0, st,
                         L.N, L.TX, nbp, nbw, L.max_pairs, L.D, L.digit_bits, L.n_tiles, rect,
                         counts, bsum, bcull, offsets, ka, kb, hist, misc, brect,
                         at<int>(ws, L.tile_start));
      return hipGetLastError();
    }
    hipLaunchKernelGGL(k_emit_wide, dim3(nbw), dim3(WIDE_BLOCK), 0, st, L.N, L.TX, nbp,
                       L.max_pairs, L.D, rect, counts, bsum, bcull, offsets, ka, hist, misc,
                       step_tick);
    hipLaunchKernelGGL(k_scatter_wide, dim3(nbw * WIDE_SPLIT), dim3(WIDE_SCATTER), 0, st, ka, kb,
                       misc, nbw, nbp, L.D, L.digit_bits, L.n_tiles, bsum, bcull, hist,
                       at<int>(ws, L.tile_start));
    return hipGetLastError();
  }
  if (adam) {
    const PendingAdam &a = *adam;
    const hipError_t e = launch_adam(L.N, a.xy, a.chol, a.rgb, a.g_xy, a.g_chol, a.g_rgb, a.m, a.v,
                                     const_cast<int32_t *>(a.step), a.cfg, a.active, 1, a.loss_part,
                                     a.n_part, a.loss_scale, a.trace, a.trace_len, st);
    if (e != hipSuccess) return e;
  }
  const int nb = (L.N + BIN_BLOCK - 1) / BIN_BLOCK;
  hipLaunchKernelGGL(k_project, dim3(nb), dim3(BIN_BLOCK), 0, st, L.N, L.TX, L.TY,
                     1.0f / (float)L.T, xy, chol, geom, rect, counts, bsum, bcull);
  hipLaunchKernelGGL(k_emit_keys, dim3(nb), dim3(BIN_BLOCK), 0, st, L.N, L.TX, nb, L.max_pairs,
                     rect, counts, bsum, bcull, offsets, ka, hist, misc, step_tick);
  hipLaunchKernelGGL(k_scatter_first, dim3(nb), dim3(SORT_BLOCK), 0, st, ka, kb, misc, nb, bsum,
                     bcull, hist);
  const uint32_t *sorted = kb;
  if (L.sort_passes == 2) {
    const int G = L.sort_blocks;
    hipLaunchKernelGGL(k_radix_hist, dim3(G), dim3(SORT_BLOCK), 0, st, kb, misc, 16 + RADIX_BITS,
                       G, hist);
    hipLaunchKernelGGL(k_radix_scatter, dim3(G), dim3(SORT_BLOCK), 0, st, kb, ka, misc,
                       16 + RADIX_BITS, G, hist);
    sorted = ka;
  }
  hipLaunchKernelGGL(k_tile_ranges, dim3(256), dim3(256), 0, st, sorted, misc, L.n_tiles,
                     at<int>(ws, L.tile_start));
  return hipGetLastError();
}

hipError_t launch_radix_sort_tiles(uint32_t *a, uint32_t *b, const int *misc, int G, uint32_t *hist,
                                   int passes, hipStream_t st, const uint32_t **sorted) {
  uint32_t *src = a, *dst = b;
  for (int p = 0; p < passes; ++p) {
    const int shift = 16 + RADIX_BITS * p;
    hipLaunchKernelGGL(k_radix_hist, dim3(G), dim3(SORT_BLOCK), 0, st, src, misc, shift, G, hist);
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
