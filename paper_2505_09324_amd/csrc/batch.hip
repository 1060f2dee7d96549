// Batched fitting: many frames of different sizes and Gaussian counts fitted
// in lockstep, one launch per stage per iteration.
//
//  - binning runs segmented per frame with the same launches as one frame:
//    one thread per Gaussian of the whole batch for projection and key
//    emission, the first radix pass over each emission block's keys, a
//    block table mapping the second pass's blocks to (frame, key chunk),
//    and a (block, frame) grid for the tile ranges;
//  - the raster is ONE launch per iteration over a queue of (frame, tile)
//    work items, largest frames first, running the same fused forward +
//    loss + backward tile code as the one-frame kernel: by default one
//    workgroup per item in queue order (the one-frame kernel's single-tile
//    path with exact block masks), or (gs2d_fit_opts.batch_persistent) a
//    grid sized to the device's resident capacity that pulls the items
//    through an atomic counter;
//  - Adam runs over the concatenated parameters of all frames; a per-frame
//    reduction writes each frame's loss into its column of the trace.
// Keys, geometry and tile lists stay frame-local (16-bit Gaussian index,
// frame-local tile id), so every frame's lists are identical to what the
// one-frame path produces for it alone.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <vector>

#include "bin_common.h"
#include "raster_tile.h"

namespace gs2d {

namespace {

// Device descriptor of one frame of a batch (offsets in elements).
struct BFrame {
  int W, H, N, TX, TY, n_tiles, G, cap;
  int nb;              // projection blocks of BIN_BLOCK Gaussians
  int blk_off;         // first projection block of the frame
  long long g_off;     // first Gaussian of the frame in the concatenated arrays
  long long px_off;    // first float of the frame's target ([3][H][W])
  long long key_off;   // first key slot
  long long hist_off;  // first word of the frame's second-pass histogram (RADIX * G)
  long long tile_off;  // first tile of the frame among all tiles of the batch
};

// Per-frame status words.  Lazy binning (gs2d_fit_opts.bin_skin > 0):
// BM_VALID = 1 while the frame's lists hold every pair of the rectangles in
// brect (set after each iteration by k_b_loss, cleared by the projection
// when a Gaussian leaves its rectangle; 0 at the start of a call), and
// BM_REBINS counts the frame's rebuilds.
enum BMisc : int {
  BM_N_PAIRS = 0,
  BM_STATUS = 1,
  BM_N_CULLED = 2,
  BM_STICKY = 3,
  BM_VALID = 4,
  BM_REBINS = 5,
  BM_STRIDE = 8
};

struct BatchLayout {
  int F, T, ppl, passes, sort_blocks, proj_blocks;
  int nw;  // raster wavefronts per tile: loss partials per tile
  long long Ntot, keys_tot, hist_tot, tiles_tot;
  size_t desc, blk_frame, blk_chunk, pblk_frame, queue, geom, rect, brect, counts, offsets, bsum,
      bcull, keys_a, keys_b, hist, hist2, tile_start, loss_part, grads, misc, counter, total;
  std::vector<BFrame> frames;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool batch_layout(int F, const gs2d_frame *fr, int tile, int ppl_in, BatchLayout *B) {
  if (F < 1 || F > 4096 || !fr) return false;
  if (tile != 8 && tile != 16 && tile != 32) return false;
  const int ppl = ppl_in == 0 ? 1 : ppl_in;
  if ((ppl != 1 && ppl != 2 && ppl != 4) || 8 * ppl > tile) return false;
  B->F = F;
  B->T = tile;
  B->ppl = ppl;
  B->nw = (tile / 8) * (tile / (8 * ppl));
  B->frames.resize(F);
  long long g = 0, px = 0, key = 0, hist = 0, tiles = 0;
  int blocks = 0, pblocks = 0, maxbits = 1;
  for (int f = 0; f < F; ++f) {
    const gs2d_frame &s = fr[f];
    if (s.W < 1 || s.H < 1 || s.N < 1 || s.N > 65536) return false;
    BFrame &d = B->frames[f];
    d.W = s.W;
    d.H = s.H;
    d.N = s.N;
    d.TX = (s.W + tile - 1) / tile;
    d.TY = (s.H + tile - 1) / tile;
    if ((long long)d.TX * d.TY > 65536) return false;
    d.n_tiles = d.TX * d.TY;
    const long long cap = std::max<long long>(1 << 16, 16LL * s.N + 4LL * d.n_tiles);
    if (cap > (1 << 30)) return false;
    d.cap = (int)cap;
    d.G = std::min(SORT_MAX_BLOCKS, (s.N + 255) / 256);
    d.nb = (s.N + BIN_BLOCK - 1) / BIN_BLOCK;
    d.blk_off = pblocks;
    pblocks += d.nb;
    d.g_off = g;
    d.px_off = px;
    d.key_off = key;
    d.hist_off = hist;
    d.tile_off = tiles;
    g += s.N;
    px += 3LL * s.W * s.H;
    key += d.cap;
    hist += (long long)RADIX * d.G;
    tiles += d.n_tiles;
    blocks += d.G;
    int bits = 1;
    while ((1LL << bits) < (long long)d.n_tiles) ++bits;
    maxbits = std::max(maxbits, bits);
  }
  B->passes = (maxbits + RADIX_BITS - 1) / RADIX_BITS;
  B->sort_blocks = blocks;
  B->proj_blocks = pblocks;
  B->Ntot = g;
  B->keys_tot = key;
  B->hist_tot = hist;
  B->tiles_tot = tiles;
  size_t o = 0;
  auto take = [&o](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  B->desc = take(sizeof(BFrame) * F);
  B->blk_frame = take(4 * (size_t)blocks);
  B->blk_chunk = take(4 * (size_t)blocks);
  B->pblk_frame = take(4 * (size_t)pblocks);
  B->queue = take(4 * (size_t)tiles);
  B->geom = take(32 * (size_t)g);
  B->rect = take(16 * (size_t)g);
  B->brect = take(16 * (size_t)g);  // lazy binning: the rectangles the lists were built from
  B->counts = take(4 * (size_t)g);
  B->offsets = take(4 * ((size_t)g + F));
  B->bsum = take(4 * (size_t)pblocks);
  B->bcull = take(4 * (size_t)pblocks);
  B->keys_a = take(4 * (size_t)key);
  B->keys_b = take(4 * (size_t)key);
  B->hist = take(4 * (size_t)RADIX * pblocks);
  B->hist2 = take(4 * (size_t)hist);
  B->tile_start = take(4 * ((size_t)tiles + F));
  B->loss_part = take(4 * (size_t)tiles * B->nw);
  B->grads = take(32 * (size_t)g);
  B->misc = take(4 * (size_t)BM_STRIDE * F);
  B->counter = take(64);
  B->total = o;
  return true;
}

// ------------------------------------------------------------ binning ----
// Projection blocks never straddle frames: block b covers Gaussians
// [b - blk_off, ...) * BIN_BLOCK of frame pblk_frame[b].  With skin > 0
// (lazy binning) the rectangles are grown by the skin and a Gaussian whose
// exact rectangle has left brect (or that is culled with keys) marks its
// frame's lists invalid.
__global__ void __launch_bounds__(BIN_BLOCK)
k_b_project(const BFrame *__restrict__ D, const int *__restrict__ pblk_frame, int tile,
            const float *__restrict__ xy, const float *__restrict__ chol, float4 *__restrict__ geom,
            int4 *__restrict__ rect, int *__restrict__ counts, int *__restrict__ bsum,
            int *__restrict__ bcull, float skin, const int4 *__restrict__ brect,
            int *__restrict__ misc) {
  const int f = pblk_frame[blockIdx.x];
  const BFrame d = D[f];
  const int c = blockIdx.x - d.blk_off;
  const long long g = d.g_off;
  if (skin > 0.f) {
    const int n = c * BIN_BLOCK + (int)threadIdx.x;
    int v = 0;
    bool stale = false;
    if (n < d.N) {
      const long long i = g + n;
      v = project_values<true>(n, d.TX, d.TY, 1.0f / (float)tile, xy[2 * i], xy[2 * i + 1],
                               chol[3 * i], chol[3 * i + 1], chol[3 * i + 2], geom + 2 * g,
                               rect + g, counts + g, skin, brect + g, &stale);
    }
    if (__ballot(stale) && (threadIdx.x & 63) == 0) misc[BM_STRIDE * f + BM_VALID] = 0;
    block_count_sums<BIN_BLOCK>(v, bsum + blockIdx.x, bcull + blockIdx.x);
    return;
  }
  project_block(c * BIN_BLOCK, d.N, d.TX, d.TY, 1.0f / (float)tile, xy + 2 * g, chol + 3 * g,
                geom + 2 * g, rect + g, counts + g, bsum + blockIdx.x, bcull + blockIdx.x);
}

// Key emission of projection block b of frame f: prefix of its pair count
// among the frame's blocks, then the keys and histogram row b of the first
// radix pass.  The frame's first block publishes its pair
// count and status; block 0 also advances the step counter (when given) and
// clears the persistent raster's work counter for this iteration.  lazy:
// a frame whose lists are still valid keeps them (its blocks return), a
// rebuild records the rectangles it bins in brect and counts itself.
__global__ void __launch_bounds__(BIN_BLOCK)
k_b_emit_keys(const BFrame *__restrict__ D, const int *__restrict__ pblk_frame,
              const int4 *__restrict__ rect, const int *__restrict__ counts,
              const int *__restrict__ bsum, const int *__restrict__ bcull,
              int *__restrict__ offsets, uint32_t *__restrict__ keys, uint32_t *__restrict__ hist,
              int *__restrict__ misc, int *__restrict__ tick, unsigned *__restrict__ work_counter,
              int lazy, int4 *__restrict__ brect) {
  const int f = pblk_frame[blockIdx.x];
  const BFrame d = D[f];
  const int c = blockIdx.x - d.blk_off;
  if (lazy) {
    if (misc[BM_STRIDE * f + BM_VALID]) {  // uniform over the frame's blocks
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (tick) tick[0] += 1;
        work_counter[0] = 0u;
      }
      return;
    }
    const int n = c * BIN_BLOCK + (int)threadIdx.x;
    if (n < d.N) brect[d.g_off + n] = rect[d.g_off + n];
    if (c == 0 && threadIdx.x == 0) misc[BM_STRIDE * f + BM_REBINS] += 1;
  }
  long long pre, total;
  int culled;
  block_sum_prefix(d.nb, c, bsum + d.blk_off, bcull + d.blk_off, &pre, &total, &culled);
  const int np = (int)min(total, (long long)d.cap);
  if (c == 0 && threadIdx.x == 0) {
    offsets[d.g_off + f + d.N] = np;
    const int st = (total > (long long)d.cap ? (int)STATUS_OVERFLOW : 0) |
                   (culled > 0 ? (int)STATUS_CULLED : 0);
    int *m = misc + BM_STRIDE * f;
    m[BM_N_PAIRS] = np;
    m[BM_STATUS] = st;
    m[BM_N_CULLED] = culled;
    m[BM_STICKY] |= st;
    if (f == 0) {
      if (tick) tick[0] += 1;
      work_counter[0] = 0u;
    }
  }
  emit_block(c * BIN_BLOCK, d.N, d.TX, pre, np, rect + d.g_off, counts + d.g_off,
             offsets + d.g_off + f, keys + d.key_off, hist + (size_t)blockIdx.x * RADIX);
}

// First radix pass: block b scatters the keys emission block b wrote.
__global__ void __launch_bounds__(SORT_BLOCK)
k_b_scatter_first(const BFrame *__restrict__ D, const int *__restrict__ pblk_frame,
                  const int *__restrict__ misc, const int *__restrict__ bsum,
                  const int *__restrict__ bcull, const uint32_t *__restrict__ in_all,
                  uint32_t *__restrict__ out_all, const uint32_t *__restrict__ hist, int lazy) {
  const int f = pblk_frame[blockIdx.x];
  if (lazy && misc[BM_STRIDE * f + BM_VALID]) return;  // the frame keeps its lists
  const BFrame d = D[f];
  const int c = blockIdx.x - d.blk_off;
  long long pre, total;
  int culled;
  block_sum_prefix(d.nb, c, bsum + d.blk_off, bcull + d.blk_off, &pre, &total, &culled);
  const long long n = misc[BM_STRIDE * f + BM_N_PAIRS];
  const int beg = (int)min(pre, n), end = (int)min(pre + bsum[blockIdx.x], n);
  scatter_chunk(in_all + d.key_off, out_all + d.key_off, beg, end, d.nb, c, 16,
                hist + (size_t)d.blk_off * RADIX);
}

// Second pass over the frame's G fixed chunks: histogram, then scatter.
__global__ void __launch_bounds__(SORT_BLOCK)
k_b_radix_hist(const BFrame *__restrict__ D, const int *__restrict__ blk_frame,
               const int *__restrict__ blk_chunk, const int *__restrict__ misc,
               const uint32_t *__restrict__ keys, int shift, uint32_t *__restrict__ hist, int lazy) {
  const int f = blk_frame[blockIdx.x], c = blk_chunk[blockIdx.x];
  if (lazy && misc[BM_STRIDE * f + BM_VALID]) return;
  const BFrame d = D[f];
  chunk_histogram(keys + d.key_off, misc[BM_STRIDE * f + BM_N_PAIRS], d.G, c, shift,
                  hist + d.hist_off);
}

__global__ void __launch_bounds__(SORT_BLOCK)
k_b_radix_scatter(const BFrame *__restrict__ D, const int *__restrict__ blk_frame,
                  const int *__restrict__ blk_chunk, const int *__restrict__ misc,
                  const uint32_t *__restrict__ in_all, uint32_t *__restrict__ out_all, int shift,
                  const uint32_t *__restrict__ hist, int lazy) {
  const int f = blk_frame[blockIdx.x], c = blk_chunk[blockIdx.x];
  if (lazy && misc[BM_STRIDE * f + BM_VALID]) return;
  const BFrame d = D[f];
  const int n = misc[BM_STRIDE * f + BM_N_PAIRS];
  const int chunk = chunk_len(n, d.G);
  int beg, end;
  sort_chunk(n, d.G, c, &beg, &end);
  scatter_chunk(in_all + d.key_off, out_all + d.key_off, beg, end, (n + chunk - 1) / chunk, c,
                shift, hist + d.hist_off);
}

// Grid (RB, F): tile ranges of frame blockIdx.y.
__global__ void __launch_bounds__(256)
k_b_tile_ranges(const BFrame *__restrict__ D, const int *__restrict__ misc,
                const uint32_t *__restrict__ keys_all, int *__restrict__ tile_start_all, int lazy) {
  const int f = blockIdx.y;
  if (lazy && misc[BM_STRIDE * f + BM_VALID]) return;
  const BFrame d = D[f];
  tile_ranges(keys_all + d.key_off, misc[BM_STRIDE * f + BM_N_PAIRS], d.n_tiles,
              tile_start_all + d.tile_off + f);
}

// ------------------------------------------------------------- raster ----
struct BatchRaster {
  const BFrame *D;
  const uint32_t *queue;  // (frame << 16) | tile, processing order
  unsigned n_items;
  unsigned *counter;
  const float4 *geom;
  const uint32_t *keys;
  const int *tile_start;
  const float *rgb;
  const float *targets;
  float *loss_part;
  float *g_xy, *g_chol, *g_rgb;
};

template <int TILE, int PPL>
__global__ void __launch_bounds__((Cfg<TILE, PPL>::NT)) GS2D_RASTER_OCCUPANCY
k_b_render_persistent(BatchRaster a) {
  using C = Cfg<TILE, PPL>;
  __shared__ Smem<C::NW> S;
  __shared__ float acc[CH * 8];
  __shared__ unsigned s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1u);
    __syncthreads();
    const unsigned item = s_item;
    __syncthreads();
    if (item >= a.n_items) break;  // every wavefront leaves together
    const uint32_t q = a.queue[item];
    const int f = (int)(q >> 16), t = (int)(q & 0xFFFFu);
    const BFrame d = a.D[f];
    FrameArgs fa;
    fa.W = d.W;
    fa.H = d.H;
    fa.TX = d.TX;
    fa.geom = a.geom + 2 * d.g_off;
    fa.keys = a.keys + d.key_off;
    fa.tile_start = a.tile_start + d.tile_off + f;
    fa.rgb = a.rgb + 3 * d.g_off;
    fa.active = nullptr;
    fa.lazy_misc = nullptr;
    fa.sig_lo = fa.sig_hi = 0;
    fa.tick = nullptr;
    const float gs = (float)(2.0 / (3.0 * (double)d.W * (double)d.H));
    fused_tile<TILE, PPL, false>(S, acc, fa, t, a.targets + d.px_off,
                          a.loss_part + (d.tile_off + t) * Cfg<TILE, PPL>::NW, gs,
                          a.g_xy + 2 * d.g_off, a.g_chol + 3 * d.g_off, a.g_rgb + 3 * d.g_off);
  }
}

// One workgroup per queue item (the queue's order is the dispatch order):
// the one-frame kernel's single-tile path, exact block masks included.
template <int TILE, int PPL>
__global__ void __launch_bounds__((Cfg<TILE, PPL>::NT)) GS2D_RASTER_OCCUPANCY
k_b_render_grid(BatchRaster a) {
  using C = Cfg<TILE, PPL>;
  __shared__ Smem<C::NW> S;
  __shared__ float acc[CH * 8];
  const uint32_t q = a.queue[blockIdx.x];
  const int f = (int)(q >> 16), t = (int)(q & 0xFFFFu);
  const BFrame d = a.D[f];
  FrameArgs fa;
  fa.W = d.W;
  fa.H = d.H;
  fa.TX = d.TX;
  fa.geom = a.geom + 2 * d.g_off;
  fa.keys = a.keys + d.key_off;
  fa.tile_start = a.tile_start + d.tile_off + f;
  fa.rgb = a.rgb + 3 * d.g_off;
  fa.active = nullptr;
  fa.lazy_misc = nullptr;
  fa.sig_lo = fa.sig_hi = 0;
  fa.tick = nullptr;
  const float gs = (float)(2.0 / (3.0 * (double)d.W * (double)d.H));
  fused_tile<TILE, PPL, true, true>(S, acc, fa, t, a.targets + d.px_off,
                                    a.loss_part + (d.tile_off + t) * C::NW, gs,
                                    a.g_xy + 2 * d.g_off, a.g_chol + 3 * d.g_off,
                                    a.g_rgb + 3 * d.g_off);
}

// One block per frame: loss of this iteration into trace[(t-1) * F + f].
__global__ void __launch_bounds__(256)
k_b_loss(const BFrame *__restrict__ D, int F, int nw, const float *__restrict__ loss_part,
         const int *__restrict__ step, float *__restrict__ trace, int trace_rows,
         int *__restrict__ lazy_misc) {
  __shared__ double red[4];
  const int f = blockIdx.x;
  const BFrame d = D[f];
  double s = 0.0;
  const float *lp = loss_part + d.tile_off * nw;
  s = thread_sum_parts(lp, d.n_tiles * nw);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    // lazy binning: the binning kernels are done, so frame f's lists now
    // hold every pair of the rectangles in brect
    if (lazy_misc) lazy_misc[BM_STRIDE * f + BM_VALID] = 1;
    const int row = step[0] - 1;
    if (row >= 0 && row < trace_rows)
      trace[(size_t)row * F + f] =
          (float)((red[0] + red[1] + red[2] + red[3]) / (3.0 * (double)d.W * (double)d.H));
  }
}

// ------------------------------------------------------------- host side --
struct BatchRun {
  BatchLayout B;
  void *ws;
  int grid;  // persistent raster grid
};

hipError_t upload_tables(const BatchLayout &B, void *ws, hipStream_t st) {
  std::vector<int> bf, bc, pf;
  std::vector<uint32_t> queue;
  queue.reserve((size_t)B.tiles_tot);
  for (int f = 0; f < B.F; ++f) {
    const BFrame &d = B.frames[f];
    for (int c = 0; c < d.G; ++c) {
      bf.push_back(f);
      bc.push_back(c);
    }
    for (int c = 0; c < d.nb; ++c) pf.push_back(f);
  }
  // work order: frames by decreasing area (largest lists first), tiles in order
  std::vector<int> order(B.F);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return (long long)B.frames[a].W * B.frames[a].H > (long long)B.frames[b].W * B.frames[b].H;
  });
  for (int f : order)
    for (int t = 0; t < B.frames[f].n_tiles; ++t) queue.push_back(((uint32_t)f << 16) | (uint32_t)t);
  hipError_t e = hipMemcpyAsync(at<char>(ws, B.desc), B.frames.data(), sizeof(BFrame) * B.F,
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(at<char>(ws, B.blk_frame), bf.data(), 4 * bf.size(), hipMemcpyHostToDevice,
                       st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(at<char>(ws, B.blk_chunk), bc.data(), 4 * bc.size(), hipMemcpyHostToDevice,
                       st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(at<char>(ws, B.pblk_frame), pf.data(), 4 * pf.size(), hipMemcpyHostToDevice,
                       st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(at<char>(ws, B.queue), queue.data(), 4 * queue.size(),
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);  // host vectors go out of scope
  return e;
}

template <int TT, int PP>
int persistent_grid() {
  int dev = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_b_render_persistent<TT, PP>,
                                                   Cfg<TT, PP>::NT, 0) != hipSuccess)
    return 0;
  return std::max(1, per_cu) * prop.multiProcessorCount;
}

int batch_grid(const BatchLayout &B) {
#define CASE(TT, PP) \
  if (B.T == TT && B.ppl == PP) return persistent_grid<TT, PP>();
  CASE(8, 1) CASE(16, 1) CASE(16, 2) CASE(32, 1) CASE(32, 2) CASE(32, 4)
#undef CASE
  return 0;
}

// Binning of every frame of the batch; skin > 0: lazy binning (each frame
// rebuilds its lists only when a Gaussian has left its recorded rectangle,
// or at the first iteration of a call).
hipError_t enqueue_batch_binning(const BatchLayout &B, void *ws, const float *xy, const float *chol,
                                 int *tick, hipStream_t st, float skin = 0.f) {
  const int lazy = skin > 0.f ? 1 : 0;
  int4 *brect = at<int4>(ws, B.brect);
  const BFrame *D = at<const BFrame>(ws, B.desc);
  const int *bf = at<const int>(ws, B.blk_frame), *bc = at<const int>(ws, B.blk_chunk);
  float4 *geom = at<float4>(ws, B.geom);
  int4 *rect = at<int4>(ws, B.rect);
  int *counts = at<int>(ws, B.counts), *offsets = at<int>(ws, B.offsets);
  int *misc = at<int>(ws, B.misc);
  unsigned *counter = at<unsigned>(ws, B.counter);
  uint32_t *ka = at<uint32_t>(ws, B.keys_a), *kb = at<uint32_t>(ws, B.keys_b);
  uint32_t *hist = at<uint32_t>(ws, B.hist), *hist2 = at<uint32_t>(ws, B.hist2);
  const int *pf = at<const int>(ws, B.pblk_frame);
  int *bsum = at<int>(ws, B.bsum), *bcull = at<int>(ws, B.bcull);
  hipLaunchKernelGGL(k_b_project, dim3(B.proj_blocks), dim3(BIN_BLOCK), 0, st, D, pf, B.T, xy, chol,
                     geom, rect, counts, bsum, bcull, skin, brect, misc);
  hipLaunchKernelGGL(k_b_emit_keys, dim3(B.proj_blocks), dim3(BIN_BLOCK), 0, st, D, pf, rect, counts,
                     bsum, bcull, offsets, ka, hist, misc, tick, counter, lazy, brect);
  hipLaunchKernelGGL(k_b_scatter_first, dim3(B.proj_blocks), dim3(SORT_BLOCK), 0, st, D, pf, misc,
                     bsum, bcull, ka, kb, hist, lazy);
  const uint32_t *sorted = kb;
  if (B.passes == 2) {
    hipLaunchKernelGGL(k_b_radix_hist, dim3(B.sort_blocks), dim3(SORT_BLOCK), 0, st, D, bf, bc,
                       misc, kb, 16 + RADIX_BITS, hist2, lazy);
    hipLaunchKernelGGL(k_b_radix_scatter, dim3(B.sort_blocks), dim3(SORT_BLOCK), 0, st, D, bf, bc,
                       misc, kb, ka, 16 + RADIX_BITS, hist2, lazy);
    sorted = ka;
  }
  hipLaunchKernelGGL(k_b_tile_ranges, dim3(32, B.F), dim3(256), 0, st, D, misc, sorted,
                     at<int>(ws, B.tile_start), lazy);
  return hipGetLastError();
}

const uint32_t *batch_sorted_keys(const BatchLayout &B, void *ws) {
  return at<const uint32_t>(ws, (B.passes & 1) ? B.keys_b : B.keys_a);
}

// The fused raster of every (frame, tile) item: one workgroup per item, or
// with `persistent` a grid of `grid` workgroups popping the items.
hipError_t enqueue_batch_raster(const BatchLayout &B, void *ws, int grid, const float *rgb,
                                const float *targets, float *g_xy, float *g_chol, float *g_rgb,
                                hipStream_t st, bool persistent = false) {
  BatchRaster a;
  a.D = at<const BFrame>(ws, B.desc);
  a.queue = at<const uint32_t>(ws, B.queue);
  a.n_items = (unsigned)B.tiles_tot;
  a.counter = at<unsigned>(ws, B.counter);
  a.geom = at<const float4>(ws, B.geom);
  a.keys = batch_sorted_keys(B, ws);
  a.tile_start = at<const int>(ws, B.tile_start);
  a.rgb = rgb;
  a.targets = targets;
  a.loss_part = at<float>(ws, B.loss_part);
  a.g_xy = g_xy;
  a.g_chol = g_chol;
  a.g_rgb = g_rgb;
  bool done = false;
#define CASE(TT, PP)                                                                          \
  if (!done && B.T == TT && B.ppl == PP) {                                                    \
    if (persistent)                                                                          \
      hipLaunchKernelGGL((k_b_render_persistent<TT, PP>), dim3(grid), dim3(Cfg<TT, PP>::NT),   \
                         0, st, a);                                                           \
    else                                                                                      \
      hipLaunchKernelGGL((k_b_render_grid<TT, PP>), dim3(a.n_items), dim3(Cfg<TT, PP>::NT), 0, \
                         st, a);                                                              \
    done = true;                                                                              \
  }
  CASE(8, 1) CASE(16, 1) CASE(16, 2) CASE(32, 1) CASE(32, 2) CASE(32, 4)
#undef CASE
  return done ? hipGetLastError() : hipErrorInvalidValue;
}

hipError_t enqueue_batch_iteration(const BatchLayout &B, void *ws, int grid, const float *targets,
                                   float *xy, float *chol, float *rgb, float *m, float *v,
                                   int32_t *step, float *trace, int trace_rows,
                                   const gs2d_adam_cfg &cfg, hipStream_t st, float skin,
                                   bool persistent) {
  float *g = at<float>(ws, B.grads);
  float *g_xy = g, *g_chol = g + 2 * B.Ntot, *g_rgb = g + 5 * B.Ntot;
  hipError_t e = enqueue_batch_binning(B, ws, xy, chol, step, st, skin);
  if (e == hipSuccess)
    e = enqueue_batch_raster(B, ws, grid, rgb, targets, g_xy, g_chol, g_rgb, st, persistent);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_b_loss, dim3(B.F), dim3(256), 0, st, at<const BFrame>(ws, B.desc), B.F,
                       B.nw, at<const float>(ws, B.loss_part), step, trace, trace_rows,
                       skin > 0.f ? at<int>(ws, B.misc) : nullptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = launch_adam((int)B.Ntot, xy, chol, rgb, g_xy, g_chol, g_rgb, m, v, step, cfg, nullptr, 1,
                    nullptr, 0, 0.f, nullptr, 0, st);
  return e;
}

int check_batch_ws(int F, const gs2d_frame *frames, int tile, int ppl, void *ws, size_t ws_bytes,
                   BatchLayout *B) {
  if (!batch_layout(F, frames, tile, ppl, B)) return GS2D_EINVAL;
  if (B->Ntot > (1LL << 31) / 8) return GS2D_EINVAL;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return GS2D_EINVAL;
  if (ws_bytes < B->total) return GS2D_ENOSPACE;
  return GS2D_OK;
}

struct Events {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~Events() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

}  // namespace

}  // namespace gs2d

using namespace gs2d;

extern "C" size_t gs2d_batch_workspace_bytes(int32_t n_frames, const gs2d_frame *frames,
                                             int32_t tile, int32_t px_per_lane) {
  try {
    BatchLayout B;
    return batch_layout(n_frames, frames, tile, px_per_lane, &B) ? B.total : 0;
  } catch (...) {
    return 0;
  }
}

extern "C" int gs2d_fit_batch(gs2d_ctx *ctx, int32_t n_frames, const gs2d_frame *frames,
                              int32_t tile, int32_t px_per_lane, const float *targets, float *xy,
                              float *chol, float *rgb, float *m, float *v, int32_t *step,
                              float *loss_trace, int32_t trace_rows, void *ws, size_t ws_bytes,
                              const gs2d_fit_opts *opts, gs2d_fit_stats *stats, void *stream) {
  try {
    const auto t0 = std::chrono::steady_clock::now();
    BatchLayout B;
    int rc = check_batch_ws(n_frames, frames, tile, px_per_lane, ws, ws_bytes, &B);
    if (rc != GS2D_OK) return rc;
    if (!targets || !xy || !chol || !rgb || !m || !v || !step || !loss_trace || !opts)
      return GS2D_EINVAL;
    if (opts->iters < 0 || opts->check_every < 1 || opts->active || opts->qat) return GS2D_EINVAL;
    if (!(opts->bin_skin >= 0.f && opts->bin_skin <= 64.f)) return GS2D_EINVAL;
    rc = gs2d_ctx_check(ctx);
    if (rc != GS2D_OK) return rc;
    if (stats) {
      stats->iters_run = 0;
      stats->iter_hit_target = -1;
      stats->final_loss = NAN;
      stats->final_psnr = NAN;
      stats->seconds = 0.0;
      stats->status = 0;
      stats->n_culled = 0;
      stats->rebins = 0;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int32_t step0 = 0;
    if (hipMemcpyAsync(&step0, step, sizeof(int32_t), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return GS2D_EHIP;
    if (step0 < 0 || (long long)step0 + opts->iters >= (long long)trace_rows) return GS2D_EINVAL;
    gs2d_ctx local;  // without a context the call's graphs live until it returns
    gs2d_ctx *cx = ctx ? ctx : &local;
    if (upload_tables(B, ws, st) != hipSuccess) return GS2D_EHIP;
    const int grid = batch_grid(B);
    if (grid < 1) return GS2D_EHIP;
    if (launch_fill_zero_u32(at<uint32_t>(ws, B.misc), (size_t)BM_STRIDE * B.F, st) != hipSuccess ||
        launch_fill_zero_u32(at<uint32_t>(ws, B.counter), 16, st) != hipSuccess ||
        launch_fill_zero(at<float>(ws, B.grads), 8 * (size_t)B.Ntot, st) != hipSuccess)
      return GS2D_EHIP;
    const int F = B.F;
    std::vector<float> rows((size_t)opts->check_every * F);
    std::vector<int> misc_host((size_t)BM_STRIDE * F);
    int done = 0, hit = -1;
    double last_mean = NAN;
    uint32_t sticky = 0;
    while (done < opts->iters) {
      const int k = std::min(opts->check_every, opts->iters - done);
      auto enqueue = [&](hipStream_t s) {
        hipError_t ce = hipSuccess;
        for (int i = 0; i < k && ce == hipSuccess; ++i)
          ce = enqueue_batch_iteration(B, ws, grid, targets, xy, chol, rgb, m, v, step,
                                       loss_trace, trace_rows, opts->adam, s, opts->bin_skin,
                                       opts->batch_persistent != 0);
        return ce;
      };
      if (opts->use_graph) {
        GraphKey key{2, (uint64_t)F, (uint64_t)B.T, (uint64_t)B.ppl, (uint64_t)grid,
                     key_word(targets), key_word(xy), key_word(chol), key_word(rgb),
                     key_word(m), key_word(v), key_word(step), key_word(loss_trace),
                     (uint64_t)trace_rows, key_word(ws), (uint64_t)k};
        for (int f = 0; f < F; ++f)
          key.push_back(((uint64_t)frames[f].W << 40) ^ ((uint64_t)frames[f].H << 20) ^
                        (uint64_t)frames[f].N);
        for (float x : opts->adam.lr) key.push_back(key_word(x));
        key.push_back(key_word(opts->adam.beta1));
        key.push_back(key_word(opts->adam.beta2));
        key.push_back(key_word(opts->adam.eps));
        key.push_back(key_word(opts->bin_skin));
        key.push_back((uint64_t)(opts->batch_persistent != 0));
        hipGraphExec_t x = nullptr;
        if (cx->graph_for(key, enqueue, &x) != hipSuccess || hipGraphLaunch(x, st) != hipSuccess)
          return GS2D_EHIP;
      } else if (enqueue(st) != hipSuccess) {
        return GS2D_EHIP;
      }
      if (hipMemcpyAsync(rows.data(), loss_trace + (size_t)(step0 + done) * F,
                         sizeof(float) * (size_t)k * F, hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipMemcpyAsync(misc_host.data(), at<int>(ws, B.misc), sizeof(int) * misc_host.size(),
                         hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return GS2D_EHIP;
      sticky = 0;
      for (int f = 0; f < F; ++f) sticky |= (uint32_t)misc_host[(size_t)BM_STRIDE * f + BM_STICKY];
      for (int i = 0; i < k; ++i) {
        double worst = INFINITY, mean = 0.0;
        for (int f = 0; f < F; ++f) {
          const double l = rows[(size_t)i * F + f];
          mean += l / F;
          worst = std::min(worst, l > 0 ? 10.0 * std::log10(1.0 / l) : INFINITY);
        }
        last_mean = mean;
        if (hit < 0 && opts->psnr_target > 0.f && worst >= opts->psnr_target) hit = done + i;
      }
      done += k;
      if ((sticky & STATUS_OVERFLOW) || hit >= 0) break;
    }
    if (stats) {
      int culled = 0, rebins = 0;
      for (int f = 0; f < F; ++f) {
        culled += misc_host[(size_t)BM_STRIDE * f + BM_N_CULLED];
        rebins += misc_host[(size_t)BM_STRIDE * f + BM_REBINS];
      }
      stats->rebins = rebins;
      stats->iters_run = done;
      stats->iter_hit_target = hit;
      stats->final_loss = (float)last_mean;
      stats->final_psnr = last_mean > 0 ? (float)(10.0 * std::log10(1.0 / last_mean)) : INFINITY;
      stats->status = sticky;
      stats->n_culled = culled;
      stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return (sticky & STATUS_OVERFLOW) ? GS2D_EOVERFLOW : GS2D_OK;
  } catch (...) {
    return GS2D_EHIP;
  }
}

// Binning + raster (one workgroup per item) of a batch (no optimiser step), for
// inspection and timing: builds every frame's tile lists and accumulates the
// gradients of the summed per-frame MSE into g_* (not cleared).
extern "C" int gs2d_batch_render_grads(int32_t n_frames, const gs2d_frame *frames, int32_t tile,
                                       int32_t px_per_lane, const float *targets, const float *xy,
                                       const float *chol, const float *rgb, float *g_xy,
                                       float *g_chol, float *g_rgb, float *loss_per_frame,
                                       void *ws, size_t ws_bytes, void *stream) {
  try {
    BatchLayout B;
    int rc = check_batch_ws(n_frames, frames, tile, px_per_lane, ws, ws_bytes, &B);
    if (rc != GS2D_OK) return rc;
    if (!targets || !xy || !chol || !rgb || !g_xy || !g_chol || !g_rgb) return GS2D_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (upload_tables(B, ws, st) != hipSuccess) return GS2D_EHIP;
    const int grid = batch_grid(B);
    if (grid < 1) return GS2D_EHIP;
    hipError_t e = launch_fill_zero_u32(at<uint32_t>(ws, B.misc), (size_t)BM_STRIDE * B.F, st);
    if (e == hipSuccess) e = launch_fill_zero_u32(at<uint32_t>(ws, B.counter), 16, st);
    if (e == hipSuccess)
      e = enqueue_batch_binning(B, ws, xy, chol, nullptr, st);
    if (e == hipSuccess)
      e = enqueue_batch_raster(B, ws, grid, rgb, targets, g_xy, g_chol, g_rgb, st);
    if (e == hipSuccess && loss_per_frame) {
      // a step counter of 1 makes k_b_loss write row 0 = loss_per_frame
      int32_t *one = at<int32_t>(ws, B.counter) + 8;
      const int32_t h_one = 1;
      e = hipMemcpyAsync(one, &h_one, sizeof(int32_t), hipMemcpyHostToDevice, st);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_b_loss, dim3(B.F), dim3(256), 0, st, at<const BFrame>(ws, B.desc), B.F,
                           B.nw, at<const float>(ws, B.loss_part), one, loss_per_frame, 1,
                           nullptr);
        e = hipGetLastError();
      }
      if (e == hipSuccess) e = hipStreamSynchronize(st);  // h_one leaves scope
    }
    return e == hipSuccess ? GS2D_OK : GS2D_EHIP;
  } catch (...) {
    return GS2D_EHIP;
  }
}

// Device views of frame f's binning results inside a batch workspace (after
// gs2d_batch_render_grads or gs2d_fit_batch), in the one-frame format.
extern "C" int gs2d_batch_bins_view(int32_t n_frames, const gs2d_frame *frames, int32_t tile,
                                    int32_t px_per_lane, int32_t f, void *ws, size_t ws_bytes,
                                    gs2d_bins *out) {
  try {
    BatchLayout B;
    int rc = check_batch_ws(n_frames, frames, tile, px_per_lane, ws, ws_bytes, &B);
    if (rc != GS2D_OK) return rc;
    if (!out || f < 0 || f >= n_frames) return GS2D_EINVAL;
    const BFrame &d = B.frames[f];
    int *misc = at<int>(ws, B.misc) + BM_STRIDE * f;
    out->geom = at<const float>(ws, B.geom) + 8 * d.g_off;
    out->counts = at<const int32_t>(ws, B.counts) + d.g_off;
    out->offsets = at<const int32_t>(ws, B.offsets) + d.g_off + f;
    out->keys = batch_sorted_keys(B, ws) + d.key_off;
    out->tile_start = at<const int32_t>(ws, B.tile_start) + d.tile_off + f;
    out->n_pairs = misc + BM_N_PAIRS;
    out->status = reinterpret_cast<const uint32_t *>(misc + BM_STATUS);
    out->n_culled = misc + BM_N_CULLED;
    out->n_tiles = d.n_tiles;
    out->tiles_x = d.TX;
    out->tiles_y = d.TY;
    return GS2D_OK;
  } catch (...) {
    return GS2D_EHIP;
  }
}

// Autotuner: times `reps` rounds of (batched binning + fused raster, one
// workgroup per item) for each candidate (tile, px_per_lane) with HIP events and
// returns the mean milliseconds per round in out_ms[i] and the fastest
// candidate's index in *best.  ws must hold gs2d_batch_workspace_bytes for
// every candidate; grad_scratch must hold 8 * sum(N) floats.
extern "C" int gs2d_autotune_batch(int32_t n_frames, const gs2d_frame *frames,
                                   const float *targets, const float *xy, const float *chol,
                                   const float *rgb, int32_t n_cand, const int32_t *cand_tile,
                                   const int32_t *cand_ppl, int32_t reps, float *grad_scratch,
                                   void *ws, size_t ws_bytes, float *out_ms, int32_t *best,
                                   void *stream) {
  try {
    if (n_cand < 1 || !cand_tile || !cand_ppl || reps < 1 || !out_ms || !best || !grad_scratch)
      return GS2D_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    Events O;
    if (hipEventCreate(&O.e0) != hipSuccess || hipEventCreate(&O.e1) != hipSuccess)
      return GS2D_EHIP;
    float best_ms = INFINITY;
    *best = -1;
    for (int c = 0; c < n_cand; ++c) {
      BatchLayout B;
      int rc = check_batch_ws(n_frames, frames, cand_tile[c], cand_ppl[c], ws, ws_bytes, &B);
      if (rc != GS2D_OK) return rc;
      if (upload_tables(B, ws, st) != hipSuccess) return GS2D_EHIP;
      const int grid = batch_grid(B);
      if (grid < 1) return GS2D_EHIP;
      float *g_xy = grad_scratch, *g_chol = g_xy + 2 * B.Ntot, *g_rgb = g_xy + 5 * B.Ntot;
      hipError_t e = launch_fill_zero_u32(at<uint32_t>(ws, B.misc), (size_t)BM_STRIDE * B.F, st);
      if (e == hipSuccess) e = launch_fill_zero_u32(at<uint32_t>(ws, B.counter), 16, st);
      // one untimed round, then the timed ones
      for (int r = 0; r <= reps && e == hipSuccess; ++r) {
        if (r == 1) e = hipEventRecord(O.e0, st);
        if (e == hipSuccess) e = enqueue_batch_binning(B, ws, xy, chol, nullptr, st);
        if (e == hipSuccess)
          e = enqueue_batch_raster(B, ws, grid, rgb, targets, g_xy, g_chol, g_rgb, st);
      }
      if (e == hipSuccess) e = hipEventRecord(O.e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(O.e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, O.e0, O.e1);
      if (e != hipSuccess) return GS2D_EHIP;
      out_ms[c] = ms / reps;
      if (out_ms[c] < best_ms) {
        best_ms = out_ms[c];
        *best = c;
      }
    }
    return GS2D_OK;
  } catch (...) {
    return GS2D_EHIP;
  }
}
