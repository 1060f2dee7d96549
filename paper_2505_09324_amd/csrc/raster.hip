// Tile rasteriser for Eq. 2 (accumulated summation, Sec. 3.1) and its
// backward pass.
//
// One workgroup per TILE x TILE screen tile; each wavefront owns an 8 x 8
// pixel sub-block (one pixel per lane).  The tile's Gaussian list is staged
// through LDS in chunks; while staging, each Gaussian's 3-sigma box is tested
// against every sub-block, and each wavefront compacts the chunk into its own
// list of Gaussians that can reach its pixels.  Per (pixel, Gaussian):
//
//   d = (x+1/2, y+1/2) - mu;  u1 = d1 / l1;  u2 = (d2 - l2 u1) / l3   (u = L^-1 d)
//   q = u1^2 + u2^2;  w = exp(-q/2) if q <= 9 else 0;  C += c' w
//
// Backward: with g = dL/dC at the pixel, s = (g . c') w, v = L^-T u,
//   dL/dmu += s v;  dL/dl1 += s v1 u1;  dL/dl2 += s v2 u1;  dL/dl3 += s v2 u2;
//   dL/dc' += g w.
// The eight per-lane terms of one Gaussian are summed across the wavefront
// by a transposing butterfly (each exchange halves the values a lane
// carries), added into an LDS accumulator shared by the tile's wavefronts,
// and flushed with one global atomic per (tile, Gaussian, parameter).
#include "gs2d_internal.h"

namespace gs2d {

namespace {

constexpr float NEG_HALF_LOG2E = -0.72134752044448170368f;  // -log2(e)/2
constexpr float CUTOFF_Q = 9.0f;

template <int TILE>
struct Cfg {
  static constexpr int NT = TILE * TILE;    // threads per tile
  static constexpr int NW = NT / 64;        // wavefronts per tile
  static constexpr int SBX = TILE / 8;      // 8x8 sub-blocks per tile row
  static constexpr int CH = NT < 256 ? NT : 256;  // Gaussians per LDS chunk
};

template <int TILE>
struct Smem {
  float4 A[Cfg<TILE>::CH];           // mx, my, 1/l1, l2
  float4 B[Cfg<TILE>::CH];           // 1/l3, c'0, c'1, c'2
  uint32_t mask[Cfg<TILE>::CH];      // bit w: box meets sub-block w
  int id[Cfg<TILE>::CH];
  uint16_t list[Cfg<TILE>::NW][Cfg<TILE>::CH];
  float red[Cfg<TILE>::NW];
};

// Stage keys[beg, beg+cnt) into LDS with their sub-block masks.
template <int TILE>
__device__ inline void stage_chunk(Smem<TILE> &S, const uint32_t *__restrict__ keys, int beg, int cnt,
                                   int tx, int ty, const float4 *__restrict__ geom,
                                   const float *__restrict__ rgb) {
  constexpr int SBX = Cfg<TILE>::SBX;
  const int j = threadIdx.x;
  if (j < cnt) {
    const int id = (int)(keys[beg + j] & 0xFFFFu);
    const float4 g0 = geom[2 * id], g1 = geom[2 * id + 1];
    float c0 = 0.f, c1 = 0.f, c2 = 0.f;
    if (rgb) {  // pair counting stages geometry only
      c0 = rgb[3 * id];
      c1 = rgb[3 * id + 1];
      c2 = rgb[3 * id + 2];
    }
    S.A[j] = g0;
    S.B[j] = make_float4(g1.x, c0, c1, c2);
    S.id[j] = id;
    const float xlo = __fsub_rn(g0.x, g1.y), xhi = __fadd_rn(g0.x, g1.y);
    const float ylo = __fsub_rn(g0.y, g1.z), yhi = __fadd_rn(g0.y, g1.z);
    // sub-block columns/rows (8 px each) met by the box, tile-local
    const float bx0f = floorf(xlo * 0.125f) - (float)(tx * SBX);
    const float bx1f = floorf(xhi * 0.125f) - (float)(tx * SBX);
    const float by0f = floorf(ylo * 0.125f) - (float)(ty * SBX);
    const float by1f = floorf(yhi * 0.125f) - (float)(ty * SBX);
    const int bx0 = (int)fmaxf(bx0f, 0.f), bx1 = (int)fminf(bx1f, (float)(SBX - 1));
    const int by0 = (int)fmaxf(by0f, 0.f), by1 = (int)fminf(by1f, (float)(SBX - 1));
    uint32_t m = 0;
    for (int by = by0; by <= by1; ++by)
      for (int bx = bx0; bx <= bx1; ++bx) m |= 1u << (by * SBX + bx);
    S.mask[j] = m;
  }
}

// Each wavefront builds its list of staged Gaussians; returns its length.
template <int TILE>
__device__ inline int compact_chunk(Smem<TILE> &S, int cnt) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const unsigned long long lt = lanemask_lt();
  int len = 0;
  for (int j0 = 0; j0 < cnt; j0 += 64) {
    const int j = j0 + lane;
    const bool hit = (j < cnt) && ((S.mask[j] >> w) & 1u);
    const unsigned long long bal = __ballot(hit);
    if (hit) S.list[w][len + __popcll(bal & lt)] = (uint16_t)j;
    len += __popcll(bal);
  }
  return len;
}

// Sum of 8 per-lane values over the wavefront; lane L returns the total of
// value ((L >> 3) & 7).  Each exchange step halves the number of values a
// lane carries, so the 64-lane sum of 8 values costs 4+2+1 exchanges and
// 3 in-row steps:
//   - across the two 32-lane halves: v_permlane32_swap of (value i, value
//     i+4) leaves value i of both halves in the low half and value i+4 in the
//     high half, one add finishes the pair;
//   - across 16-lane rows: v_permlane16_swap, the same way;
//   - across 8 lanes inside a row, then within each 8-lane group: DPP
//     (row_ror:8, row_half_mirror, quad_perm) folded into the adds.
template <int CTRL>
__device__ inline float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

__device__ inline void swap32(float x, float y, float &lo_sum_part, float &hi_sum_part) {
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  lo_sum_part = __uint_as_float(r[0]);
  hi_sum_part = __uint_as_float(r[1]);
}

__device__ inline void swap16(float x, float y, float &a, float &b) {
  auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  a = __uint_as_float(r[0]);
  b = __uint_as_float(r[1]);
}

constexpr int DPP_ROW_ROR8 = 0x128;
constexpr int DPP_ROW_HALF_MIRROR = 0x141;
constexpr int DPP_QUAD_XOR2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int DPP_QUAD_XOR1 = 0xB1;  // quad_perm [1,0,3,2]

__device__ inline float reduce8_transpose(const float (&a)[8]) {
  const int lane = threadIdx.x & 63;
  float b[4], c[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float p, q;
    swap32(a[i], a[i + 4], p, q);
    b[i] = p + q;
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    float p, q;
    swap16(b[i], b[i + 2], p, q);
    c[i] = p + q;
  }
  const bool hi = lane & 8;
  float d = (hi ? c[1] : c[0]) + dpp<DPP_ROW_ROR8>(hi ? c[0] : c[1]);
  d += dpp<DPP_ROW_HALF_MIRROR>(d);
  d += dpp<DPP_QUAD_XOR2>(d);
  d += dpp<DPP_QUAD_XOR1>(d);
  return d;
}

template <int TILE>
__device__ inline void pixel_of_thread(int tx, int ty, int *px, int *py) {
  constexpr int SBX = Cfg<TILE>::SBX;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  *px = tx * TILE + (w % SBX) * 8 + (lane & 7);
  *py = ty * TILE + (w / SBX) * 8 + (lane >> 3);
}

// Forward accumulation over one staged, compacted chunk.  With KEEP_HITS the
// wavefront's list is compacted in place to the Gaussians that have at least
// one in-frame pixel with q <= 9 in this sub-block (the only ones the
// backward pass needs); returns the new length (else `len`).
template <int TILE, bool KEEP_HITS>
__device__ inline int fwd_chunk(Smem<TILE> &S, int len, float pxc, float pyc, bool inside,
                                float &a0, float &a1, float &a2) {
  const int w = threadIdx.x >> 6;
  int kept = 0;
  for (int k = 0; k < len; ++k) {
    const int j = S.list[w][k];
    const float4 A = S.A[j], B = S.B[j];
    const float dx = pxc - A.x, dy = pyc - A.y;
    const float u1 = dx * A.z;
    const float u2 = (dy - A.w * u1) * B.x;
    const float q = u1 * u1 + u2 * u2;
    const float e = __builtin_amdgcn_exp2f(q * NEG_HALF_LOG2E);
    const bool in_cut = q <= CUTOFF_Q;
    const float wgt = in_cut ? e : 0.f;
    a0 += wgt * B.y;
    a1 += wgt * B.z;
    a2 += wgt * B.w;
    if (KEEP_HITS) {
      if (__ballot(in_cut && inside)) {
        if ((threadIdx.x & 63) == 0) S.list[w][kept] = (uint16_t)j;  // kept <= k
        ++kept;
      }
    }
  }
  return KEEP_HITS ? kept : len;
}

// Backward over one staged, compacted chunk; adds into acc[CH][8] in LDS.
// CHECK_HITS skips (uniformly per wavefront) Gaussians with no lane inside
// the cutoff, for lists that were not already reduced to such Gaussians.
template <int TILE, bool CHECK_HITS>
__device__ inline void bwd_chunk(const Smem<TILE> &S, float *acc, int len, float pxc, float pyc,
                                 float g0, float g1, float g2) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int k = 0; k < len; ++k) {
    const int j = S.list[w][k];
    const float4 A = S.A[j], B = S.B[j];
    const float dx = pxc - A.x, dy = pyc - A.y;
    const float u1 = dx * A.z;
    const float u2 = (dy - A.w * u1) * B.x;
    const float q = u1 * u1 + u2 * u2;
    if (CHECK_HITS && !__ballot(q <= CUTOFF_Q)) continue;  // wave-uniform skip
    const float e = __builtin_amdgcn_exp2f(q * NEG_HALF_LOG2E);
    const float wgt = (q <= CUTOFF_Q) ? e : 0.f;
    const float sn = (g0 * B.y + g1 * B.z + g2 * B.w) * wgt;
    const float v2 = u2 * B.x;
    const float v1 = (u1 - A.w * v2) * A.z;
    const float t1 = sn * v1, t2 = sn * v2;
    const float vals[8] = {t1, t2, t1 * u1, t2 * u1, t2 * u2, g0 * wgt, g1 * wgt, g2 * wgt};
    const float r = reduce8_transpose(vals);
    if ((lane & 7) == 0) atomicAdd(&acc[j * 8 + (lane >> 3)], r);
  }
}

// Flush the LDS accumulators of a chunk to the global gradients.
template <int TILE>
__device__ inline void flush_grads(const Smem<TILE> &S, const float *acc, int cnt,
                                   float *__restrict__ g_xy, float *__restrict__ g_chol,
                                   float *__restrict__ g_rgb) {
  const int j = threadIdx.x;
  if (j < cnt) {
    const int id = S.id[j];
    const float *a = acc + j * 8;
    if (a[0] != 0.f) atomicAdd(&g_xy[2 * id + 0], a[0]);
    if (a[1] != 0.f) atomicAdd(&g_xy[2 * id + 1], a[1]);
    if (a[2] != 0.f) atomicAdd(&g_chol[3 * id + 0], a[2]);
    if (a[3] != 0.f) atomicAdd(&g_chol[3 * id + 1], a[3]);
    if (a[4] != 0.f) atomicAdd(&g_chol[3 * id + 2], a[4]);
    if (a[5] != 0.f) atomicAdd(&g_rgb[3 * id + 0], a[5]);
    if (a[6] != 0.f) atomicAdd(&g_rgb[3 * id + 1], a[6]);
    if (a[7] != 0.f) atomicAdd(&g_rgb[3 * id + 2], a[7]);
  }
}

template <int TILE>
__device__ inline float block_sum(Smem<TILE> &S, float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) S.red[threadIdx.x >> 6] = v;
  __syncthreads();
  float s = 0.f;
  if (threadIdx.x == 0)
    for (int w = 0; w < Cfg<TILE>::NW; ++w) s += S.red[w];
  return s;
}

struct FrameArgs {
  int W, H, TX;
  const float4 *geom;
  const uint32_t *keys;
  const int *tile_start;
  const float *rgb;
};

}  // namespace

// ----------------------------------------------------------------- forward --
template <int TILE>
__global__ void __launch_bounds__(TILE *TILE)
k_render_fwd(FrameArgs f, const float *__restrict__ target, float *__restrict__ img,
             float *__restrict__ dl_dimg, float *__restrict__ loss_part, float grad_scale) {
  constexpr int CH = Cfg<TILE>::CH;
  __shared__ Smem<TILE> S;
  const int tile = blockIdx.x;
  const int tx = tile % f.TX, ty = tile / f.TX;
  const int beg = f.tile_start[tile], end = f.tile_start[tile + 1];
  int px, py;
  pixel_of_thread<TILE>(tx, ty, &px, &py);
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f;
  for (int c = beg; c < end; c += CH) {
    const int cnt = min(CH, end - c);
    __syncthreads();
    stage_chunk<TILE>(S, f.keys, c, cnt, tx, ty, f.geom, f.rgb);
    __syncthreads();
    const int len = compact_chunk<TILE>(S, cnt);
    __syncthreads();
    fwd_chunk<TILE, false>(S, len, pxc, pyc, true, a0, a1, a2);
  }
  const bool inside = px < f.W && py < f.H;
  float l = 0.f;
  if (inside) {
    const size_t HW = (size_t)f.W * f.H, p = (size_t)py * f.W + px;
    if (img) {
      img[p] = a0;
      img[HW + p] = a1;
      img[2 * HW + p] = a2;
    }
    if (target) {
      const float r0 = a0 - target[p], r1 = a1 - target[HW + p], r2 = a2 - target[2 * HW + p];
      l = r0 * r0 + r1 * r1 + r2 * r2;
      if (dl_dimg) {
        dl_dimg[p] = r0 * grad_scale;
        dl_dimg[HW + p] = r1 * grad_scale;
        dl_dimg[2 * HW + p] = r2 * grad_scale;
      }
    }
  }
  if (loss_part) {
    __syncthreads();
    const float s = block_sum<TILE>(S, l);
    if (threadIdx.x == 0) loss_part[tile] = s;
  }
}

// ---------------------------------------------------------------- backward --
template <int TILE>
__global__ void __launch_bounds__(TILE *TILE)
k_render_bwd(FrameArgs f, const float *__restrict__ dl_dimg, float *__restrict__ g_xy,
             float *__restrict__ g_chol, float *__restrict__ g_rgb) {
  constexpr int CH = Cfg<TILE>::CH;
  __shared__ Smem<TILE> S;
  __shared__ float acc[CH * 8];
  const int tile = blockIdx.x;
  const int tx = tile % f.TX, ty = tile / f.TX;
  const int beg = f.tile_start[tile], end = f.tile_start[tile + 1];
  if (beg >= end) return;
  int px, py;
  pixel_of_thread<TILE>(tx, ty, &px, &py);
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  float g0 = 0.f, g1 = 0.f, g2 = 0.f;
  if (px < f.W && py < f.H) {
    const size_t HW = (size_t)f.W * f.H, p = (size_t)py * f.W + px;
    g0 = dl_dimg[p];
    g1 = dl_dimg[HW + p];
    g2 = dl_dimg[2 * HW + p];
  }
  for (int c = beg; c < end; c += CH) {
    const int cnt = min(CH, end - c);
    __syncthreads();
    stage_chunk<TILE>(S, f.keys, c, cnt, tx, ty, f.geom, f.rgb);
    for (int i = threadIdx.x; i < CH * 8; i += blockDim.x) acc[i] = 0.f;
    __syncthreads();
    const int len = compact_chunk<TILE>(S, cnt);
    __syncthreads();
    bwd_chunk<TILE, true>(S, acc, len, pxc, pyc, g0, g1, g2);
    __syncthreads();
    flush_grads<TILE>(S, acc, cnt, g_xy, g_chol, g_rgb);
  }
}

// ------------------------------------------- fused forward + loss + backward --
// Eq. 2 is an order-free sum and every Gaussian reaching a pixel is in that
// pixel's tile list, so a tile can finish its forward pass, form
// dL/dC = 2 (C - target) / (3HW) in registers and run its backward pass
// without dL/dC ever reaching memory.
template <int TILE>
__global__ void __launch_bounds__(TILE *TILE)
k_render_fused(FrameArgs f, const float *__restrict__ target, float *__restrict__ loss_part,
               float grad_scale, float *__restrict__ g_xy, float *__restrict__ g_chol,
               float *__restrict__ g_rgb) {
  constexpr int CH = Cfg<TILE>::CH;
  __shared__ Smem<TILE> S;
  __shared__ float acc[CH * 8];
  const int tile = blockIdx.x;
  const int tx = tile % f.TX, ty = tile / f.TX;
  const int beg = f.tile_start[tile], end = f.tile_start[tile + 1];
  int px, py;
  pixel_of_thread<TILE>(tx, ty, &px, &py);
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const bool inside = px < f.W && py < f.H;
  const bool single = (end - beg) <= CH;  // the whole list fits one LDS chunk
  float a0 = 0.f, a1 = 0.f, a2 = 0.f;
  int len = 0;
  for (int c = beg; c < end; c += CH) {
    const int cnt = min(CH, end - c);
    __syncthreads();
    stage_chunk<TILE>(S, f.keys, c, cnt, tx, ty, f.geom, f.rgb);
    __syncthreads();
    len = compact_chunk<TILE>(S, cnt);
    __syncthreads();
    // a single chunk stays in LDS for the backward pass: keep only the
    // Gaussians that reach this wavefront's pixels
    if (single)
      len = fwd_chunk<TILE, true>(S, len, pxc, pyc, inside, a0, a1, a2);
    else
      fwd_chunk<TILE, false>(S, len, pxc, pyc, inside, a0, a1, a2);
  }
  float g0 = 0.f, g1 = 0.f, g2 = 0.f, l = 0.f;
  if (inside) {
    const size_t HW = (size_t)f.W * f.H, p = (size_t)py * f.W + px;
    const float r0 = a0 - target[p], r1 = a1 - target[HW + p], r2 = a2 - target[2 * HW + p];
    l = r0 * r0 + r1 * r1 + r2 * r2;
    g0 = r0 * grad_scale;
    g1 = r1 * grad_scale;
    g2 = r2 * grad_scale;
  }
  __syncthreads();
  const float s = block_sum<TILE>(S, l);
  if (threadIdx.x == 0) loss_part[tile] = s;
  if (beg >= end) return;
  for (int c = beg; c < end; c += CH) {
    const int cnt = min(CH, end - c);
    __syncthreads();
    if (!single) stage_chunk<TILE>(S, f.keys, c, cnt, tx, ty, f.geom, f.rgb);
    for (int i = threadIdx.x; i < CH * 8; i += blockDim.x) acc[i] = 0.f;
    __syncthreads();
    if (!single) {
      len = compact_chunk<TILE>(S, cnt);
      __syncthreads();
      bwd_chunk<TILE, true>(S, acc, len, pxc, pyc, g0, g1, g2);
    } else {
      bwd_chunk<TILE, false>(S, acc, len, pxc, pyc, g0, g1, g2);
    }
    __syncthreads();
    flush_grads<TILE>(S, acc, cnt, g_xy, g_chol, g_rgb);
  }
}

// ------------------------------------------------- in-cutoff pair counting --
// Number of (pixel, Gaussian) pairs with q <= 9 inside the frame: the terms
// Eq. 2 actually sums (the algorithmic work of one render).
template <int TILE>
__global__ void __launch_bounds__(TILE *TILE)
k_count_pairs(FrameArgs f, unsigned long long *__restrict__ out) {
  constexpr int CH = Cfg<TILE>::CH;
  __shared__ Smem<TILE> S;
  const int tile = blockIdx.x;
  const int tx = tile % f.TX, ty = tile / f.TX;
  const int beg = f.tile_start[tile], end = f.tile_start[tile + 1];
  int px, py;
  pixel_of_thread<TILE>(tx, ty, &px, &py);
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const bool inside = px < f.W && py < f.H;
  const int w = threadIdx.x >> 6;
  unsigned int n = 0;
  for (int c = beg; c < end; c += CH) {
    const int cnt = min(CH, end - c);
    __syncthreads();
    stage_chunk<TILE>(S, f.keys, c, cnt, tx, ty, f.geom, f.rgb);
    __syncthreads();
    const int len = compact_chunk<TILE>(S, cnt);
    __syncthreads();
    for (int k = 0; k < len; ++k) {
      const int j = S.list[w][k];
      const float4 A = S.A[j], B = S.B[j];
      const float dx = pxc - A.x, dy = pyc - A.y;
      const float u1 = dx * A.z;
      const float u2 = (dy - A.w * u1) * B.x;
      n += (inside && u1 * u1 + u2 * u2 <= CUTOFF_Q) ? 1u : 0u;
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
  for (int i = threadIdx.x; i < n; i += 1024) s += (double)part[i];
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
  return f;
}

static float grad_scale(const Layout &L) { return (float)(2.0 / (3.0 * L.W * (double)L.H)); }

#define GS2D_TILE_SWITCH(T, CALL) \
  switch (T) {                    \
    case 8: CALL(8); break;       \
    case 16: CALL(16); break;     \
    case 32: CALL(32); break;     \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_render_fwd(const Layout &L, void *ws, const float *rgb, const float *target,
                             float *img, float *dl_dimg, hipStream_t st) {
  FrameArgs f = frame_args(L, ws, rgb);
  float *lp = target ? at<float>(ws, L.loss_part) : nullptr;
#define CALL(TT)                                                                              \
  hipLaunchKernelGGL(k_render_fwd<TT>, dim3(L.n_tiles), dim3(TT * TT), 0, st, f, target, img, \
                     dl_dimg, lp, grad_scale(L))
  GS2D_TILE_SWITCH(L.T, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_render_bwd(const Layout &L, void *ws, const float *rgb, const float *dl_dimg,
                             float *g_xy, float *g_chol, float *g_rgb, hipStream_t st) {
  FrameArgs f = frame_args(L, ws, rgb);
#define CALL(TT)                                                                               \
  hipLaunchKernelGGL(k_render_bwd<TT>, dim3(L.n_tiles), dim3(TT * TT), 0, st, f, dl_dimg, g_xy, \
                     g_chol, g_rgb)
  GS2D_TILE_SWITCH(L.T, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_render_fused(const Layout &L, void *ws, const float *rgb, const float *target,
                               float *g_xy, float *g_chol, float *g_rgb, hipStream_t st) {
  FrameArgs f = frame_args(L, ws, rgb);
  float *lp = at<float>(ws, L.loss_part);
#define CALL(TT)                                                                                \
  hipLaunchKernelGGL(k_render_fused<TT>, dim3(L.n_tiles), dim3(TT * TT), 0, st, f, target, lp, \
                     grad_scale(L), g_xy, g_chol, g_rgb)
  GS2D_TILE_SWITCH(L.T, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_count_pairs(const Layout &L, void *ws, unsigned long long *out, hipStream_t st) {
  FrameArgs f = frame_args(L, ws, nullptr);
  hipError_t e = launch_fill_zero_u32(reinterpret_cast<uint32_t *>(out), 2, st);
  if (e != hipSuccess) return e;
#define CALL(TT) \
  hipLaunchKernelGGL(k_count_pairs<TT>, dim3(L.n_tiles), dim3(TT * TT), 0, st, f, out)
  GS2D_TILE_SWITCH(L.T, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_loss_reduce(const Layout &L, void *ws, float *loss, hipStream_t st) {
  hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(1024), 0, st, at<const float>(ws, L.loss_part),
                     L.n_tiles, (float)(1.0 / (3.0 * L.W * (double)L.H)), loss);
  return hipGetLastError();
}

}  // namespace gs2d
