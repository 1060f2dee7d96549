// Device-side building blocks of the tile rasteriser for Eq. 2 and its
// backward pass, shared by the one-frame kernels (raster.hip) and the
// persistent batched kernel (batch.hip).  See raster.hip for the scheme.
#pragma once

#include "gs2d_internal.h"

namespace gs2d {

// exp(-q/2) = exp2(-q h) with h = log2(e)/2.  Staging multiplies 1/l1 and
// 1/l3 by sqrt(h) and divides l2 by it, so the per-pixel quantities are
// u' = sqrt(h) u and q' = h q: the exponent needs no multiply and the cutoff
// q <= 9 becomes q' <= 9 h.  Gradients summed in these units are rescaled
// by 1/h (mean) and 1/h^1.5 (Cholesky vector) when flushed.
constexpr float EXP_SCALE = 0.84932180028801904f;     // sqrt(log2(e)/2)
constexpr float CUTOFF_QS = 6.4921276840003355f;      // 9 log2(e)/2
constexpr float INV_H = 1.3862943611198906f;          // 2 / log2(e)
constexpr float INV_H15 = 1.6322368749392462f;        // (2 / log2(e))^1.5
constexpr int CH = 256;  // Gaussians staged per LDS chunk

// Raster kernels are compiled for 8 wavefronts per SIMD (at most 64 VGPRs
// where the LDS allows it): with 512-thread tiles that is 4 workgroups per
// CU, the wave-slot limit, which the latency of staging and the barriers
// between a tile's phases need.
#define GS2D_RASTER_OCCUPANCY __attribute__((amdgpu_waves_per_eu(8, 8)))

template <int TILE, int PPL>
struct Cfg {
  static constexpr int SBH = 8 * PPL;      // sub-block height (px)
  static constexpr int SBX = TILE / 8;     // sub-blocks per tile row
  static constexpr int SBY = TILE / SBH;   // sub-block rows per tile
  static constexpr int NW = SBX * SBY;     // wavefronts per tile
  static constexpr int NT = NW * 64;       // threads per tile
  static_assert(SBY >= 1 && NW <= 16, "unsupported tile / pixels-per-lane");
};

template <int NW>
struct Smem {
  float4 A[CH];           // mx, my, 1/l1, l2
  float4 B[CH];           // 1/l3, c'0, c'1, c'2
  uint16_t mask[CH];      // bit w: box meets sub-block w (at most 16)
  int id[CH];
  uint16_t list[NW][CH];
  uint8_t act[CH];        // the Gaussian is optimised (FrameArgs::active)
};

struct FrameArgs {
  int W, H, TX;
  const float4 *geom;
  const uint32_t *keys;
  const int *tile_start;
  const float *rgb;
  // nullable [N]: the fused backward skips Gaussians with active[n] == 0
  // (they are not optimised, Sec. 3.2.C); the forward renders them all
  const uint8_t *active;
  // nullable, lazy binning: the workspace's misc array.  The binning
  // kernels that read misc[MISC_STALE] have finished when the fused raster
  // runs; if the flag is set (this iteration rebuilt the lists) the raster
  // stamps the lists with (sig_lo, sig_hi), or clears the stamp if a
  // rebuild's wait ran out, then clears the flag.
  int *lazy_misc;
  uint32_t sig_lo, sig_hi;
  // nullable: the fused raster adds 1 to *tick (the optimiser's step)
  int *tick;
};

// Whether the ellipse q' <= qmax (staged units: u1 = dx a, u2 = (dy - l2s u1)
// r3s) reaches the rectangle [X0, X1] x [Y0, Y1].  q' is a convex quadratic,
// so outside its centre its minimum over the rectangle lies on an edge that
// faces the centre: on the edge x = Xe the minimum sits where u2 = 0 (dy =
// l2s u1), clamped to the edge; on the edge y = Ye, q' = (a dx)^2 +
// (e - c dx)^2 with c = l2s a r3s and e = dy r3s, minimised at dx = c e /
// (a^2 + c^2), clamped.  A NaN anywhere counts as a hit.
__device__ inline bool ellipse_meets_rect(float mx, float my, float a, float l2s, float r3s,
                                          float X0, float X1, float Y0, float Y1, float qmax) {
  const bool left = mx < X0, right = mx > X1, below = my < Y0, above = my > Y1;
  if (!(left || right || below || above)) return true;
  float best = INFINITY;
  if (left || right) {
    const float u1 = ((left ? X0 : X1) - mx) * a;
    const float t = l2s * u1;
    const float dy = fminf(fmaxf(t, Y0 - my), Y1 - my);
    const float u2 = (dy - t) * r3s;
    best = u1 * u1 + u2 * u2;
  }
  if (below || above) {
    const float dy = (below ? Y0 : Y1) - my;
    const float c = l2s * a * r3s, e = dy * r3s;
    // an approximate reciprocal only moves the evaluated point off the
    // minimiser, which raises q' by a second-order amount
    const float dx = fminf(fmaxf(c * e * __builtin_amdgcn_rcpf(a * a + c * c), X0 - mx), X1 - mx);
    const float u1 = dx * a;
    const float u2 = (dy - l2s * u1) * r3s;
    best = fminf(best, u1 * u1 + u2 * u2);
  }
  return !(best > qmax);
}

// Stage keys[beg, beg+cnt) into LDS with their sub-block masks: bit w is set
// when the Gaussian's 3-sigma box meets sub-block w and, with EXACT, its
// cutoff ellipse also comes within a rounding margin of one of the
// sub-block's in-frame pixel centres (on fitted frames about one box-met
// sub-block in six fails the ellipse test).  The margin, 0.01 (1 + |l2 /
// l3|) in staged q units, bounds the rounding of both this test and the
// per-pixel evaluation (each about 1e-5 (1 + |l2 / l3|)), so no sub-block
// with a pixel the raster counts inside the cutoff is dropped.  Exact masks
// leave few Gaussians without a pixel in the cutoff, so their users skip
// the per-Gaussian hit checks; the persistent batched kernel, whose
// register budget the test's live values overrun, keeps box masks.
template <int TILE, int PPL, bool EXACT = true>
__device__ inline void stage_chunk(Smem<Cfg<TILE, PPL>::NW> &S, const uint32_t *__restrict__ keys,
                                   int beg, int cnt, int tx, int ty, int W, int H,
                                   const float4 *__restrict__ geom, const float *__restrict__ rgb,
                                   const uint8_t *__restrict__ active = nullptr) {
  using C = Cfg<TILE, PPL>;
  constexpr float inv_w = 0.125f, inv_h = 1.0f / (float)C::SBH;
  const float xlast = (float)W - 0.5f, ylast = (float)H - 0.5f;  // last pixel centres
  for (int j = threadIdx.x; j < cnt; j += C::NT) {
    const int id = (int)(keys[beg + j] & 0xFFFFu);
    const float4 g0 = geom[2 * id], g1 = geom[2 * id + 1];
    float c0 = 0.f, c1 = 0.f, c2 = 0.f;
    if (rgb) {  // pair counting stages geometry only
      c0 = rgb[3 * id];
      c1 = rgb[3 * id + 1];
      c2 = rgb[3 * id + 2];
    }
    const float a = g0.z * EXP_SCALE, l2s = g0.w * (1.0f / EXP_SCALE), r3s = g1.x * EXP_SCALE;
    S.A[j] = make_float4(g0.x, g0.y, a, l2s);
    S.B[j] = make_float4(r3s, c0, c1, c2);
    S.id[j] = id;
    if (active) S.act[j] = active[id];
    const float xlo = __fsub_rn(g0.x, g1.y), xhi = __fadd_rn(g0.x, g1.y);
    const float ylo = __fsub_rn(g0.y, g1.z), yhi = __fadd_rn(g0.y, g1.z);
    // sub-block columns/rows met by the box, tile-local
    const float bx0f = floorf(xlo * inv_w) - (float)(tx * C::SBX);
    const float bx1f = floorf(xhi * inv_w) - (float)(tx * C::SBX);
    const float by0f = floorf(ylo * inv_h) - (float)(ty * C::SBY);
    const float by1f = floorf(yhi * inv_h) - (float)(ty * C::SBY);
    const int bx0 = (int)fmaxf(bx0f, 0.f), bx1 = (int)fminf(bx1f, (float)(C::SBX - 1));
    const int by0 = (int)fmaxf(by0f, 0.f), by1 = (int)fminf(by1f, (float)(C::SBY - 1));
    const float qmax = CUTOFF_QS + 0.01f * (1.0f + fabsf(l2s * r3s));
    uint32_t m = 0;
    for (int by = by0; by <= by1; ++by) {
      const float Y0 = (float)(ty * TILE + by * C::SBH) + 0.5f;
      const float Y1 = fminf(Y0 + (float)(C::SBH - 1), ylast);
      for (int bx = bx0; bx <= bx1; ++bx) {
        const float X0 = (float)(tx * TILE + bx * 8) + 0.5f;
        const float X1 = fminf(X0 + 7.0f, xlast);
        if (!EXACT ||
            (X0 <= X1 && Y0 <= Y1 && ellipse_meets_rect(g0.x, g0.y, a, l2s, r3s, X0, X1, Y0, Y1, qmax)))
          m |= 1u << (by * C::SBX + bx);
      }
    }
    S.mask[j] = (uint16_t)m;
  }
}

// Each wavefront builds its list of staged Gaussians; returns its length.
template <int NW>
__device__ inline int compact_chunk(Smem<NW> &S, int cnt) {
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

// ---- wavefront reduction of 8 values ----
// Sum of 8 per-lane values over the wavefront; lane L returns the total of
// value ((L >> 3) & 7).  Each exchange halves the number of values a lane
// carries:
//   - across the two 32-lane halves, v_permlane32_swap of (value i, value
//     i+4) leaves value i of both halves in the low half and value i+4 of
//     both halves in the high half; one add finishes the pair;
//   - across 16-lane rows, v_permlane16_swap, the same way;
//   - across 8 lanes inside a row and then within each 8-lane group, DPP
//     (row_ror:8, row_half_mirror, quad_perm) folded into the adds.
template <int CTRL>
__device__ inline float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
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
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a[i]), __float_as_uint(a[i + 4]),
                                              false, false);
    b[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(b[i]), __float_as_uint(b[i + 2]),
                                              false, false);
    c[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  const bool hi = lane & 8;
  float d = (hi ? c[1] : c[0]) + dpp<DPP_ROW_ROR8>(hi ? c[0] : c[1]);
  d += dpp<DPP_ROW_HALF_MIRROR>(d);
  d += dpp<DPP_QUAD_XOR2>(d);
  d += dpp<DPP_QUAD_XOR1>(d);
  return d;
}

// Drop the Gaussians whose staged active flag is 0 from this wavefront's
// list (in place, order kept); returns the new length.
template <int NW>
__device__ inline int keep_active(Smem<NW> &S, int len) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const unsigned long long lt = lanemask_lt();
  int kept = 0;
  for (int k0 = 0; k0 < len; k0 += 64) {
    const int j = (k0 + lane < len) ? S.list[w][k0 + lane] : 0;
    const bool keep = (k0 + lane < len) && S.act[j];
    const unsigned long long bal = __ballot(keep);
    if (keep) S.list[w][kept + __popcll(bal & lt)] = (uint16_t)j;
    kept += __popcll(bal);
  }
  return kept;
}

// Pixel column and first row of this thread.
template <int TILE, int PPL>
__device__ inline void pixel_of_thread(int tx, int ty, int *px, int *py0) {
  using C = Cfg<TILE, PPL>;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  *px = tx * TILE + (w % C::SBX) * 8 + (lane & 7);
  *py0 = ty * TILE + (w / C::SBX) * C::SBH + (lane >> 3) * PPL;
}

// Forward accumulation over one staged, compacted chunk.  With KEEP_HITS the
// wavefront's list is compacted in place to the Gaussians that have at least
// one in-frame pixel with q <= 9 in this sub-block (the only ones the
// backward pass needs); returns the new length (else `len`).
template <int NW, int PPL, bool KEEP_HITS>
__device__ inline int fwd_chunk(Smem<NW> &S, int len, float pxc, float pyc0, unsigned inside,
                                float (&acc)[PPL][3]) {
  const int w = threadIdx.x >> 6;
  int kept = 0;
  for (int k = 0; k < len; ++k) {
    const int j = S.list[w][k];
    const float4 A = S.A[j], B = S.B[j];
    const float u1 = (pxc - A.x) * A.z;
    const float u1s = u1 * u1;
    const float base = (pyc0 - A.y) - A.w * u1;
    bool any = false;
    float u2 = base * B.x;  // the next pixel row adds 1/l3 (staged units)
#pragma unroll
    for (int r = 0; r < PPL; ++r, u2 += B.x) {
      const float q = u1s + u2 * u2;
      const float e = __builtin_amdgcn_exp2f(-q);
      const bool in_cut = q <= CUTOFF_QS;
      const float wgt = in_cut ? e : 0.f;
      acc[r][0] += wgt * B.y;
      acc[r][1] += wgt * B.z;
      acc[r][2] += wgt * B.w;
      any |= in_cut && ((inside >> r) & 1u);
    }
    if (KEEP_HITS) {
      if (__ballot(any)) {
        if ((threadIdx.x & 63) == 0) S.list[w][kept] = (uint16_t)j;  // kept <= k
        ++kept;
      }
    }
  }
  return KEEP_HITS ? kept : len;
}

// Backward over one staged, compacted chunk; adds into acc[CH][8] in LDS.
// CHECK_HITS skips (uniformly per wavefront) Gaussians with no pixel inside
// the cutoff, for lists that were not already reduced to such Gaussians.
template <int NW, int PPL, bool CHECK_HITS>
__device__ inline void bwd_chunk(const Smem<NW> &S, float *acc, int len, float pxc, float pyc0,
                                 const float (&g)[PPL][3]) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int k = 0; k < len; ++k) {
    const int j = S.list[w][k];
    const float4 A = S.A[j], B = S.B[j];
    const float u1 = (pxc - A.x) * A.z;
    const float u1s = u1 * u1;
    const float base = (pyc0 - A.y) - A.w * u1;
    float u2[PPL], q[PPL];
    bool any = false;
#pragma unroll
    for (int r = 0; r < PPL; ++r) {
      u2[r] = r == 0 ? base * B.x : u2[r - 1] + B.x;  // the next pixel row adds 1/l3
      q[r] = u1s + u2[r] * u2[r];
      any |= q[r] <= CUTOFF_QS;
    }
    if (CHECK_HITS && !__ballot(any)) continue;  // wavefront-uniform skip
    float s0 = 0.f, s2 = 0.f, s3 = 0.f, c0 = 0.f, c1 = 0.f, c2 = 0.f;
#pragma unroll
    for (int r = 0; r < PPL; ++r) {
      const float e = __builtin_amdgcn_exp2f(-q[r]);
      const float wgt = (q[r] <= CUTOFF_QS) ? e : 0.f;
      const float sn = (g[r][0] * B.y + g[r][1] * B.z + g[r][2] * B.w) * wgt;
      const float v2 = u2[r] * B.x;
      const float t2 = sn * v2;
      s0 += sn;
      s2 += t2;
      s3 += t2 * u2[r];
      c0 += g[r][0] * wgt;
      c1 += g[r][1] * wgt;
      c2 += g[r][2] * wgt;
    }
    // v1 = (u1 - l2 v2) / l1 with u1 common to the lane's pixels, so
    // sum s v1 = (u1 sum s - l2 sum s v2) / l1; likewise dL/dl1 = sum s v1 u1
    // and dL/dl2 = sum s v2 u1 take the lane's u1 once.  In the staged units
    // (u' = sqrt(h) u, v2' = h v2) these sums come out as h dL/dmu and
    // h^1.5 dL/dl; flush_grads rescales them.
    const float s1 = (u1 * s0 - A.w * s2) * A.z;
    const float vals[8] = {s1, s2, s1 * u1, s2 * u1, s3, c0, c1, c2};
    const float red = reduce8_transpose(vals);
    if ((lane & 7) == 0) atomicAdd(&acc[j * 8 + (lane >> 3)], red);
  }
}

// Flush the LDS accumulators of a chunk to the global gradients: thread t
// adds parameter t % 8 of the chunk's Gaussians t / 8, t / 8 + NT / 8, ...,
// so the eight parameters of a Gaussian leave from adjacent lanes of one
// instruction and every wavefront of the tile takes a share.  PIN forms the
// lane's pointer, stride and scale at the flush rather than letting the
// compiler hoist them out of a caller's chunk loop, where they would hold
// registers through the passes (which of the two spills less depends on the
// caller).
template <int NT, int NW, bool PIN = false>
__device__ inline void flush_grads(const Smem<NW> &S, const float *acc, int cnt,
                                   float *__restrict__ g_xy, float *__restrict__ g_chol,
                                   float *__restrict__ g_rgb) {
  static_assert(NT % 8 == 0, "a thread keeps one parameter");
  int k = threadIdx.x & 7;
  if constexpr (PIN) asm volatile("" : "+v"(k));
  float *base;
  int stride;
  float scale;
  if (k < 2) {
    base = g_xy + k;
    stride = 2;
    scale = INV_H;
  } else if (k < 5) {
    base = g_chol + (k - 2);
    stride = 3;
    scale = INV_H15;
  } else {
    base = g_rgb + (k - 5);
    stride = 3;
    scale = 1.f;
  }
  for (int e = threadIdx.x; e < cnt * 8; e += NT) {
    const float v = acc[e];
    if (v != 0.f) atomicAdd(base + stride * S.id[e >> 3], v * scale);
  }
}

// Wavefront sum of one float per lane; lane 0 writes it to *slot.  Loss
// partials are kept per wavefront (tile t, wavefront w at t * NW + w), so a
// wavefront never waits for the rest of its tile to record its loss.
__device__ inline void wave_loss(float v, float *__restrict__ slot) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) *slot = v;
}

// Bit r set: pixel row r of this lane lies inside the frame.
template <int PPL>
__device__ inline unsigned inside_mask(const FrameArgs &f, int px, int py0) {
  unsigned m = 0;
#pragma unroll
  for (int r = 0; r < PPL; ++r) m |= (px < f.W && py0 + r < f.H) ? (1u << r) : 0u;
  return m;
}


// ------------------------------------------- fused forward + loss + backward --
// Eq. 2 is an order-free sum and every Gaussian reaching a pixel is in that
// pixel's tile list, so a tile can finish its forward pass, form
// dL/dC = 2 (C - target) / (3HW) in registers and run its backward pass
// without dL/dC ever reaching memory.  One call processes one tile with the
// whole workgroup; each wavefront's sum of squared residuals goes to
// loss_slots[w].
//
// A list that fits one LDS chunk (the common case) is staged once; after
// one barrier every wavefront compacts it to its sub-block, runs its
// forward pass (with box masks also keeping only the Gaussians that reach
// its pixels), its residuals and its backward pass on its own, and a second
// barrier precedes the flush
// of the tile's gradient accumulators.  Longer lists are staged chunk by
// chunk, twice.
template <int TILE, int PPL>
__device__ inline void residuals(const float (&a)[PPL][3], const float (&tg)[PPL][3],
                                 unsigned inside, float grad_scale, float (&g)[PPL][3], float *l) {
  float s = 0.f;
#pragma unroll
  for (int r = 0; r < PPL; ++r) {
    g[r][0] = g[r][1] = g[r][2] = 0.f;
    if ((inside >> r) & 1u) {
      const float r0 = a[r][0] - tg[r][0], r1 = a[r][1] - tg[r][1], r2 = a[r][2] - tg[r][2];
      s += r0 * r0 + r1 * r1 + r2 * r2;
      g[r][0] = r0 * grad_scale;
      g[r][1] = r1 * grad_scale;
      g[r][2] = r2 * grad_scale;
    }
  }
  *l = s;
}

// ONE: the caller runs one tile per workgroup (no LDS of an earlier tile to
// wait for before staging).
template <int TILE, int PPL, bool EXACT = true, bool ONE = false>
__device__ inline void fused_tile(Smem<Cfg<TILE, PPL>::NW> &S, float *acc, const FrameArgs &f,
                                  int tile, const float *__restrict__ target,
                                  float *__restrict__ loss_slots, float grad_scale,
                                  float *__restrict__ g_xy, float *__restrict__ g_chol,
                                  float *__restrict__ g_rgb) {
  using C = Cfg<TILE, PPL>;
  const int w = threadIdx.x >> 6;
  const int tx = tile % f.TX, ty = tile / f.TX;
  const int beg = f.tile_start[tile], end = f.tile_start[tile + 1];
  int px, py0;
  pixel_of_thread<TILE, PPL>(tx, ty, &px, &py0);
  const float pxc = (float)px + 0.5f, pyc0 = (float)py0 + 0.5f;
  const unsigned inside = inside_mask<PPL>(f, px, py0);
  // the target pixels are loaded first, their latency hidden by the staging
  const size_t HW = (size_t)f.W * f.H;
  float tg[PPL][3];
#pragma unroll
  for (int r = 0; r < PPL; ++r) {
    const size_t p = ((inside >> r) & 1u) ? (size_t)(py0 + r) * f.W + px : 0;
    tg[r][0] = target[p];
    tg[r][1] = target[HW + p];
    tg[r][2] = target[2 * HW + p];
  }
  float a[PPL][3] = {};
  float g[PPL][3];
  float l;
  if (end - beg <= CH) {
    const int cnt = end - beg;
    if constexpr (!ONE) __syncthreads();  // LDS of a previous tile (persistent callers) is free
    stage_chunk<TILE, PPL, EXACT>(S, f.keys, beg, cnt, tx, ty, f.W, f.H, f.geom, f.rgb, f.active);
    for (int i = threadIdx.x; i < cnt * 8; i += C::NT) acc[i] = 0.f;
    __syncthreads();
    int len = compact_chunk<C::NW>(S, cnt);
    len = fwd_chunk<C::NW, PPL, !EXACT>(S, len, pxc, pyc0, inside, a);
    residuals<TILE, PPL>(a, tg, inside, grad_scale, g, &l);
    wave_loss(l, loss_slots + w);
    if (f.active) len = keep_active<C::NW>(S, len);
    bwd_chunk<C::NW, PPL, false>(S, acc, len, pxc, pyc0, g);
    __syncthreads();
    flush_grads<C::NT, C::NW, ONE>(S, acc, cnt, g_xy, g_chol, g_rgb);
    return;
  }
  for (int c = beg; c < end; c += CH) {
    const int cnt = min(CH, end - c);
    __syncthreads();
    stage_chunk<TILE, PPL, EXACT>(S, f.keys, c, cnt, tx, ty, f.W, f.H, f.geom, f.rgb);
    __syncthreads();
    const int len = compact_chunk<C::NW>(S, cnt);
    fwd_chunk<C::NW, PPL, false>(S, len, pxc, pyc0, inside, a);
  }
  residuals<TILE, PPL>(a, tg, inside, grad_scale, g, &l);
  wave_loss(l, loss_slots + w);
  for (int c = beg; c < end; c += CH) {
    const int cnt = min(CH, end - c);
    __syncthreads();
    stage_chunk<TILE, PPL, EXACT>(S, f.keys, c, cnt, tx, ty, f.W, f.H, f.geom, f.rgb, f.active);
    for (int i = threadIdx.x; i < cnt * 8; i += C::NT) acc[i] = 0.f;
    __syncthreads();
    int len = compact_chunk<C::NW>(S, cnt);
    if (f.active) len = keep_active<C::NW>(S, len);
    bwd_chunk<C::NW, PPL, !EXACT>(S, acc, len, pxc, pyc0, g);
    __syncthreads();
    flush_grads<C::NT, C::NW, ONE>(S, acc, cnt, g_xy, g_chol, g_rgb);
  }
}

}  // namespace gs2d
