// Learned initialiser: a small convolutional regressor (Sec. 3.2.B, made
// per-tile) with hand-written training and inference kernels.
//
// Network: input [H][W][8] (RGB, residual vs the previous frame, 2 zero
// channels) -> 4 x (conv3x3 stride 2 pad 1, 64 channels, ReLU) -> conv3x3
// stride 1 head with 73 channels = 9 count logits + 8 slots x 8 parameters,
// one output per 16x16 screen tile.  Activations are channels-last BF16,
// weights BF16 copies of FP32 master weights, accumulation FP32 on MFMA
// (v_mfma_f32_16x16x32_bf16).
//
// Every convolution pass is an implicit GEMM C[M x N] = A[M x K] B[K x N]
// whose operand tiles are staged in LDS as [row][k] (k contiguous, row pitch
// padded so that the 16-byte reads of one MFMA step hit distinct banks) and
// whose next stage is loaded into registers while the current one is
// multiplied:
//   forward      M = Cout, N = output pixels, K = (tap, Cin)
//                A = W[co][tap][ci], B = input gathered per tap (im2col);
//                bias, ReLU and the BF16 rounding run in the epilogue
//   grad input   M = Cin, N = input pixels of one stride-parity class,
//                K = (the class's taps, Cout).  With stride 2 an input pixel
//                (y, x) receives output gradients only through the taps
//                with ty = y + 1 (mod 2) and tx = x + 1 (mod 2): 1, 2, 2 or 4
//                of the 9, so the four parity classes are separate GEMMs and
//                no multiply-by-zero is issued.  The epilogue applies the
//                previous layer's ReLU' and writes its BF16 dZ directly.
//   grad weight  M = Cout, N = (tap, Cin), K = output pixels, split over
//                workgroups whose partial tiles a second kernel sums (plain
//                stores: FP32 atomics from every workgroup cost more than the
//                GEMM).  Both
//                operands are channels-last in memory and pixel-contiguous in
//                LDS: each thread loads an 8 pixel x 8 channel block and
//                transposes it in registers.  The blocks of the first N tile
//                also sum dZ over their pixels: the bias gradient.
// dZ = dL/d(layer output) masked by ReLU', held as BF16 [pixels][CoutS].
#include <cmath>

#include "gs2d_internal.h"

namespace gs2d {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int NLAYER = 5;
constexpr int HEAD_CH = 73;
constexpr int NSLOT = 8, NPAR = 8;
constexpr int KPAD = 32;     // K of the weight matrices is padded to one MFMA step
constexpr int KS = 64;       // k per LDS stage (forward, grad input)
constexpr int LP = KS + 8;   // its row pitch in halves (144 B = 9 x 16 B)
constexpr int PS = 128;      // output pixels per LDS stage (grad weight)
constexpr int LPW = PS + 8;  // its row pitch in halves (272 B = 17 x 16 B)
constexpr int GW_MIN_PIX = 4 * PS;  // smallest pixel range of a grad-weight block

__device__ inline uint16_t f2bf(float x) {  // round to nearest even
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

struct ConvDims {
  int Hin, Win, Cin, Hout, Wout, Cout, stride, relu;
  int Mpad;   // rows of the weight matrix (Cout rounded up to 64)
  int Kf;     // forward K = 9 * Cin, padded to a multiple of KPAD
  int CoutS;  // channel stride of dZ (Cout rounded up to 8)
  int Kb;     // row length of the transposed weights = 9 * CoutS, padded to KPAD
};

struct ConvArgs {
  ConvDims d;
  const uint16_t *x;     // layer input [Hin*Win][Cin] bf16 (grad input: its ReLU mask)
  const uint16_t *w;     // [Mpad][Kf] bf16, k = tap * Cin + ci
  const uint16_t *wt;    // [Cin][Kb] bf16, k = tap * CoutS + co (grad input)
  const float *bias;     // [Mpad]
  uint16_t *y;           // forward output [Hout*Wout][Cout] bf16 (hidden layers)
  float *y_planar;       // forward output [Cout][Hout*Wout] fp32 (head)
  const uint16_t *dz;    // dZ of this layer [Hout*Wout][CoutS] bf16
  uint16_t *dz_prev;     // grad input: dZ of the previous layer [Hin*Win][Cin] bf16
  float *gpart;          // grad weight: partial tiles [work][64 col][64 row] fp32
  float *bpart;          // grad weight: bias partials [split][M tile][64] fp32
  int ksplit;            // grad weight: output pixels per workgroup (multiple of PS)
  int ntile_n, nwork;    // grad weight: N tiles, real workgroups (grid rounded up to 8)
  int ncls;              // grad input: parity classes (4 for stride 2, else 1)
  int cls_tile0[5];      // grad input: first workgroup of each class, then the total
};

// One 32-deep MFMA step of a wave's (16 MI) x (16 NJ) tile.  As / Bs point at
// the wave's first A / B row in LDS ([row][k] with pitch PITCH); lane l reads
// row l & 15 of every 16-row block at k + 8 (l >> 4) as one 16-byte load.
template <int MI, int NJ, int PITCH>
__device__ __forceinline__ void mfma_step(const uint16_t *As, const uint16_t *Bs, int k, int lane,
                                          floatx4 (&acc)[MI][NJ]) {
  const int r = lane & 15, kk = k + (lane >> 4) * 8;
  bf16x8 av[MI], bv[NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
    av[i] = __builtin_bit_cast(bf16x8,
                               *reinterpret_cast<const uint4 *>(As + (16 * i + r) * PITCH + kk));
#pragma unroll
  for (int j = 0; j < NJ; ++j)
    bv[j] = __builtin_bit_cast(bf16x8,
                               *reinterpret_cast<const uint4 *>(Bs + (16 * j + r) * PITCH + kk));
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
}

// --------------------------------------------------------------- forward --
// Workgroup tile 64 (Cout) x 32 WN (pixels); waves 2 x 2, each 32 x 16 WN.
// Staging: A row t >> 2, k chunks (t & 3) * 8 and +32; B pixel rows
// (t >> 3) + 32 j, k chunk (t & 7) * 8 (one tap and 8 channels: Cin % 8 == 0).
template <int WN>
__global__ void __launch_bounds__(256) k_conv_fwd(ConvArgs a) {
  constexpr int BN = 32 * WN;
  __shared__ __attribute__((aligned(16))) uint16_t As[64 * LP];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN * LP];
  const ConvDims &d = a.d;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.y * 64;
  const long long P = (long long)d.Hout * d.Wout;
  const long long n0 = (long long)blockIdx.x * BN;
  const int K = d.Kf;
  const int ar = tid >> 2, ak = (tid & 3) * 8;
  const uint16_t *wrow = a.w + (size_t)(m0 + ar) * K;
  const int br = tid >> 3, bk = (tid & 7) * 8;
  int iy0[WN], ix0[WN];
  bool pv[WN];
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const long long p = n0 + br + 32 * j;
    pv[j] = p < P;
    const int oy = pv[j] ? (int)(p / d.Wout) : 0, ox = pv[j] ? (int)(p - (long long)oy * d.Wout) : 0;
    iy0[j] = oy * d.stride - 1;
    ix0[j] = ox * d.stride - 1;
  }
  uint4 ra[2], rb[WN];
  auto load = [&](int k0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k = k0 + ak + 32 * h;
      ra[h] = (k < K) ? *reinterpret_cast<const uint4 *>(wrow + k) : make_uint4(0, 0, 0, 0);
    }
    const int k = k0 + bk;
    const int tap = k / d.Cin, ci = k - tap * d.Cin;
    const int ty = tap / 3, tx = tap - 3 * ty;
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      rb[j] = make_uint4(0, 0, 0, 0);
      const int iy = iy0[j] + ty, ix = ix0[j] + tx;
      if (pv[j] && k < K && tap < 9 && iy >= 0 && iy < d.Hin && ix >= 0 && ix < d.Win)
        rb[j] = *reinterpret_cast<const uint4 *>(a.x + ((size_t)iy * d.Win + ix) * d.Cin + ci);
    }
  };
  floatx4 acc[2][WN];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int wm = w & 1, wn = w >> 1;
  load(0);
  for (int k0 = 0; k0 < K; k0 += KS) {
    __syncthreads();
    *reinterpret_cast<uint4 *>(As + ar * LP + ak) = ra[0];
    *reinterpret_cast<uint4 *>(As + ar * LP + ak + 32) = ra[1];
#pragma unroll
    for (int j = 0; j < WN; ++j) *reinterpret_cast<uint4 *>(Bs + (br + 32 * j) * LP + bk) = rb[j];
    __syncthreads();
    if (k0 + KS < K) load(k0 + KS);
    mfma_step<2, WN, LP>(As + 32 * wm * LP, Bs + 16 * WN * wn * LP, 0, lane, acc);
    if (k0 + 32 < K) mfma_step<2, WN, LP>(As + 32 * wm * LP, Bs + 16 * WN * wn * LP, 32, lane, acc);
  }
  // lane holds D[4 (lane >> 4) + r][lane & 15] of each 16 x 16 block
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int row = m0 + 32 * wm + 16 * i + 4 * (lane >> 4);
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      const long long col = n0 + 16 * WN * wn + 16 * j + (lane & 15);
      if (col >= P) continue;
      if (a.y) {
        if (row < d.Cout) {  // Cout is a multiple of 4 for the hidden layers
          uint16_t o[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            float v = acc[i][j][r] + a.bias[row + r];
            if (d.relu) v = fmaxf(v, 0.f);
            o[r] = f2bf(v);
          }
          *reinterpret_cast<uint2 *>(a.y + col * d.Cout + row) = *reinterpret_cast<uint2 *>(o);
        }
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (row + r < d.Cout) a.y_planar[(size_t)(row + r) * P + col] = acc[i][j][r] + a.bias[row + r];
      }
    }
  }
}

// ------------------------------------------------------------ grad input --
// Parity class c of a stride-2 layer: (py, px) = pixel parities, in order of
// decreasing K: (1,1) 4 taps, (1,0) 2, (0,1) 2, (0,0) 1.  Stride 1: one class
// with all 9 taps.  Class pixel (yy, xx) is input pixel (s yy + py, s xx + px);
// its j-th tap is (ty, tx) with ty = py ? 2 jy : 1 (stride 2) or jy (stride 1).
struct ParityClass {
  int py, px, nty, ntx, Hc, Wc;
};
__device__ __forceinline__ ParityClass parity_class(const ConvDims &d, int c) {
  ParityClass k;
  if (d.stride == 1) {
    k.py = k.px = 0;
    k.nty = k.ntx = 3;
    k.Hc = d.Hin;
    k.Wc = d.Win;
  } else {
    k.py = (c < 2) ? 1 : 0;
    k.px = (c == 0 || c == 2) ? 1 : 0;
    k.nty = k.py ? 2 : 1;
    k.ntx = k.px ? 2 : 1;
    k.Hc = (d.Hin - k.py + 1) / 2;
    k.Wc = (d.Win - k.px + 1) / 2;
  }
  return k;
}

// Workgroup tile 64 (Cin) x 32 WN (class pixels), staging as the forward.
template <int WN>
__global__ void __launch_bounds__(256) k_conv_bwd_data(ConvArgs a) {
  constexpr int BN = 32 * WN;
  __shared__ __attribute__((aligned(16))) uint16_t As[64 * LP];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN * LP];
  const ConvDims &d = a.d;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  int c = 0;
  while (c + 1 < a.ncls && (int)blockIdx.x >= a.cls_tile0[c + 1]) ++c;
  const ParityClass pc = parity_class(d, c);
  const long long Pc = (long long)pc.Hc * pc.Wc;
  const long long n0 = (long long)(blockIdx.x - a.cls_tile0[c]) * BN;
  const int m0 = blockIdx.y * 64;
  const int K = pc.nty * pc.ntx * d.CoutS;
  const int ar = tid >> 2, ak = (tid & 3) * 8;
  const bool arow_ok = m0 + ar < d.Cin;
  const uint16_t *wrow = a.wt + (size_t)(arow_ok ? m0 + ar : 0) * d.Kb;
  const int br = tid >> 3, bk = (tid & 7) * 8;
  int yb[WN], xb[WN];
  bool pv[WN];
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const long long q = n0 + br + 32 * j;
    pv[j] = q < Pc;
    const int yy = pv[j] ? (int)(q / pc.Wc) : 0, xx = pv[j] ? (int)(q - (long long)yy * pc.Wc) : 0;
    yb[j] = yy * d.stride + pc.py + 1;  // y + 1
    xb[j] = xx * d.stride + pc.px + 1;
  }
  auto tap_of = [&](int jt, int &ty, int &tx) {
    const int jy = jt / pc.ntx, jx = jt - jy * pc.ntx;
    ty = (d.stride == 1) ? jy : (pc.py ? 2 * jy : 1);
    tx = (d.stride == 1) ? jx : (pc.px ? 2 * jx : 1);
  };
  uint4 ra[2], rb[WN];
  auto load = [&](int k0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k = k0 + ak + 32 * h;
      ra[h] = make_uint4(0, 0, 0, 0);
      if (arow_ok && k < K) {
        const int jt = k / d.CoutS, co = k - jt * d.CoutS;
        int ty, tx;
        tap_of(jt, ty, tx);
        ra[h] = *reinterpret_cast<const uint4 *>(wrow + (ty * 3 + tx) * d.CoutS + co);
      }
    }
    const int k = k0 + bk;
    const int jt = k / d.CoutS, co = k - jt * d.CoutS;
    int ty, tx;
    tap_of(jt, ty, tx);
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      rb[j] = make_uint4(0, 0, 0, 0);
      // output pixel (oy, ox) with s oy = y + 1 - ty (exact by the class choice)
      const int oy2 = yb[j] - ty, ox2 = xb[j] - tx;
      if (pv[j] && k < K && oy2 >= 0 && ox2 >= 0) {
        const int oy = oy2 / d.stride, ox = ox2 / d.stride;
        if (oy < d.Hout && ox < d.Wout)
          rb[j] = *reinterpret_cast<const uint4 *>(a.dz + ((size_t)oy * d.Wout + ox) * d.CoutS + co);
      }
    }
  };
  floatx4 acc[2][WN];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int wm = w & 1, wn = w >> 1;
  load(0);
  // the epilogue's output pixels and their ReLU masks (the previous layer's
  // output), fetched now so that the loads overlap the K loop
  size_t po[WN];
  uint2 mask[2][WN];
#pragma unroll
  for (int j = 0; j < WN; ++j) {
    const long long q = n0 + 16 * WN * wn + 16 * j + (lane & 15);
    po[j] = ~(size_t)0;
    if (q < Pc) {
      const int yy = (int)(q / pc.Wc), xx = (int)(q - (long long)yy * pc.Wc);
      po[j] = (size_t)(yy * d.stride + pc.py) * d.Win + (xx * d.stride + pc.px);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int ci = m0 + 32 * wm + 16 * i + 4 * (lane >> 4);
      mask[i][j] = (po[j] != ~(size_t)0 && ci < d.Cin)
                       ? *reinterpret_cast<const uint2 *>(a.x + po[j] * d.Cin + ci)
                       : make_uint2(0, 0);
    }
  }
  for (int k0 = 0; k0 < K; k0 += KS) {
    __syncthreads();
    *reinterpret_cast<uint4 *>(As + ar * LP + ak) = ra[0];
    *reinterpret_cast<uint4 *>(As + ar * LP + ak + 32) = ra[1];
#pragma unroll
    for (int j = 0; j < WN; ++j) *reinterpret_cast<uint4 *>(Bs + (br + 32 * j) * LP + bk) = rb[j];
    __syncthreads();
    if (k0 + KS < K) load(k0 + KS);
    mfma_step<2, WN, LP>(As + 32 * wm * LP, Bs + 16 * WN * wn * LP, 0, lane, acc);
    if (k0 + 32 < K) mfma_step<2, WN, LP>(As + 32 * wm * LP, Bs + 16 * WN * wn * LP, 32, lane, acc);
  }
  // dZ of the previous layer = dL/dx masked by its ReLU' (x > 0), as BF16
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int ci = m0 + 32 * wm + 16 * i + 4 * (lane >> 4);
    if (ci >= d.Cin) continue;
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      if (po[j] == ~(size_t)0) continue;
      const uint16_t *mb = reinterpret_cast<const uint16_t *>(&mask[i][j]);
      uint16_t o[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) o[r] = f2bf(bf2f(mb[r]) > 0.f ? acc[i][j][r] : 0.f);
      *reinterpret_cast<uint2 *>(a.dz_prev + po[j] * d.Cin + ci) = *reinterpret_cast<uint2 *>(o);
    }
  }
}

// ----------------------------------------------------------- grad weight --
__device__ __forceinline__ uint32_t u4_at(const uint4 &u, int i) {
  return i == 0 ? u.x : i == 1 ? u.y : i == 2 ? u.z : u.w;
}

// Workgroup tile 64 (Cout) x 64 (tap, Cin) over a range of ksplit output
// pixels, PS per stage; waves 2 x 2, each 32 x 32; the tile goes to gpart.  Threads 0..127 stage A
// (dZ), 128..255 stage B (the input gathered at the tile's tap); thread
// chunk: 8 channels (group g = c >> 4) x 8 pixels (group q = c & 15).  The
// 1D grid is ordered so that the N tiles of one pixel range are consecutive
// work items on one XCD (workgroup b runs on XCD b % 8): dZ of that range is
// fetched into one L2.
__global__ void __launch_bounds__(256) k_conv_bwd_weight(ConvArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t As[64 * LPW];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[64 * LPW];
  const ConvDims &d = a.d;
  const int per_xcd = (int)(gridDim.x >> 3);
  const int work = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  if (work >= a.nwork) return;
  const int ntm = d.Mpad / 64;
  const int nt = work % a.ntile_n, mt = (work / a.ntile_n) % ntm, split = work / (a.ntile_n * ntm);
  const int m0 = mt * 64, n0 = nt * 64;
  const long long P = (long long)d.Hout * d.Wout;
  const long long kbeg = (long long)split * a.ksplit, kend = min(P, kbeg + a.ksplit);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const bool isA = tid < 128;
  const int ch = tid & 127, q = ch & 15, g = ch >> 4;
  // A: channels co0 .. co0 + 7 of dZ; B: columns n .. n + 7 = one tap, 8 channels
  const int co0 = m0 + 8 * g;
  const int n = n0 + 8 * g, tap = n / d.Cin, ci = n - tap * d.Cin;
  const int ty = tap / 3, tx = tap - 3 * ty;
  const bool colok = isA ? (co0 < d.CoutS) : (n < d.Kf && tap < 9);
  const bool do_bias = isA && nt == 0;
  uint4 v[8];
  auto load = [&](long long k0) {
    const long long p0 = k0 + 8 * q;
    if (isA) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const long long p = p0 + j;
        v[j] = (colok && p < kend)
                   ? *reinterpret_cast<const uint4 *>(a.dz + p * d.CoutS + co0)
                   : make_uint4(0, 0, 0, 0);
      }
    } else {
      int oy = (int)(min(p0, P - 1) / d.Wout);
      int ox = (int)(min(p0, P - 1) - (long long)oy * d.Wout);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        v[j] = make_uint4(0, 0, 0, 0);
        const int iy = oy * d.stride + ty - 1, ix = ox * d.stride + tx - 1;
        if (colok && p0 + j < kend && iy >= 0 && iy < d.Hin && ix >= 0 && ix < d.Win)
          v[j] = *reinterpret_cast<const uint4 *>(a.x + ((size_t)iy * d.Win + ix) * d.Cin + ci);
        if (++ox == d.Wout) {
          ox = 0;
          ++oy;
        }
      }
    }
  };
  float bsum[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) bsum[r] = 0.f;
  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int wm = w & 1, wn = w >> 1;
  uint16_t *dst = (isA ? As : Bs) + 8 * g * LPW + 8 * q;
  load(kbeg);
  for (long long k0 = kbeg; k0 < kend; k0 += PS) {
    __syncthreads();
    // 8 x 8 transpose: row 2i + (0|1) of channel pair i = the even / odd
    // halves of dword i of the 8 pixels
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      uint32_t lo[4], hi[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t e = u4_at(v[2 * j], i), o = u4_at(v[2 * j + 1], i);
        lo[j] = (e & 0xFFFFu) | (o << 16);
        hi[j] = (e >> 16) | (o & 0xFFFF0000u);
      }
      *reinterpret_cast<uint4 *>(dst + (2 * i) * LPW) = make_uint4(lo[0], lo[1], lo[2], lo[3]);
      *reinterpret_cast<uint4 *>(dst + (2 * i + 1) * LPW) = make_uint4(hi[0], hi[1], hi[2], hi[3]);
      if (do_bias) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          bsum[2 * i] += __uint_as_float(lo[j] << 16) + __uint_as_float(lo[j] & 0xFFFF0000u);
          bsum[2 * i + 1] += __uint_as_float(hi[j] << 16) + __uint_as_float(hi[j] & 0xFFFF0000u);
        }
      }
    }
    __syncthreads();
    if (k0 + PS < kend) load(k0 + PS);
    const int nsub = (int)min((long long)(PS / 32), (kend - k0 + 31) / 32);
#pragma unroll
    for (int s = 0; s < PS / 32; ++s)
      if (s < nsub) mfma_step<2, 2, LPW>(As + 32 * wm * LPW, Bs + 32 * wn * LPW, 32 * s, lane, acc);
  }
  if (do_bias) {  // lanes 16 k .. 16 k + 15 share the channel group
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      float s = bsum[r];
      s += __shfl_xor(s, 1, 64);
      s += __shfl_xor(s, 2, 64);
      s += __shfl_xor(s, 4, 64);
      s += __shfl_xor(s, 8, 64);
      if (q == 0) a.bpart[((size_t)split * ntm + mt) * 64 + 8 * g + r] = s;
    }
  }
  // partial tile, column-major: the 4 rows a lane holds are contiguous
  float *pt = a.gpart + (size_t)work * 4096;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int row = 32 * wm + 16 * i + 4 * (lane >> 4);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = 32 * wn + 16 * j + (lane & 15);
      *reinterpret_cast<float4 *>(pt + col * 64 + row) =
          make_float4(acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]);
    }
  }
}

// Sum of the grad-weight partial tiles over the pixel splits, added into dW
// (and the bias partials into dbias).  Grid x: 16 workgroups per 64 x 64
// tile (one element per thread), then one per M tile for the bias; grid y:
// chunks of GW_CHUNK splits, combined with FP32 atomics.
constexpr int GW_CHUNK = 32;
__global__ void __launch_bounds__(256)
k_gw_reduce(ConvDims d, int splits, int ntile_n, const float *__restrict__ gpart,
            const float *__restrict__ bpart, float *__restrict__ dw, float *__restrict__ db) {
  const int ntm = d.Mpad / 64, tiles = ntile_n * ntm;
  const int s0 = blockIdx.y * GW_CHUNK, s1 = min(splits, s0 + GW_CHUNK);
  const int tid = threadIdx.x;
  if ((int)blockIdx.x < 16 * tiles) {
    const int tile = blockIdx.x >> 4, e = (blockIdx.x & 15) * 256 + tid;
    const int row = (tile / ntile_n) * 64 + (e & 63), col = (tile % ntile_n) * 64 + (e >> 6);
    if (row >= d.Cout || col >= d.Kf) return;
    const float *src = gpart + (size_t)tile * 4096 + e;
    float sum = 0.f;
#pragma unroll 8
    for (int sp = s0; sp < s1; ++sp) sum += src[(size_t)sp * tiles * 4096];
    if (sum != 0.f) atomicAdd(&dw[(size_t)row * d.Kf + col], sum);
  } else {
    const int mt = blockIdx.x - 16 * tiles, co = mt * 64 + tid;
    if (tid >= 64 || co >= d.Cout) return;
    float sum = 0.f;
#pragma unroll 8
    for (int sp = s0; sp < s1; ++sp) sum += bpart[((size_t)sp * ntm + mt) * 64 + tid];
    if (sum != 0.f) atomicAdd(&db[co], sum);
  }
}

// Frame (+ residual) -> channels-last bf16 input [H*W][8].
__global__ void __launch_bounds__(256)
k_cnn_input(int H, int W, const float *__restrict__ frame, const float *__restrict__ prev,
            uint16_t *__restrict__ x) {
  const size_t HW = (size_t)H * W;
  for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < HW;
       p += (size_t)gridDim.x * blockDim.x) {
    uint16_t v[8];
    for (int c = 0; c < 3; ++c) {
      const float f = frame[c * HW + p];
      v[c] = f2bf(f);
      v[3 + c] = f2bf(prev ? f - prev[c * HW + p] : 0.f);
    }
    v[6] = v[7] = 0;
    *reinterpret_cast<uint4 *>(x + p * 8) = *reinterpret_cast<uint4 *>(v);
  }
}

__device__ inline float sigm(float z) { return 1.f / (1.f + __expf(-z)); }

// Per-tile loss: CE over the 9 count logits + Chamfer between the first k
// slots and the k targets (8-vectors).  16 lanes per tile: lane c < 9 holds
// count logit c, lane s < 8 holds prediction slot s and target s.  The head
// gradient goes out as dZ of the head (BF16 [n_tiles][CoutS]); per-tile loss
// sums to tile_loss (CE, CD).
__global__ void __launch_bounds__(256)
k_head_loss(int n_tiles, int CoutS, const float *__restrict__ head, const int *__restrict__ tcount,
            const float *__restrict__ tvec, const int *__restrict__ n_cd_dev,
            uint16_t *__restrict__ dz, float *__restrict__ tile_loss) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = gid >> 4, l = gid & 15, base = threadIdx.x & 48;  // group's first lane in the wave
  const bool live = t < n_tiles;
  const int tt = live ? t : 0;
  const float inv_tiles = 1.f / (float)n_tiles;
  const int n_cd = max(1, *n_cd_dev);
  const int k = min(max(tcount[tt], 0), NSLOT);
  // cross entropy of the count logits
  const float z = (l < 9) ? head[(size_t)l * n_tiles + tt] : -INFINITY;
  float mx = z;
  for (int o = 1; o < 16; o <<= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  float se = (l < 9) ? __expf(z - mx) : 0.f;
  for (int o = 1; o < 16; o <<= 1) se += __shfl_xor(se, o, 64);
  const float lse = mx + __logf(se);
  const float zk = __shfl(z, base + k, 64);
  const float ce = lse - zk;
  const float gce = (l < 9) ? (__expf(z - lse) - (l == k ? 1.f : 0.f)) * inv_tiles : 0.f;
  // Chamfer: predictions P (sigmoid on the two offsets), targets Q
  const int s = l & 7;
  float Pv[NPAR], Qv[NPAR], raw[2];
#pragma unroll
  for (int j = 0; j < NPAR; ++j) {
    const float r = head[(size_t)(9 + s * NPAR + j) * n_tiles + tt];
    if (j < 2) raw[j] = r;
    Pv[j] = (j < 2) ? sigm(r) : r;
    Qv[j] = tvec[((size_t)tt * NSLOT + s) * NPAR + j];
  }
  const float inv_k = k > 0 ? 1.f / (float)k : 0.f;
  // prediction s -> nearest target (first minimum)
  float bd = INFINITY, Qb[NPAR];
#pragma unroll
  for (int j = 0; j < NPAR; ++j) Qb[j] = 0.f;
  for (int qq = 0; qq < NSLOT; ++qq) {
    float Qq[NPAR], dd = 0.f;
#pragma unroll
    for (int j = 0; j < NPAR; ++j) {
      Qq[j] = __shfl(Qv[j], base + qq, 64);
      dd += (Pv[j] - Qq[j]) * (Pv[j] - Qq[j]);
    }
    if (qq < k && dd < bd) {
      bd = dd;
#pragma unroll
      for (int j = 0; j < NPAR; ++j) Qb[j] = Qq[j];
    }
  }
  // target s -> nearest prediction (first minimum)
  float bd2 = INFINITY;
  int best2 = 0;
  for (int ss = 0; ss < NSLOT; ++ss) {
    float dd = 0.f;
#pragma unroll
    for (int j = 0; j < NPAR; ++j) {
      const float Ps = __shfl(Pv[j], base + ss, 64);
      dd += (Ps - Qv[j]) * (Ps - Qv[j]);
    }
    if (ss < k && dd < bd2) bd2 = dd, best2 = ss;
  }
  const bool own = l < 8 && s < k;
  float cd = own ? (bd + bd2) * inv_k : 0.f;
  for (int o = 1; o < 16; o <<= 1) cd += __shfl_xor(cd, o, 64);
  float gp[NPAR];
#pragma unroll
  for (int j = 0; j < NPAR; ++j) gp[j] = 2.f * (Pv[j] - Qb[j]) * inv_k;
  for (int qq = 0; qq < NSLOT; ++qq) {  // targets whose nearest prediction is s
    const int b = __shfl(best2, base + qq, 64);
#pragma unroll
    for (int j = 0; j < NPAR; ++j) {
      const float Qq = __shfl(Qv[j], base + qq, 64);
      if (qq < k && b == s) gp[j] += 2.f * (Pv[j] - Qq) * inv_k;
    }
  }
  if (!live) return;
  uint16_t *out = dz + (size_t)t * CoutS;
  if (l < 9) out[l] = f2bf(gce);
  if (l < 8) {
    const float sc = 1.f / (float)n_cd;
#pragma unroll
    for (int j = 0; j < NPAR; ++j) {
      float v = own ? gp[j] * sc : 0.f;
      if (j < 2) {
        const float sg = sigm(raw[j]);
        v *= sg * (1.f - sg);
      }
      out[9 + s * NPAR + j] = f2bf(v);
    }
  }
  if (l == 15)
    for (int c = HEAD_CH; c < CoutS; ++c) out[c] = 0;
  if (l == 0) {
    tile_loss[2 * t] = ce;
    tile_loss[2 * t + 1] = cd;
  }
}

__global__ void __launch_bounds__(256)
k_count_target_tiles(int n_tiles, const int *__restrict__ tcount, int *__restrict__ out) {
  __shared__ int red[4];
  int c = 0;
  for (int t = threadIdx.x; t < n_tiles; t += 256) c += tcount[t] > 0;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) *out = red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(1024)
k_loss_sum(int n_tiles, const float *__restrict__ tile_loss, const int *__restrict__ n_cd_dev,
           float *__restrict__ out) {
  __shared__ double red[2][16];
  double ce = 0.0, cd = 0.0;
  for (int t = threadIdx.x; t < n_tiles; t += 1024) {
    const float2 v = *reinterpret_cast<const float2 *>(tile_loss + 2 * t);
    ce += v.x;
    cd += v.y;
  }
  for (int o = 32; o > 0; o >>= 1) {
    ce += __shfl_xor(ce, o, 64);
    cd += __shfl_xor(cd, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = ce;
    red[1][threadIdx.x >> 6] = cd;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double c1 = 0.0, c2 = 0.0;
    for (int w = 0; w < 16; ++w) {
      c1 += red[0][w];
      c2 += red[1][w];
    }
    const int n_cd = *n_cd_dev;
    out[0] = (float)(c1 / n_tiles + (n_cd > 0 ? c2 / n_cd : 0.0));
    out[1] = (float)(c1 / n_tiles);
    out[2] = (float)(n_cd > 0 ? c2 / n_cd : 0.0);
  }
}

}  // namespace

// ------------------------------------------------------------ layout ----
// Grad-weight work split: about 1024 workgroups (split x tile), each over a
// multiple of PS and at least GW_MIN_PIX output pixels.
struct GwSplit {
  int ntile_n, tiles, ksplit, splits;
};
static GwSplit gw_split(const ConvDims &d) {
  GwSplit g;
  const long long P = (long long)d.Hout * d.Wout;
  g.ntile_n = (d.Kf + 63) / 64;
  g.tiles = g.ntile_n * (d.Mpad / 64);
  const long long want = std::max(1, 1024 / g.tiles);
  long long ks = (P + want - 1) / want;
  ks = std::max<long long>(GW_MIN_PIX, (ks + PS - 1) / PS * PS);
  g.ksplit = (int)ks;
  g.splits = (int)((P + ks - 1) / ks);
  return g;
}

struct CnnLayout {
  int H, W;
  ConvDims L[NLAYER];
  size_t w_off[NLAYER], b_off[NLAYER], n_params;   // FP32 master / grad offsets (floats)
  size_t wb_off[NLAYER], n_wb;                    // bf16 weight offsets (elements)
  size_t wt_off[NLAYER], n_wt;                    // bf16 transposed weights (elements)
  // workspace (bytes)
  size_t x_in, act[NLAYER], head, dz[NLAYER], gpart, bpart, tcount, tvec, tile_loss, ncd, total;
  int TX, TY, n_tiles;
};

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

static bool cnn_layout(int H, int W, CnnLayout *C) {
  if (H < 16 || W < 16 || (long long)H * W > (1LL << 26)) return false;
  C->H = H;
  C->W = W;
  int h = H, w = W, cin = 8;
  size_t pw = 0, wb = 0, wt = 0;
  for (int i = 0; i < NLAYER; ++i) {
    ConvDims &d = C->L[i];
    const bool head = (i == NLAYER - 1);
    d.Hin = h;
    d.Win = w;
    d.Cin = cin;
    d.stride = head ? 1 : 2;
    d.Hout = (h + 2 - 3) / d.stride + 1;
    d.Wout = (w + 2 - 3) / d.stride + 1;
    d.Cout = head ? HEAD_CH : 64;
    d.relu = head ? 0 : 1;
    d.Mpad = (d.Cout + 63) / 64 * 64;
    d.Kf = (9 * d.Cin + KPAD - 1) / KPAD * KPAD;
    d.CoutS = (d.Cout + 7) / 8 * 8;
    d.Kb = (9 * d.CoutS + KPAD - 1) / KPAD * KPAD;
    C->w_off[i] = pw;
    pw += (size_t)d.Mpad * d.Kf;
    C->b_off[i] = pw;
    pw += d.Mpad;
    C->wb_off[i] = wb;
    wb += (size_t)d.Mpad * d.Kf;
    C->wt_off[i] = wt;
    wt += (size_t)d.Cin * d.Kb;
    h = d.Hout;
    w = d.Wout;
    cin = d.Cout;
  }
  C->n_params = pw;
  C->n_wb = wb;
  C->n_wt = wt;
  const ConvDims &hd = C->L[NLAYER - 1];
  C->TX = hd.Wout;
  C->TY = hd.Hout;
  C->n_tiles = C->TX * C->TY;
  size_t o = 0;
  auto take = [&o](size_t b) {
    const size_t at = o;
    o = al256(o + b);
    return at;
  };
  C->x_in = take((size_t)H * W * 8 * 2);
  for (int i = 0; i < NLAYER; ++i) {
    const ConvDims &d = C->L[i];
    C->act[i] = (i < NLAYER - 1) ? take((size_t)d.Hout * d.Wout * d.Cout * 2) : 0;
  }
  C->head = take((size_t)HEAD_CH * C->n_tiles * 4);
  size_t gp = 0, bp = 0;
  for (int i = 0; i < NLAYER; ++i) {  // dZ of every layer's output, BF16
    const ConvDims &d = C->L[i];
    C->dz[i] = take((size_t)d.Hout * d.Wout * d.CoutS * 2);
    const GwSplit g = gw_split(d);
    gp = std::max(gp, (size_t)g.splits * g.tiles * 4096 * 4);
    bp = std::max(bp, (size_t)g.splits * (d.Mpad / 64) * 64 * 4);
  }
  C->gpart = take(gp);
  C->bpart = take(bp);
  C->tcount = take((size_t)C->n_tiles * 4);
  C->tvec = take((size_t)C->n_tiles * NSLOT * NPAR * 4);
  C->tile_loss = take((size_t)C->n_tiles * 2 * 4);
  C->ncd = take(64);
  C->total = o;
  return true;
}

// Pixel tile 32 WN: the widest that still gives >= min_blocks workgroups.
static int pick_wn(long long pixels, int mtiles, long long min_blocks) {
  for (int wn = 4; wn > 1; wn >>= 1)
    if ((pixels + 32 * wn - 1) / (32 * wn) * mtiles >= min_blocks) return wn;
  return 1;
}

// Forward: 64-pixel tiles where they still give >= 2000 workgroups, else
// 32 (measured at 1080p: 128-pixel tiles are slower on every layer).
static hipError_t launch_conv_fwd(const ConvArgs &a, hipStream_t st) {
  const ConvDims &d = a.d;
  const long long P = (long long)d.Hout * d.Wout;
  const int mt = d.Mpad / 64, wn = std::min(2, pick_wn(P, mt, 2000));
  const dim3 g((unsigned)((P + 32 * wn - 1) / (32 * wn)), (unsigned)mt);
  if (wn == 4) hipLaunchKernelGGL(k_conv_fwd<4>, g, dim3(256), 0, st, a);
  else if (wn == 2) hipLaunchKernelGGL(k_conv_fwd<2>, g, dim3(256), 0, st, a);
  else hipLaunchKernelGGL(k_conv_fwd<1>, g, dim3(256), 0, st, a);
  return hipGetLastError();
}

// Grad input: the parity classes' tiles are concatenated along grid x in
// the class order of parity_class (largest K first).
static hipError_t launch_conv_bwd_data(ConvArgs a, hipStream_t st) {
  const ConvDims &d = a.d;
  const int mt = (d.Cin + 63) / 64, wn = pick_wn((long long)d.Hin * d.Win, mt, 1000);
  const long long bn = 32 * wn;
  a.ncls = d.stride == 2 ? 4 : 1;
  long long tiles = 0;
  for (int c = 0; c < a.ncls; ++c) {
    long long px;
    if (d.stride == 2) {
      const int py = c < 2 ? 1 : 0, pxp = (c == 0 || c == 2) ? 1 : 0;
      px = (long long)((d.Hin - py + 1) / 2) * ((d.Win - pxp + 1) / 2);
    } else {
      px = (long long)d.Hin * d.Win;
    }
    a.cls_tile0[c] = (int)tiles;
    tiles += (px + bn - 1) / bn;
  }
  a.cls_tile0[a.ncls] = (int)tiles;
  if (tiles == 0) return hipSuccess;
  const dim3 g((unsigned)tiles, (unsigned)mt);
  if (wn == 4) hipLaunchKernelGGL(k_conv_bwd_data<4>, g, dim3(256), 0, st, a);
  else if (wn == 2) hipLaunchKernelGGL(k_conv_bwd_data<2>, g, dim3(256), 0, st, a);
  else hipLaunchKernelGGL(k_conv_bwd_data<1>, g, dim3(256), 0, st, a);
  return hipGetLastError();
}

// Grad weight: partial tiles (gw_split), then their sum into dw / db.
static hipError_t launch_conv_bwd_weight(ConvArgs a, float *dw, float *db, hipStream_t st) {
  const ConvDims &d = a.d;
  const GwSplit g = gw_split(d);
  a.ntile_n = g.ntile_n;
  a.ksplit = g.ksplit;
  a.nwork = g.splits * g.tiles;
  const unsigned grid = (unsigned)((a.nwork + 7) / 8 * 8);
  hipLaunchKernelGGL(k_conv_bwd_weight, dim3(grid), dim3(256), 0, st, a);
  const dim3 rg((unsigned)(16 * g.tiles + d.Mpad / 64), (unsigned)((g.splits + GW_CHUNK - 1) / GW_CHUNK));
  hipLaunchKernelGGL(k_gw_reduce, rg, dim3(256), 0, st, d, g.splits, g.ntile_n, a.gpart, a.bpart,
                     dw, db);
  return hipGetLastError();
}

// ---------------------------------------------- weight conversion / Adam --
// Master FP32 weights -> BF16 copies in forward layout and, for the layers
// whose input gradient is needed, the transposed layout W^T[ci][tap][co].
__global__ void __launch_bounds__(256)
k_cnn_weights_to_bf16(ConvDims d, const float *__restrict__ wm, uint16_t *__restrict__ wb,
                      uint16_t *__restrict__ wt) {
  const size_t n = (size_t)d.Mpad * d.Kf;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const int co = (int)(i / d.Kf), k = (int)(i % d.Kf);
    const uint16_t b = f2bf(wm[i]);
    wb[i] = b;
    if (wt && co < d.Cout && k < 9 * d.Cin) {
      const int tap = k / d.Cin, ci = k % d.Cin;
      wt[(size_t)ci * d.Kb + tap * d.CoutS + co] = b;
    }
  }
}

// Where each layer's parameters live: FP32 master / gradient offsets
// (weights [Mpad][Kf] then bias [Mpad]) and the BF16 copies.
struct CnnParamMap {
  ConvDims d[NLAYER];
  long long w_off[NLAYER], b_off[NLAYER], wb_off[NLAYER], wt_off[NLAYER];
};

// Adam with decoupled weight decay on the FP32 master weights; each updated
// weight is written to its BF16 copies in the same pass (forward layout, and
// for the layers whose input gradient is needed the transposed one, whose
// padding keeps the zeros of the last full conversion).
__global__ void __launch_bounds__(256)
k_cnn_adam(size_t n, CnnParamMap map, float *__restrict__ p, float *__restrict__ g,
           float *__restrict__ m, float *__restrict__ v, const int32_t *__restrict__ step,
           float lr, float b1, float b2, float eps, float wd, uint16_t *__restrict__ wb,
           uint16_t *__restrict__ wt) {
  __shared__ float s_bc1, s_bc2;
  if (threadIdx.x == 0) {
    const int t = step[0];
    s_bc1 = (float)(1.0 - pow((double)b1, (double)t));
    s_bc2 = (float)(1.0 - pow((double)b2, (double)t));
  }
  __syncthreads();
  const float bc1 = s_bc1, bc2 = s_bc2;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const float gr = g[i], p0 = p[i];
    g[i] = 0.f;
    const float mm = b1 * m[i] + (1.f - b1) * gr;
    const float vv = b2 * v[i] + (1.f - b2) * gr * gr;
    m[i] = mm;
    v[i] = vv;
    // the decay acts on the weight itself, outside the adaptive scaling
    const float pn = p0 - lr * ((mm / bc1) / (sqrtf(vv / bc2) + eps) + wd * p0);
    p[i] = pn;
    int l = 0;
#pragma unroll
    for (int j = 1; j < NLAYER; ++j)
      if ((long long)i >= map.w_off[j]) l = j;
    if ((long long)i >= map.b_off[l]) continue;  // a bias
    const ConvDims &d = map.d[l];
    const long long e = (long long)i - map.w_off[l];
    const int co = (int)(e / d.Kf), k = (int)(e - (long long)co * d.Kf);
    const uint16_t b = f2bf(pn);
    wb[map.wb_off[l] + e] = b;
    if (l > 0 && co < d.Cout && k < 9 * d.Cin) {
      const int tap = k / d.Cin, ci = k - tap * d.Cin;
      wt[map.wt_off[l] + (long long)ci * d.Kb + tap * d.CoutS + co] = b;
    }
  }
}

// ------------------------------------------------------------- decode ----
// Per tile: k = argmax of the count logits (first maximum), slots 0..k-1 ->
// Gaussians.  counts[t] = k; a scan and a write kernel place them in tile
// order.
__global__ void __launch_bounds__(256)
k_decode_counts(int n_tiles, const float *__restrict__ head, int *__restrict__ counts) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  int best = 0;
  float bv = head[t];
  for (int c = 1; c < 9; ++c) {
    const float z = head[(size_t)c * n_tiles + t];
    if (z > bv) bv = z, best = c;
  }
  counts[t] = best;
}

__global__ void __launch_bounds__(1024)
k_decode_scan(int n_tiles, const int *__restrict__ counts, int *__restrict__ offsets) {
  // single block, sequential chunks per thread + block scan
  __shared__ int part[1024];
  const int per = (n_tiles + 1023) / 1024;
  const int beg = min(n_tiles, (int)threadIdx.x * per), end = min(n_tiles, beg + per);
  int s = 0;
  for (int i = beg; i < end; ++i) s += counts[i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int x = (int)threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += x;
    __syncthreads();
  }
  int run = part[threadIdx.x] - s;
  for (int i = beg; i < end; ++i) {
    offsets[i] = run;
    run += counts[i];
  }
  if (threadIdx.x == 1023) offsets[n_tiles] = part[1023];
}

// Slot s of tile t (column tx, row ty) of the head [73][n_tiles] as a
// Gaussian: mu = tile origin + T sigmoid(p0, p1), l1 = exp(clamp(p2, +-4)),
// l2 = p3, l3 = exp(clamp(p4, +-4)), colour (p5, p6, p7); returns whether
// the eight raw parameters are finite.
__device__ inline bool decode_slot(const float *__restrict__ head, int n_tiles, int t, int s,
                                   int tx, int ty, int T, float *__restrict__ xy,
                                   float *__restrict__ chol, float *__restrict__ rgb) {
  float p[NPAR];
  bool ok = true;
  for (int j = 0; j < NPAR; ++j) {
    p[j] = head[(size_t)(9 + s * NPAR + j) * n_tiles + t];
    ok = ok && isfinite(p[j]);
  }
  xy[0] = (float)(tx * T) + (float)T * sigm(p[0]);
  xy[1] = (float)(ty * T) + (float)T * sigm(p[1]);
  chol[0] = __expf(fminf(fmaxf(p[2], -4.f), 4.f));
  chol[1] = p[3];
  chol[2] = __expf(fminf(fmaxf(p[4], -4.f), 4.f));
  rgb[0] = p[5];
  rgb[1] = p[6];
  rgb[2] = p[7];
  return ok;
}

__global__ void __launch_bounds__(256)
k_decode_write(int n_tiles, int TX, int T, const float *__restrict__ head,
               const int *__restrict__ counts, const int *__restrict__ offsets, int N_out,
               float *__restrict__ xy, float *__restrict__ chol, float *__restrict__ rgb,
               int *__restrict__ bad) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const int tx = t % TX, ty = t / TX;
  const int k = counts[t], o = offsets[t];
  for (int s = 0; s < k; ++s) {
    const int n = o + s;
    if (n >= N_out) break;
    decode_slot(head, n_tiles, t, s, tx, ty, T, xy + 2 * n, chol + 3 * n, rgb + 3 * n);
    bool ok = isfinite(xy[2 * n]) && isfinite(xy[2 * n + 1]) && isfinite(chol[3 * n + 1]);
    for (int j = 0; j < 3; ++j) ok = ok && isfinite(rgb[3 * n + j]);
    if (!ok) atomicOr(bad, 1);
  }
}

// Fill slots [n_pred, N) of the output from the plain initialisation, or
// everything when the prediction is unusable (non-finite, or fewer than
// half of N Gaussians).
__global__ void __launch_bounds__(256)
k_decode_merge(int N, const int *__restrict__ total, const int *__restrict__ bad,
               const float *__restrict__ pxy, const float *__restrict__ pchol,
               const float *__restrict__ prgb, float *__restrict__ xy, float *__restrict__ chol,
               float *__restrict__ rgb, int *__restrict__ used_pred) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  const int np = min(*total, N);
  const bool fallback = (*bad != 0) || (2 * np < N);
  if (n == 0) *used_pred = fallback ? 0 : np;
  if (n >= N) return;
  if (!fallback && n < np) return;
  const int src = fallback ? n : n - np;
  xy[2 * n] = pxy[2 * src];
  xy[2 * n + 1] = pxy[2 * src + 1];
  for (int j = 0; j < 3; ++j) {
    chol[3 * n + j] = pchol[3 * src + j];
    rgb[3 * n + j] = prgb[3 * src + j];
  }
}

// ------------------------------------------- P-frame re-initialisation ----
// Tiles of a P-frame whose mean squared residual against the previous frame
// exceeds tau are re-initialised from the network's predictions.  One
// thread per T x T tile: e = (dr*dr + dg*dg) + db*db per pixel, the tile's
// in-frame pixels summed one at a time in row-major order, divided by their
// count (FP32, each operation rounded once: the selection is a decision).
// A selected tile's prediction count is the argmax of its count logits
// (first maximum); a non-finite raw parameter of a used slot sets *bad.
__global__ void __launch_bounds__(256)
k_pf_tiles(int H, int W, int TX, int n_tiles, int T, const float *__restrict__ frame,
           const float *__restrict__ prev, float tau, const float *__restrict__ head,
           uint8_t *__restrict__ sel, int *__restrict__ pcount, int *__restrict__ stats,
           int *__restrict__ bad) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const size_t HW = (size_t)H * W;
  const int tx = t % TX, ty = t / TX;
  const int x0 = tx * T, y0 = ty * T, x1 = min(x0 + T, W), y1 = min(y0 + T, H);
  float acc = 0.f;
  for (int y = y0; y < y1; ++y)
    for (int x = x0; x < x1; ++x) {
      const size_t p = (size_t)y * W + x;
      const float dr = f32_sub(frame[p], prev[p]);
      const float dg = f32_sub(frame[HW + p], prev[HW + p]);
      const float db = f32_sub(frame[2 * HW + p], prev[2 * HW + p]);
      acc = f32_add(acc, f32_add(f32_add(f32_mul(dr, dr), f32_mul(dg, dg)), f32_mul(db, db)));
    }
  const bool on = __fdiv_rn(acc, (float)((x1 - x0) * (y1 - y0))) > tau;
  sel[t] = on ? 1 : 0;
  int k = 0;
  if (on) {
    atomicAdd(&stats[0], 1);
    float bv = head[t];
    for (int c = 1; c < 9; ++c) {
      const float z = head[(size_t)c * n_tiles + t];
      if (z > bv) bv = z, k = c;
    }
    bool ok = true;
    for (int sl = 0; sl < k; ++sl)
      for (int j = 0; j < NPAR; ++j) ok = ok && isfinite(head[(size_t)(9 + sl * NPAR + j) * n_tiles + t]);
    if (!ok) atomicOr(bad, 1);
  }
  pcount[t] = k;
}

// One block: the warm-started Gaussians centred in a selected tile
// (floor(mu / T) in FP32) get their rank among those, in index order
// (frank[n], -1 for the others); stats = {selected tiles, freed,
// predicted, replaced = bad ? 0 : min(freed, predicted)}.
__global__ void __launch_bounds__(1024)
k_pf_freed(int N, int TX, int TY, int T, const float *__restrict__ xy,
           const uint8_t *__restrict__ sel, const int *__restrict__ pred_total,
           const int *__restrict__ bad, int *__restrict__ frank, int *__restrict__ stats) {
  __shared__ int part[1024];
  const int per = (N + 1023) / 1024;
  const int beg = min(N, (int)threadIdx.x * per), end = min(N, beg + per);
  const float fT = (float)T;
  auto freed = [&](int n) {
    const float gx = floorf(__fdiv_rn(xy[2 * n], fT)), gy = floorf(__fdiv_rn(xy[2 * n + 1], fT));
    if (!(gx >= 0.f && gx < (float)TX && gy >= 0.f && gy < (float)TY)) return false;
    return sel[(int)gy * TX + (int)gx] != 0;
  };
  int c = 0;
  for (int n = beg; n < end; ++n) c += freed(n) ? 1 : 0;
  part[threadIdx.x] = c;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int x = (int)threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += x;
    __syncthreads();
  }
  int r = part[threadIdx.x] - c;
  for (int n = beg; n < end; ++n) frank[n] = freed(n) ? r++ : -1;
  if (threadIdx.x == 1023) {
    const int f = part[1023], np = *pred_total;
    stats[1] = f;
    stats[2] = np;
    stats[3] = *bad ? 0 : min(f, np);
  }
}

// Freed Gaussian of rank r < replaced takes prediction r: the tile t with
// poff[t] <= r < poff[t + 1] (binary search), slot r - poff[t].
__global__ void __launch_bounds__(256)
k_pf_replace(int N, int n_tiles, int TX, int T, const int *__restrict__ frank,
             const int *__restrict__ stats, const int *__restrict__ poff,
             const float *__restrict__ head, float *__restrict__ xy, float *__restrict__ chol,
             float *__restrict__ rgb) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const int r = frank[n];
  if (r < 0 || r >= stats[3]) return;
  int lo = 0, hi = n_tiles;  // largest t with poff[t] <= r
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (poff[mid] <= r) lo = mid;
    else hi = mid;
  }
  decode_slot(head, n_tiles, lo, r - poff[lo], lo % TX, lo / TX, T, xy + 2 * n, chol + 3 * n,
              rgb + 3 * n);
}

// Per-tile targets from fitted Gaussians: the Gaussians whose centre lies
// in the tile, at most 8, those with the largest mass
//   m = |l1 * l3| * ((c0*c0 + c1*c1) + c2*c2)   (FP32, this order)
// (ties to the lower index), listed by increasing index.  One thread per
// tile walks that tile's centre list (sorted keys, ascending index).
__global__ void __launch_bounds__(256)
k_cnn_targets(int n_tiles, int TX, int T, const uint32_t *__restrict__ keys,
              const int *__restrict__ tile_start, const float *__restrict__ xy,
              const float *__restrict__ chol, const float *__restrict__ rgb,
              int *__restrict__ tcount, float *__restrict__ tvec) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  int sel[NSLOT];
  float sm[NSLOT];
  int k = 0;
  for (int i = tile_start[t]; i < tile_start[t + 1]; ++i) {
    const int n = (int)(keys[i] & 0xFFFFu);
    const float a = fabsf(f32_mul(chol[3 * n], chol[3 * n + 2]));
    const float c0 = rgb[3 * n], c1 = rgb[3 * n + 1], c2 = rgb[3 * n + 2];
    const float s = f32_add(f32_add(f32_mul(c0, c0), f32_mul(c1, c1)), f32_mul(c2, c2));
    const float m = f32_mul(a, s);
    if (k < NSLOT) {
      sel[k] = n;
      sm[k] = m;
      ++k;
    } else {
      // replace the lightest (largest index among equal masses) if heavier
      int worst = 0;
      for (int j = 1; j < NSLOT; ++j)
        if (sm[j] < sm[worst] || (sm[j] == sm[worst] && sel[j] > sel[worst])) worst = j;
      if (m > sm[worst]) {
        sel[worst] = n;
        sm[worst] = m;
      }
    }
  }
  // increasing index order
  for (int i = 1; i < k; ++i)
    for (int j = i; j > 0 && sel[j - 1] > sel[j]; --j) {
      const int ts = sel[j];
      sel[j] = sel[j - 1];
      sel[j - 1] = ts;
      const float tm = sm[j];
      sm[j] = sm[j - 1];
      sm[j - 1] = tm;
    }
  tcount[t] = k;
  const int tx = t % TX, ty = t / TX;
  for (int s = 0; s < NSLOT; ++s) {
    float v[NPAR] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (s < k) {
      const int n = sel[s];
      v[0] = (xy[2 * n] - (float)(tx * T)) / (float)T;
      v[1] = (xy[2 * n + 1] - (float)(ty * T)) / (float)T;
      v[2] = __logf(fabsf(chol[3 * n]));
      v[3] = chol[3 * n + 1];
      v[4] = __logf(fabsf(chol[3 * n + 2]));
      v[5] = rgb[3 * n];
      v[6] = rgb[3 * n + 1];
      v[7] = rgb[3 * n + 2];
    }
    for (int j = 0; j < NPAR; ++j) tvec[((size_t)t * NSLOT + s) * NPAR + j] = v[j];
  }
}

// keys[n] = (tile of the centre << 16) | n, or 0xFFFFFFFF when the centre is
// outside the frame or the Gaussian is degenerate (sorts last).
__global__ void __launch_bounds__(256)
k_centre_keys(int N, int W, int H, int TX, int T, const float *__restrict__ xy,
              const float *__restrict__ chol, uint32_t *__restrict__ keys, int *__restrict__ n_keys,
              int *__restrict__ n_valid) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n == 0) *n_keys = N;  // the sort's key count (all N keys are sorted)
  if (n >= N) return;
  const float x = xy[2 * n], y = xy[2 * n + 1];
  const float l1 = chol[3 * n], l3 = chol[3 * n + 2];
  bool ok = isfinite(x) && isfinite(y) && x >= 0.f && y >= 0.f && x < (float)W && y < (float)H &&
            isfinite(l1) && isfinite(l3) && l1 != 0.f && l3 != 0.f;
  uint32_t key = 0xFFFFFFFFu;
  if (ok) {
    const int tx = (int)floorf(x / (float)T), ty = (int)floorf(y / (float)T);
    key = ((uint32_t)(ty * TX + tx) << 16) | (uint32_t)n;
    atomicAdd(n_valid, 1);
  }
  keys[n] = key;
}

// He-normal initial weights from caller-supplied standard normal draws
// (one per parameter slot): W = z * sqrt(2 / (9 * fan_in_channels)) on the
// real (co < Cout, tap < 9, ci < cin_real) entries, 0 elsewhere; bias 0.
__global__ void __launch_bounds__(256)
k_cnn_init(ConvDims d, int cin_real, const float *__restrict__ z, float *__restrict__ w,
           float *__restrict__ b) {
  const size_t n = (size_t)d.Mpad * d.Kf;
  const float sc = sqrtf(2.f / (9.f * (float)cin_real));
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    const int co = (int)(i / d.Kf), k = (int)(i % d.Kf);
    const int tap = k / d.Cin, ci = k % d.Cin;
    w[i] = (co < d.Cout && tap < 9 && ci < cin_real) ? z[i] * sc : 0.f;
    if (i < (size_t)d.Mpad) b[i] = 0.f;
  }
}

}  // namespace gs2d

using namespace gs2d;

extern "C" {

int gs2d_cnn_init_params(int32_t H, int32_t W, const float *normal_draws, float *master,
                         void *stream) {
  CnnLayout C;
  if (!cnn_layout(H, W, &C) || !normal_draws || !master) return GS2D_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  for (int i = 0; i < NLAYER; ++i) {
    const ConvDims &d = C.L[i];
    const size_t n = (size_t)d.Mpad * d.Kf;
    hipLaunchKernelGGL(k_cnn_init, dim3((unsigned)std::min<size_t>((n + 255) / 256, 2048)),
                       dim3(256), 0, st, d, i == 0 ? 6 : d.Cin, normal_draws + C.w_off[i],
                       master + C.w_off[i], master + C.b_off[i]);
  }
  return hipGetLastError() == hipSuccess ? GS2D_OK : GS2D_EHIP;
}

size_t gs2d_cnn_param_count(int32_t H, int32_t W) {
  CnnLayout C;
  return cnn_layout(H, W, &C) ? C.n_params : 0;
}

size_t gs2d_cnn_workspace_bytes(int32_t H, int32_t W) {
  CnnLayout C;
  return cnn_layout(H, W, &C) ? C.total : 0;
}

size_t gs2d_cnn_bf16_weight_count(int32_t H, int32_t W) {
  CnnLayout C;
  return cnn_layout(H, W, &C) ? C.n_wb + C.n_wt : 0;
}

int gs2d_cnn_layer_info(int32_t H, int32_t W, int32_t layer, int32_t *info /* [12] */) {
  CnnLayout C;
  if (!cnn_layout(H, W, &C) || layer < 0 || layer >= NLAYER || !info) return GS2D_EINVAL;
  const ConvDims &d = C.L[layer];
  const int32_t v[12] = {d.Hin, d.Win, d.Cin, d.Hout, d.Wout, d.Cout, d.stride, d.relu,
                         d.Mpad, d.Kf, (int32_t)C.w_off[layer], (int32_t)C.b_off[layer]};
  for (int i = 0; i < 12; ++i) info[i] = v[i];
  return GS2D_OK;
}

int gs2d_cnn_sync_weights(int32_t H, int32_t W, const float *master, uint16_t *wbf16,
                          void *stream) {
  CnnLayout C;
  if (!cnn_layout(H, W, &C) || !master || !wbf16) return GS2D_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  uint16_t *wt = wbf16 + C.n_wb;
  // the transposed copies are written sparsely: clear their padding first
  if (launch_fill_zero_u32(reinterpret_cast<uint32_t *>(wt), (C.n_wt + 1) / 2, st) != hipSuccess)
    return GS2D_EHIP;
  for (int i = 0; i < NLAYER; ++i) {
    const ConvDims &d = C.L[i];
    const size_t n = (size_t)d.Mpad * d.Kf;
    hipLaunchKernelGGL(k_cnn_weights_to_bf16, dim3((unsigned)std::min<size_t>((n + 255) / 256, 2048)),
                       dim3(256), 0, st, d, master + C.w_off[i], wbf16 + C.wb_off[i],
                       i > 0 ? wt + C.wt_off[i] : nullptr);
  }
  return hipGetLastError() == hipSuccess ? GS2D_OK : GS2D_EHIP;
}

int gs2d_cnn_forward(int32_t H, int32_t W, const float *frame, const float *prev,
                     const float *master, const uint16_t *wbf16, float *head_out, void *ws,
                     size_t ws_bytes, void *stream) {
  CnnLayout C;
  if (!cnn_layout(H, W, &C) || !frame || !master || !wbf16 || !ws) return GS2D_EINVAL;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return GS2D_EINVAL;
  if (ws_bytes < C.total) return GS2D_ENOSPACE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  uint16_t *x = at<uint16_t>(ws, C.x_in);
  hipLaunchKernelGGL(k_cnn_input, dim3((unsigned)std::min<size_t>(((size_t)H * W + 255) / 256, 8192)),
                     dim3(256), 0, st, H, W, frame, prev, x);
  const uint16_t *in = x;
  for (int i = 0; i < NLAYER; ++i) {
    ConvArgs a = {};
    a.d = C.L[i];
    a.x = in;
    a.w = wbf16 + C.wb_off[i];
    a.bias = master + C.b_off[i];
    if (i < NLAYER - 1) {
      a.y = at<uint16_t>(ws, C.act[i]);
      in = a.y;
    } else {
      a.y_planar = at<float>(ws, C.head);
    }
    if (launch_conv_fwd(a, st) != hipSuccess) return GS2D_EHIP;
  }
  if (head_out &&
      hipMemcpyAsync(head_out, at<float>(ws, C.head), sizeof(float) * HEAD_CH * C.n_tiles,
                     hipMemcpyDeviceToDevice, st) != hipSuccess)
    return GS2D_EHIP;
  return GS2D_OK;
}

int gs2d_cnn_targets(int32_t H, int32_t W, int32_t N, const float *xy, const float *chol,
                     const float *rgb, void *ws, size_t ws_bytes, void *scratch,
                     size_t scratch_bytes, void *stream) {
  CnnLayout C;
  if (!cnn_layout(H, W, &C) || N < 1 || N > 65536 || !xy || !chol || !rgb || !ws || !scratch)
    return GS2D_EINVAL;
  if (ws_bytes < C.total) return GS2D_ENOSPACE;
  // scratch: two key buffers [N], a radix histogram, tile_start, counters
  const int G = std::max(1, std::min(SORT_MAX_BLOCKS, (N + 2047) / 2048));
  const size_t need = al256(4 * (size_t)N) * 2 + al256(4 * (size_t)RADIX * G) +
                      al256(4 * ((size_t)C.n_tiles + 1)) + 256;
  if (scratch_bytes < need || (reinterpret_cast<uintptr_t>(scratch) & 255)) return GS2D_ENOSPACE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  size_t o = 0;
  uint32_t *ka = at<uint32_t>(scratch, o);
  o += al256(4 * (size_t)N);
  uint32_t *kb = at<uint32_t>(scratch, o);
  o += al256(4 * (size_t)N);
  uint32_t *hist = at<uint32_t>(scratch, o);
  o += al256(4 * (size_t)RADIX * G);
  int *tstart = at<int>(scratch, o);
  o += al256(4 * ((size_t)C.n_tiles + 1));
  int *misc = at<int>(scratch, o);  // [0] n keys, [1] n valid
  hipError_t e = launch_fill_zero_u32(reinterpret_cast<uint32_t *>(misc), 16, st);
  if (e != hipSuccess) return GS2D_EHIP;
  // all N keys are sorted (invalid ones carry tile 0xFFFF and sort last)
  hipLaunchKernelGGL(k_centre_keys, dim3((N + 255) / 256), dim3(256), 0, st, N, W, H, C.TX, 16, xy,
                     chol, ka, misc, misc + 1);
  const uint32_t *sorted = nullptr;
  e = launch_radix_sort_tiles(ka, kb, misc, G, hist, 2, st, &sorted);
  if (e == hipSuccess) e = launch_tile_ranges(sorted, misc + 1, C.n_tiles, tstart, st);
  if (e != hipSuccess) return GS2D_EHIP;
  hipLaunchKernelGGL(k_cnn_targets, dim3((C.n_tiles + 255) / 256), dim3(256), 0, st, C.n_tiles,
                     C.TX, 16, sorted, tstart, xy, chol, rgb, at<int>(ws, C.tcount),
                     at<float>(ws, C.tvec));
  hipLaunchKernelGGL(k_count_target_tiles, dim3(1), dim3(256), 0, st, C.n_tiles,
                     at<const int>(ws, C.tcount), at<int>(ws, C.ncd));
  return hipGetLastError() == hipSuccess ? GS2D_OK : GS2D_EHIP;
}

int gs2d_cnn_tensor_view(int32_t H, int32_t W, int32_t layer, int32_t which, const void *ws,
                         size_t ws_bytes, const void **ptr, int32_t *dims) {
  CnnLayout C;
  if (!cnn_layout(H, W, &C) || layer < 0 || layer >= NLAYER || !ws || !ptr || !dims)
    return GS2D_EINVAL;
  if (ws_bytes < C.total) return GS2D_ENOSPACE;
  const ConvDims &d = C.L[layer];
  const char *b = static_cast<const char *>(ws);
  if (which == 0) {  // the layer's input activations
    *ptr = b + (layer == 0 ? C.x_in : C.act[layer - 1]);
    dims[0] = d.Hin;
    dims[1] = d.Win;
    dims[2] = d.Cin;
  } else if (which == 1) {  // dLoss / d(layer output), ReLU mask applied
    *ptr = b + C.dz[layer];
    dims[0] = d.Hout;
    dims[1] = d.Wout;
    dims[2] = d.CoutS;
  } else {
    return GS2D_EINVAL;
  }
  return GS2D_OK;
}

int gs2d_cnn_read_targets(int32_t H, int32_t W, const void *ws, size_t ws_bytes, int32_t *counts,
                          float *vectors, void *stream) {
  CnnLayout C;
  if (!cnn_layout(H, W, &C) || !ws || !counts || !vectors) return GS2D_EINVAL;
  if (ws_bytes < C.total) return GS2D_ENOSPACE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const char *b = static_cast<const char *>(ws);
  if (hipMemcpyAsync(counts, b + C.tcount, 4 * (size_t)C.n_tiles, hipMemcpyDeviceToDevice, st) !=
          hipSuccess ||
      hipMemcpyAsync(vectors, b + C.tvec, 4 * (size_t)C.n_tiles * NSLOT * NPAR,
                     hipMemcpyDeviceToDevice, st) != hipSuccess)
    return GS2D_EHIP;
  return GS2D_OK;
}

int gs2d_cnn_backward(int32_t H, int32_t W, const float *master, const uint16_t *wbf16,
                      float *grad, float *loss3, void *ws, size_t ws_bytes, void *stream) {
  CnnLayout C;
  if (!cnn_layout(H, W, &C) || !master || !wbf16 || !grad || !ws) return GS2D_EINVAL;
  if (ws_bytes < C.total) return GS2D_ENOSPACE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const ConvDims &hd = C.L[NLAYER - 1];
  hipLaunchKernelGGL(k_head_loss, dim3((unsigned)((16LL * C.n_tiles + 255) / 256)), dim3(256), 0,
                     st, C.n_tiles, hd.CoutS, at<const float>(ws, C.head),
                     at<const int>(ws, C.tcount), at<const float>(ws, C.tvec),
                     at<const int>(ws, C.ncd), at<uint16_t>(ws, C.dz[NLAYER - 1]),
                     at<float>(ws, C.tile_loss));
  if (loss3)
    hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(1024), 0, st, C.n_tiles,
                       at<const float>(ws, C.tile_loss), at<const int>(ws, C.ncd), loss3);
  const uint16_t *wt = wbf16 + C.n_wb;
  for (int i = NLAYER - 1; i >= 0; --i) {
    ConvArgs a = {};
    a.d = C.L[i];
    a.x = (i == 0) ? at<const uint16_t>(ws, C.x_in) : at<const uint16_t>(ws, C.act[i - 1]);
    a.dz = at<const uint16_t>(ws, C.dz[i]);
    a.gpart = at<float>(ws, C.gpart);
    a.bpart = at<float>(ws, C.bpart);
    if (launch_conv_bwd_weight(a, grad + C.w_off[i], grad + C.b_off[i], st) != hipSuccess)
      return GS2D_EHIP;
    if (i > 0) {
      a.wt = wt + C.wt_off[i];
      a.dz_prev = at<uint16_t>(ws, C.dz[i - 1]);
      if (launch_conv_bwd_data(a, st) != hipSuccess) return GS2D_EHIP;
    }
  }
  return hipGetLastError() == hipSuccess ? GS2D_OK : GS2D_EHIP;
}

int gs2d_cnn_adam(int32_t H, int32_t W, float *master, float *grad, float *m, float *v,
                  int32_t *step, float lr, float weight_decay, uint16_t *wbf16, void *stream) {
  CnnLayout C;
  if (!cnn_layout(H, W, &C) || !master || !grad || !m || !v || !step || !wbf16)
    return GS2D_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (launch_step_tick(step, st) != hipSuccess) return GS2D_EHIP;
  CnnParamMap map;
  for (int i = 0; i < NLAYER; ++i) {
    map.d[i] = C.L[i];
    map.w_off[i] = (long long)C.w_off[i];
    map.b_off[i] = (long long)C.b_off[i];
    map.wb_off[i] = (long long)C.wb_off[i];
    map.wt_off[i] = (long long)C.wt_off[i];
  }
  hipLaunchKernelGGL(k_cnn_adam, dim3((unsigned)std::min<size_t>((C.n_params + 255) / 256, 2048)),
                     dim3(256), 0, st, C.n_params, map, master, grad, m, v, step, lr, 0.9f, 0.999f,
                     1e-8f, weight_decay, wbf16, wbf16 + C.n_wb);
  return hipGetLastError() == hipSuccess ? GS2D_OK : GS2D_EHIP;
}

int gs2d_cnn_decode(int32_t H, int32_t W, int32_t N, const float *plain_xy,
                    const float *plain_chol, const float *plain_rgb, float *xy, float *chol,
                    float *rgb, int32_t *n_predicted, void *ws, size_t ws_bytes, void *scratch,
                    size_t scratch_bytes, void *stream) {
  CnnLayout C;
  if (!cnn_layout(H, W, &C) || N < 1 || N > 65536 || !plain_xy || !plain_chol || !plain_rgb ||
      !xy || !chol || !rgb || !n_predicted || !ws || !scratch)
    return GS2D_EINVAL;
  if (ws_bytes < C.total) return GS2D_ENOSPACE;
  const size_t need = al256(4 * ((size_t)C.n_tiles + 1)) * 2 + 256;
  if (scratch_bytes < need || (reinterpret_cast<uintptr_t>(scratch) & 255)) return GS2D_ENOSPACE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  int *counts = at<int>(scratch, 0);
  int *offsets = at<int>(scratch, al256(4 * ((size_t)C.n_tiles + 1)));
  int *flags = at<int>(scratch, 2 * al256(4 * ((size_t)C.n_tiles + 1)));  // [0] bad
  if (launch_fill_zero_u32(reinterpret_cast<uint32_t *>(flags), 4, st) != hipSuccess)
    return GS2D_EHIP;
  const float *head = at<const float>(ws, C.head);
  const unsigned nb = (C.n_tiles + 255) / 256;
  hipLaunchKernelGGL(k_decode_counts, dim3(nb), dim3(256), 0, st, C.n_tiles, head, counts);
  hipLaunchKernelGGL(k_decode_scan, dim3(1), dim3(1024), 0, st, C.n_tiles, counts, offsets);
  hipLaunchKernelGGL(k_decode_write, dim3(nb), dim3(256), 0, st, C.n_tiles, C.TX, 16, head, counts,
                     offsets, N, xy, chol, rgb, flags);
  hipLaunchKernelGGL(k_decode_merge, dim3((N + 255) / 256), dim3(256), 0, st, N,
                     offsets + C.n_tiles, flags, plain_xy, plain_chol, plain_rgb, xy, chol, rgb,
                     n_predicted);
  return hipGetLastError() == hipSuccess ? GS2D_OK : GS2D_EHIP;
}

static size_t pf_scratch_layout(int n_tiles, int N, size_t *sel, size_t *pcount, size_t *poff,
                                size_t *frank, size_t *flags) {
  size_t o = 0;
  *sel = o;
  o += al256((size_t)n_tiles);
  *pcount = o;
  o += al256(4 * ((size_t)n_tiles + 1));
  *poff = o;
  o += al256(4 * ((size_t)n_tiles + 1));
  *frank = o;
  o += al256(4 * (size_t)N);
  *flags = o;
  o += 256;
  return o;
}

size_t gs2d_cnn_pframe_scratch_bytes(int32_t H, int32_t W, int32_t N) {
  CnnLayout C;
  if (!cnn_layout(H, W, &C) || N < 1 || N > 65536) return 0;
  size_t a, b, c, d, e;
  return pf_scratch_layout(C.n_tiles, N, &a, &b, &c, &d, &e);
}

int gs2d_cnn_pframe_replace(int32_t H, int32_t W, int32_t N, const float *frame,
                            const float *prev, float tau, const float *head, float *xy,
                            float *chol, float *rgb, int32_t *stats, uint8_t *tile_sel, void *ws,
                            size_t ws_bytes, void *scratch, size_t scratch_bytes, void *stream) {
  CnnLayout C;
  if (!cnn_layout(H, W, &C) || N < 1 || N > 65536 || !frame || !prev || !xy || !chol || !rgb ||
      !stats || !scratch || !(tau >= 0.f) || !std::isfinite(tau))
    return GS2D_EINVAL;
  if (!head) {
    if (!ws) return GS2D_EINVAL;
    if (ws_bytes < C.total) return GS2D_ENOSPACE;
    head = at<const float>(ws, C.head);
  }
  size_t o_sel, o_pc, o_po, o_fr, o_fl;
  const size_t need = pf_scratch_layout(C.n_tiles, N, &o_sel, &o_pc, &o_po, &o_fr, &o_fl);
  if (scratch_bytes < need || (reinterpret_cast<uintptr_t>(scratch) & 255)) return GS2D_ENOSPACE;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  uint8_t *sel = tile_sel ? tile_sel : at<uint8_t>(scratch, o_sel);
  int *pcount = at<int>(scratch, o_pc), *poff = at<int>(scratch, o_po);
  int *frank = at<int>(scratch, o_fr), *flags = at<int>(scratch, o_fl);
  if (launch_fill_zero_u32(reinterpret_cast<uint32_t *>(flags), 4, st) != hipSuccess ||
      launch_fill_zero_u32(reinterpret_cast<uint32_t *>(stats), 4, st) != hipSuccess)
    return GS2D_EHIP;
  const unsigned nb = (C.n_tiles + 255) / 256;
  hipLaunchKernelGGL(k_pf_tiles, dim3(nb), dim3(256), 0, st, H, W, C.TX, C.n_tiles, 16, frame,
                     prev, tau, head, sel, pcount, stats, flags);
  hipLaunchKernelGGL(k_decode_scan, dim3(1), dim3(1024), 0, st, C.n_tiles, pcount, poff);
  hipLaunchKernelGGL(k_pf_freed, dim3(1), dim3(1024), 0, st, N, C.TX, C.TY, 16, xy, sel,
                     poff + C.n_tiles, flags, frank, stats);
  hipLaunchKernelGGL(k_pf_replace, dim3((N + 255) / 256), dim3(256), 0, st, N, C.n_tiles, C.TX, 16,
                     frank, stats, poff, head, xy, chol, rgb);
  return hipGetLastError() == hipSuccess ? GS2D_OK : GS2D_EHIP;
}

}  // extern "C"
