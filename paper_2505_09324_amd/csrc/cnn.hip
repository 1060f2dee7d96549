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
// with a 64 x 64 workgroup tile, K in steps of 32, both operand tiles
// staged in LDS as [row][k] (k contiguous) so that each lane reads its 8
// BF16 MFMA operands with one 16-byte LDS load:
//   forward      M = Cout, N = output pixels, K = (tap, Cin)
//                A = W[co][tap][ci], B = input gathered per tap (im2col)
//   grad input   M = Cin,  N = input pixels,  K = (tap, Cout)
//                A = W^T[ci][tap][co], B = dZ gathered from the output
//                pixel each tap maps back to (stride-parity rule)
//   grad weight  M = Cout, N = (tap, Cin),    K = output pixels (split over
//                workgroups, FP32 atomics into dW)
// with dZ = dL/d(layer output) masked by ReLU'.
#include <cmath>

#include "gs2d_internal.h"

namespace gs2d {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 32, LDK = BK + 8;  // LDS row pitch (elements)
constexpr int NLAYER = 5;
constexpr int HEAD_CH = 73;
constexpr int NSLOT = 8, NPAR = 8;

__device__ inline uint16_t f2bf(float x) {  // round to nearest even
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

struct ConvDims {
  int Hin, Win, Cin, Hout, Wout, Cout, stride, relu;
  int Mpad;   // rows of the weight matrix (Cout rounded up to 64)
  int Kf;     // forward K = 9 * Cin, padded to a multiple of BK
  int CoutS;  // channel stride of dZ / output gradients (Cout rounded up to 8)
  int Kb;     // grad-input K = 9 * CoutS, padded to BK
};

// ------------------------------------------------------------------ GEMM --
enum { MODE_FWD = 0, MODE_BWD_DATA = 1, MODE_BWD_WEIGHT = 2 };

struct ConvArgs {
  ConvDims d;
  const uint16_t *x;       // layer input [Hin*Win][Cin] bf16
  const uint16_t *w;       // [Mpad][Kf] bf16 (forward / grad-weight output layout)
  const uint16_t *wt;      // [Cin][Kb] bf16 (grad input)
  const float *bias;       // [Mpad]
  uint16_t *y;             // forward output [Hout*Wout][Cout] bf16 (hidden layers)
  float *y_planar;         // forward output [Cout][Hout*Wout] fp32 (head)
  const float *dy;         // dL/d(output) [Hout*Wout][CoutS] fp32
  const uint16_t *yact;    // forward output of this layer (ReLU mask), bf16 [..][Cout]
  float *dx;               // dL/d(input) [Hin*Win][Cin] fp32
  float *dw;               // dL/dW [Mpad][Kf] fp32 (atomic adds)
  int ksplit;              // grad-weight: pixels per workgroup (multiple of BK)
};

// dZ = dy (masked by ReLU' when the layer has one), as bf16
__device__ inline void load_dz8(const ConvArgs &a, long long p, int co, uint16_t out[8]) {
  const float *src = a.dy + p * a.d.CoutS + co;
  const float4 u0 = *reinterpret_cast<const float4 *>(src);
  const float4 u1 = *reinterpret_cast<const float4 *>(src + 4);
  float v[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
  if (a.d.relu) {
    // yact has stride Cout (= 64 for every ReLU layer)
    const uint4 m = *reinterpret_cast<const uint4 *>(a.yact + p * a.d.Cout + co);
    const uint16_t *mb = reinterpret_cast<const uint16_t *>(&m);
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (bf2f(mb[j]) > 0.f) ? v[j] : 0.f;
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) out[j] = (co + j < a.d.Cout) ? f2bf(v[j]) : (uint16_t)0;
}

template <int MODE>
__global__ void __launch_bounds__(256) k_conv_gemm(ConvArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t As[BM][LDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN][LDK];
  const ConvDims &d = a.d;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.y * BM;
  const int n0 = blockIdx.x * BN;
  int K, kbeg, kend;
  if (MODE == MODE_FWD) {
    K = d.Kf;
    kbeg = 0;
    kend = K;
  } else if (MODE == MODE_BWD_DATA) {
    K = d.Kb;
    kbeg = 0;
    kend = K;
  } else {
    K = d.Hout * d.Wout;
    kbeg = blockIdx.z * a.ksplit;
    kend = min(K, kbeg + a.ksplit);
  }
  floatx4 acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = floatx4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
    if (MODE == MODE_FWD || MODE == MODE_BWD_DATA) {
      // thread -> (row r, 8 consecutive k at kc)
      const int r = tid >> 2, kc = (tid & 3) * 8;
      const int k = k0 + kc;
      // A tile
      {
        uint4 v = make_uint4(0, 0, 0, 0);
        if (MODE == MODE_FWD) {
          v = *reinterpret_cast<const uint4 *>(a.w + (size_t)(m0 + r) * d.Kf + k);
        } else if (m0 + r < d.Cin) {
          v = *reinterpret_cast<const uint4 *>(a.wt + (size_t)(m0 + r) * d.Kb + k);
        }
        *reinterpret_cast<uint4 *>(&As[r][kc]) = v;
      }
      // B tile
      {
        uint16_t val[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        const long long p = (long long)n0 + r;
        if (MODE == MODE_FWD) {
          const int tap = k / d.Cin, ci = k % d.Cin;
          if (p < (long long)d.Hout * d.Wout && tap < 9) {
            const int oy = (int)(p / d.Wout), ox = (int)(p % d.Wout);
            const int iy = oy * d.stride + tap / 3 - 1, ix = ox * d.stride + tap % 3 - 1;
            if (iy >= 0 && iy < d.Hin && ix >= 0 && ix < d.Win) {
              const uint4 u = *reinterpret_cast<const uint4 *>(
                  a.x + ((size_t)iy * d.Win + ix) * d.Cin + ci);
              *reinterpret_cast<uint4 *>(val) = u;
            }
          }
        } else {
          const int tap = k / d.CoutS, co = k % d.CoutS;
          if (p < (long long)d.Hin * d.Win && tap < 9) {
            const int y = (int)(p / d.Win), x = (int)(p % d.Win);
            const int oy2 = y + 1 - tap / 3, ox2 = x + 1 - tap % 3;
            if (oy2 >= 0 && ox2 >= 0 && oy2 % d.stride == 0 && ox2 % d.stride == 0) {
              const int oy = oy2 / d.stride, ox = ox2 / d.stride;
              if (oy < d.Hout && ox < d.Wout) load_dz8(a, (long long)oy * d.Wout + ox, co, val);
            }
          }
        }
        *reinterpret_cast<uint4 *>(&Bs[r][kc]) = *reinterpret_cast<uint4 *>(val);
      }
    } else {
      // grad weight: k = output pixel. thread -> (pixel t>>3, 8 rows at (t&7)*8)
      const int pk = tid >> 3, rc = (tid & 7) * 8;
      const long long p = (long long)k0 + pk;
      uint16_t av[8] = {0, 0, 0, 0, 0, 0, 0, 0}, bv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (p < kend) {
        if (m0 + rc < d.CoutS) load_dz8(a, p, m0 + rc, av);
        const int n = n0 + rc;  // (tap, ci) column of dW
        const int tap = n / d.Cin, ci = n % d.Cin;
        if (tap < 9) {
          const int oy = (int)(p / d.Wout), ox = (int)(p % d.Wout);
          const int iy = oy * d.stride + tap / 3 - 1, ix = ox * d.stride + tap % 3 - 1;
          if (iy >= 0 && iy < d.Hin && ix >= 0 && ix < d.Win) {
            const uint4 u =
                *reinterpret_cast<const uint4 *>(a.x + ((size_t)iy * d.Win + ix) * d.Cin + ci);
            *reinterpret_cast<uint4 *>(bv) = u;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        As[rc + j][pk] = av[j];
        Bs[rc + j][pk] = bv[j];
      }
    }
    __syncthreads();
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    const bf16x8 A = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(&As[16 * w + r16][kq]));
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      const bf16x8 B =
          __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(&Bs[16 * nb + r16][kq]));
      acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, acc[nb], 0, 0, 0);
    }
  }

  // epilogue: lane holds D[4*(lane>>4) + r][lane & 15] of each 16x16 block
  const int mrow = m0 + 16 * w + 4 * (lane >> 4);
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const long long col = (long long)n0 + 16 * nb + (lane & 15);
    if (MODE == MODE_FWD) {
      if (col >= (long long)d.Hout * d.Wout) continue;
      if (a.y) {
        uint16_t o[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float v = acc[nb][r] + a.bias[mrow + r];
          if (d.relu) v = fmaxf(v, 0.f);
          o[r] = f2bf(v);
        }
        if (mrow < d.Cout)  // Cout is a multiple of 4 for hidden layers
          *reinterpret_cast<uint2 *>(a.y + col * d.Cout + mrow) = *reinterpret_cast<uint2 *>(o);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (mrow + r < d.Cout)
            a.y_planar[(size_t)(mrow + r) * d.Hout * d.Wout + col] = acc[nb][r] + a.bias[mrow + r];
      }
    } else if (MODE == MODE_BWD_DATA) {
      if (col >= (long long)d.Hin * d.Win || mrow >= d.Cin) continue;
      *reinterpret_cast<float4 *>(a.dx + col * d.Cin + mrow) =
          make_float4(acc[nb][0], acc[nb][1], acc[nb][2], acc[nb][3]);
    } else {
      if (col >= d.Kf) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (mrow + r < d.Cout && acc[nb][r] != 0.f)
          atomicAdd(&a.dw[(size_t)(mrow + r) * d.Kf + col], acc[nb][r]);
    }
  }
}

// dL/dbias[co] = sum over output pixels of dZ[p][co]; grid (pixel slices,
// 64-channel blocks), atomics across slices
__global__ void __launch_bounds__(256)
k_bias_grad(ConvDims d, const float *__restrict__ dy, const uint16_t *__restrict__ yact,
            float *__restrict__ db) {
  __shared__ float red[4][64];
  const int cl = threadIdx.x & 63, part = threadIdx.x >> 6;
  const int co = blockIdx.y * 64 + cl;
  const long long P = (long long)d.Hout * d.Wout;
  float s = 0.f;
  if (co < d.Cout) {
    for (long long p = blockIdx.x * 4 + part; p < P; p += (long long)gridDim.x * 4) {
      float v = dy[p * d.CoutS + co];
      if (d.relu && !(bf2f(yact[p * d.Cout + co]) > 0.f)) v = 0.f;
      s += v;
    }
  }
  red[part][cl] = s;
  __syncthreads();
  if (part == 0 && co < d.Cout) {
    const float t = red[0][cl] + red[1][cl] + red[2][cl] + red[3][cl];
    if (t != 0.f) atomicAdd(&db[co], t);
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
// slots and the k targets (8-vectors); gradients into dhead, channels-last
// [n_tiles][CoutS].  Partial loss sums per tile go to tile_loss (CE, CD).
__global__ void __launch_bounds__(256)
k_head_loss(int n_tiles, int CoutS, const float *__restrict__ head, const int *__restrict__ tcount,
            const float *__restrict__ tvec, const int *__restrict__ n_cd_dev, float *__restrict__ dhead,
            float *__restrict__ tile_loss) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const float inv_tiles = 1.f / (float)n_tiles;
  const int n_cd = max(1, *n_cd_dev);
  float z[9], g[HEAD_CH];
  for (int c = 0; c < HEAD_CH; ++c) g[c] = 0.f;
  float mx = -INFINITY;
  for (int c = 0; c < 9; ++c) {
    z[c] = head[(size_t)c * n_tiles + t];
    mx = fmaxf(mx, z[c]);
  }
  float se = 0.f;
  for (int c = 0; c < 9; ++c) se += __expf(z[c] - mx);
  const int k = min(max(tcount[t], 0), NSLOT);
  const float lse = mx + __logf(se);
  const float ce = lse - z[k];
  for (int c = 0; c < 9; ++c) g[c] = (__expf(z[c] - lse) - (c == k ? 1.f : 0.f)) * inv_tiles;
  float cd = 0.f;
  if (k > 0) {
    float P[NSLOT][NPAR], Q[NSLOT][NPAR], raw01[NSLOT][2];
    for (int s = 0; s < k; ++s)
      for (int j = 0; j < NPAR; ++j) {
        const float r = head[(size_t)(9 + s * NPAR + j) * n_tiles + t];
        if (j < 2) raw01[s][j] = r;
        P[s][j] = (j < 2) ? sigm(r) : r;
        Q[s][j] = tvec[((size_t)t * NSLOT + s) * NPAR + j];
      }
    float gp[NSLOT][NPAR];
    for (int s = 0; s < k; ++s)
      for (int j = 0; j < NPAR; ++j) gp[s][j] = 0.f;
    const float inv_k = 1.f / (float)k;
    // predictions -> nearest target; targets -> nearest prediction
    for (int s = 0; s < k; ++s) {
      int best = 0;
      float bd = INFINITY;
      for (int q = 0; q < k; ++q) {
        float dd = 0.f;
        for (int j = 0; j < NPAR; ++j) dd += (P[s][j] - Q[q][j]) * (P[s][j] - Q[q][j]);
        if (dd < bd) bd = dd, best = q;
      }
      cd += bd * inv_k;
      for (int j = 0; j < NPAR; ++j) gp[s][j] += 2.f * (P[s][j] - Q[best][j]) * inv_k;
    }
    for (int q = 0; q < k; ++q) {
      int best = 0;
      float bd = INFINITY;
      for (int s = 0; s < k; ++s) {
        float dd = 0.f;
        for (int j = 0; j < NPAR; ++j) dd += (P[s][j] - Q[q][j]) * (P[s][j] - Q[q][j]);
        if (dd < bd) bd = dd, best = s;
      }
      cd += bd * inv_k;
      for (int j = 0; j < NPAR; ++j) gp[best][j] += 2.f * (P[best][j] - Q[q][j]) * inv_k;
    }
    const float sc = 1.f / (float)n_cd;
    for (int s = 0; s < k; ++s)
      for (int j = 0; j < NPAR; ++j) {
        float v = gp[s][j] * sc;
        if (j < 2) {
          const float sg = sigm(raw01[s][j]);
          v *= sg * (1.f - sg);
        }
        g[9 + s * NPAR + j] = v;
      }
  }
  for (int c = 0; c < HEAD_CH; ++c) dhead[(size_t)t * CoutS + c] = g[c];
  for (int c = HEAD_CH; c < CoutS; ++c) dhead[(size_t)t * CoutS + c] = 0.f;
  tile_loss[2 * t] = ce;
  tile_loss[2 * t + 1] = cd;
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

__global__ void __launch_bounds__(256)
k_loss_sum(int n_tiles, const float *__restrict__ tile_loss, const int *__restrict__ n_cd_dev,
           float *__restrict__ out) {
  __shared__ double red[2][4];
  double ce = 0.0, cd = 0.0;
  for (int t = threadIdx.x; t < n_tiles; t += 256) {
    ce += tile_loss[2 * t];
    cd += tile_loss[2 * t + 1];
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
    const double c1 = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    const double c2 = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    const int n_cd = *n_cd_dev;
    out[0] = (float)(c1 / n_tiles + (n_cd > 0 ? c2 / n_cd : 0.0));
    out[1] = (float)(c1 / n_tiles);
    out[2] = (float)(n_cd > 0 ? c2 / n_cd : 0.0);
  }
}

}  // namespace

// ------------------------------------------------------------ layout ----
struct CnnLayout {
  int H, W;
  ConvDims L[NLAYER];
  size_t w_off[NLAYER], b_off[NLAYER], n_params;   // FP32 master / grad offsets (floats)
  size_t wb_off[NLAYER], n_wb;                    // bf16 weight offsets (elements)
  size_t wt_off[NLAYER], n_wt;                    // bf16 transposed weights (elements)
  // workspace (bytes)
  size_t x_in, act[NLAYER], head, dhead, dact[NLAYER], tcount, tvec, tile_loss, ncd, total;
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
    d.Mpad = (d.Cout + BM - 1) / BM * BM;
    d.Kf = (9 * d.Cin + BK - 1) / BK * BK;
    d.CoutS = (d.Cout + 7) / 8 * 8;
    d.Kb = (9 * d.CoutS + BK - 1) / BK * BK;
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
  C->dhead = take((size_t)C->n_tiles * hd.CoutS * 4);
  for (int i = 0; i < NLAYER; ++i) {
    const ConvDims &d = C->L[i];
    // gradient w.r.t. the input of layer i (not needed for layer 0)
    C->dact[i] = (i > 0) ? take((size_t)d.Hin * d.Win * d.Cin * 4) : 0;
  }
  C->tcount = take((size_t)C->n_tiles * 4);
  C->tvec = take((size_t)C->n_tiles * NSLOT * NPAR * 4);
  C->tile_loss = take((size_t)C->n_tiles * 2 * 4);
  C->ncd = take(64);
  C->total = o;
  return true;
}

static hipError_t conv_launch(int mode, const ConvArgs &a, hipStream_t st) {
  const ConvDims &d = a.d;
  if (mode == MODE_FWD) {
    dim3 g((unsigned)((d.Hout * (long long)d.Wout + BN - 1) / BN), (unsigned)(d.Mpad / BM));
    hipLaunchKernelGGL(k_conv_gemm<MODE_FWD>, g, dim3(256), 0, st, a);
  } else if (mode == MODE_BWD_DATA) {
    dim3 g((unsigned)((d.Hin * (long long)d.Win + BN - 1) / BN), (unsigned)((d.Cin + BM - 1) / BM));
    hipLaunchKernelGGL(k_conv_gemm<MODE_BWD_DATA>, g, dim3(256), 0, st, a);
  } else {
    const long long P = (long long)d.Hout * d.Wout;
    const int splits = (int)((P + a.ksplit - 1) / a.ksplit);
    dim3 g((unsigned)((d.Kf + BN - 1) / BN), (unsigned)((d.CoutS + BM - 1) / BM), (unsigned)splits);
    hipLaunchKernelGGL(k_conv_gemm<MODE_BWD_WEIGHT>, g, dim3(256), 0, st, a);
  }
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

__global__ void __launch_bounds__(256)
k_cnn_adam(size_t n, float *__restrict__ p, float *__restrict__ g, float *__restrict__ m,
           float *__restrict__ v, const int32_t *__restrict__ step, float lr, float b1, float b2,
           float eps, float wd) {
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
    const float gr = g[i] + wd * p[i];
    g[i] = 0.f;
    const float mm = b1 * m[i] + (1.f - b1) * gr;
    const float vv = b2 * v[i] + (1.f - b2) * gr * gr;
    m[i] = mm;
    v[i] = vv;
    p[i] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
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
    float p[NPAR];
    for (int j = 0; j < NPAR; ++j) p[j] = head[(size_t)(9 + s * NPAR + j) * n_tiles + t];
    const float mx = (float)(tx * T) + (float)T * sigm(p[0]);
    const float my = (float)(ty * T) + (float)T * sigm(p[1]);
    const float l1 = __expf(fminf(fmaxf(p[2], -4.f), 4.f));
    const float l3 = __expf(fminf(fmaxf(p[4], -4.f), 4.f));
    xy[2 * n] = mx;
    xy[2 * n + 1] = my;
    chol[3 * n] = l1;
    chol[3 * n + 1] = p[3];
    chol[3 * n + 2] = l3;
    rgb[3 * n] = p[5];
    rgb[3 * n + 1] = p[6];
    rgb[3 * n + 2] = p[7];
    bool ok = isfinite(mx) && isfinite(my) && isfinite(p[3]);
    for (int j = 5; j < 8; ++j) ok = ok && isfinite(p[j]);
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
    const float a = fabsf(__fmul_rn(chol[3 * n], chol[3 * n + 2]));
    const float c0 = rgb[3 * n], c1 = rgb[3 * n + 1], c2 = rgb[3 * n + 2];
    const float s = __fadd_rn(__fadd_rn(__fmul_rn(c0, c0), __fmul_rn(c1, c1)), __fmul_rn(c2, c2));
    const float m = __fmul_rn(a, s);
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
              const float *__restrict__ chol, uint32_t *__restrict__ keys, int *__restrict__ n_valid) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
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
    if (conv_launch(MODE_FWD, a, st) != hipSuccess) return GS2D_EHIP;
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
  hipLaunchKernelGGL(k_centre_keys, dim3((N + 255) / 256), dim3(256), 0, st, N, W, H, C.TX, 16, xy,
                     chol, ka, misc + 1);
  // all N keys are sorted (invalid ones carry tile 0xFFFF and sort last)
  const int32_t hN = N;
  if (hipMemcpyAsync(misc, &hN, sizeof(int32_t), hipMemcpyHostToDevice, st) != hipSuccess)
    return GS2D_EHIP;
  const uint32_t *sorted = nullptr;
  e = launch_radix_sort_tiles(ka, kb, misc, G, hist, 2, st, &sorted);
  if (e == hipSuccess) e = launch_tile_ranges(sorted, misc + 1, C.n_tiles, tstart, st);
  if (e != hipSuccess) return GS2D_EHIP;
  hipLaunchKernelGGL(k_cnn_targets, dim3((C.n_tiles + 255) / 256), dim3(256), 0, st, C.n_tiles,
                     C.TX, 16, sorted, tstart, xy, chol, rgb, at<int>(ws, C.tcount),
                     at<float>(ws, C.tvec));
  hipLaunchKernelGGL(k_count_target_tiles, dim3(1), dim3(256), 0, st, C.n_tiles,
                     at<const int>(ws, C.tcount), at<int>(ws, C.ncd));
  if (hipStreamSynchronize(st) != hipSuccess) return GS2D_EHIP;  // hN leaves scope
  return hipGetLastError() == hipSuccess ? GS2D_OK : GS2D_EHIP;
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
  hipLaunchKernelGGL(k_head_loss, dim3((C.n_tiles + 255) / 256), dim3(256), 0, st, C.n_tiles,
                     hd.CoutS, at<const float>(ws, C.head), at<const int>(ws, C.tcount),
                     at<const float>(ws, C.tvec), at<const int>(ws, C.ncd), at<float>(ws, C.dhead),
                     at<float>(ws, C.tile_loss));
  if (loss3)
    hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(256), 0, st, C.n_tiles,
                       at<const float>(ws, C.tile_loss), at<const int>(ws, C.ncd), loss3);
  const uint16_t *wt = wbf16 + C.n_wb;
  const float *dy = at<const float>(ws, C.dhead);
  for (int i = NLAYER - 1; i >= 0; --i) {
    const ConvDims &d = C.L[i];
    ConvArgs a = {};
    a.d = d;
    a.x = (i == 0) ? at<const uint16_t>(ws, C.x_in) : at<const uint16_t>(ws, C.act[i - 1]);
    a.dy = dy;
    a.yact = d.relu ? at<const uint16_t>(ws, C.act[i]) : nullptr;
    a.dw = grad + C.w_off[i];
    a.ksplit = 2048;
    if (conv_launch(MODE_BWD_WEIGHT, a, st) != hipSuccess) return GS2D_EHIP;
    const long long P = (long long)d.Hout * d.Wout;
    hipLaunchKernelGGL(k_bias_grad,
                       dim3((unsigned)std::min<long long>((P + 1023) / 1024, 1024),
                            (unsigned)((d.Cout + 63) / 64)),
                       dim3(256), 0, st, d, dy, a.yact, grad + C.b_off[i]);
    if (i > 0) {
      a.wt = wt + C.wt_off[i];
      a.dx = at<float>(ws, C.dact[i]);
      if (conv_launch(MODE_BWD_DATA, a, st) != hipSuccess) return GS2D_EHIP;
      dy = a.dx;
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
  hipLaunchKernelGGL(k_cnn_adam, dim3((unsigned)std::min<size_t>((C.n_params + 255) / 256, 2048)),
                     dim3(256), 0, st, C.n_params, master, grad, m, v, step, lr, 0.9f, 0.999f,
                     1e-8f, weight_decay);
  if (hipGetLastError() != hipSuccess) return GS2D_EHIP;
  return gs2d_cnn_sync_weights(H, W, master, wbf16, stream);
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

}  // extern "C"
