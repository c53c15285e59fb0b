// Learned warm start on gfx950: a small multilayer perceptron over per-node
// features, trained on the solvers' own steady fields (an addition to the
// paper's method; its Sec. 2 fixes the geometry the features describe).
//
// Network (fixed shape): 5 -> 128 -> 128 -> 128 -> 4, SiLU after each hidden
// layer, affine output.  Parameters live in one FP32 master vector in the
// layout W_1, b_1, ..., W_4, b_4 with W_l [out][in] row-major.  Products run
// on MFMA (v_mfma_f32_16x16x32_bf16: BF16 operands, FP32 accumulation);
// pre-activations and back-propagated errors are FP32 where they enter an
// element-wise derivative and rounded to BF16 where they enter a product.
//
// Every product is C = A Bt^T with both operands stored k-contiguous (row
// major over the reduction index), so fragments load as 16-byte vectors:
//   forward      Z_l  = A_{l-1} W_l^T      A [B][K], Bt = W_l [out][in]
//   backward     dA_l = dZ_{l+1} W_{l+1}   A = dZ [B][out], Bt = W^T [in][out]
//   weight grad  dW_l = dZ_l^T A_{l-1}     A = dZ^T [out][B], Bt = A^T [in][B]
// which is why the packed BF16 copy holds W and W^T, and why the forward of a
// training step writes each activation in both [B][128] and [128][B] order.
// Those transposed writes are cheap in the MFMA output layout: a lane holds
// four consecutive rows of one column.  The batch dimension is padded to a
// multiple of 64 (Bp); padded rows of the inputs and of dL/dy are zero, so
// they add nothing to any gradient.
//
// A block is four waves; a wave owns 16 rows and up to 128 columns (8 MFMA
// tiles, 32 accumulator registers).  The weight gradients reduce over the
// batch: the batch is split into chunks whose FP32 partials are then added in
// a fixed order, and bias gradients are fixed-order sums of per-block column
// sums, so training is bitwise reproducible.  The layered form is bound by
// HBM traffic of the activations (about 12 bytes per 256 flops of a hidden
// layer), far below the MFMA ridge.
#include <algorithm>
#include <cmath>

#include "common.hpp"

namespace mpf {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int kIn = 5, kW = 128, kOut = 4;
constexpr int kParams = kW * kIn + kW + 2 * (kW * kW + kW) + kOut * kW + kOut;
static_assert(kParams == 34308, "parameter count");
// master vector offsets
constexpr int oW1 = 0, ob1 = oW1 + kW * kIn, oW2 = ob1 + kW, ob2 = oW2 + kW * kW, oW3 = ob2 + kW,
              ob3 = oW3 + kW * kW, oW4 = ob3 + kW, ob4 = oW4 + kOut * kW;
static_assert(ob4 + kOut == kParams, "layout");
// packed BF16 copy: W1 [128][32] (in padded), W2, W2^T, W3, W3^T [128][128],
// W4 [16][128] (out padded), W4^T [128][32] (out padded)
constexpr int kK1 = 32;  // padded input width (one MFMA k-step)
constexpr int pW1 = 0, pW2 = pW1 + kW * kK1, pW2t = pW2 + kW * kW, pW3 = pW2t + kW * kW, pW3t = pW3 + kW * kW,
              pW4 = pW3t + kW * kW, pW4t = pW4 + 16 * kW, kPacked = pW4t + kW * kK1;

constexpr int kBlock = 256;
constexpr int kRowsPerBlock = 64;

__device__ __forceinline__ u16 to_bf16(float f) {  // round to nearest, ties to even
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (u16)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}

__device__ __forceinline__ float sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }

enum Epi { kPartial = 0, kHiddenFwd = 1, kOutFwd = 2, kHiddenBwd = 3 };

struct EpiArgs {
  // kPartial: C[z][m][n] (row stride ldc), FP32
  float* C;
  int64_t ldc;
  // kHiddenFwd: Z (FP32 [Bp][128], may be null), act [Bp][128], actT [128][Bp] (may be null)
  // kHiddenBwd: Z holds the pre-activation of this layer; act/actT receive dZ
  float* Z;
  u16* act;
  u16* actT;
  int64_t ldT;  // row stride of actT (= Bp)
  const float* bias;
  // kOutFwd: y [rows_valid][4]
  float* y;
  int64_t rows_valid;
  // kHiddenBwd: per-block column sums of dZ, [gridDim.x][128]
  float* colpart;
};

// C = A Bt^T over k in [z*kc, min(K, (z+1)*kc)); A [M][K] (lda), Bt [N][K]
// (ldb), rows m >= M / n >= N read as zero; K and kc multiples of 32.
template <int NT, int EPI>
__global__ __launch_bounds__(kBlock) void gemm_tn(int64_t M, int N, int64_t K, int64_t kc, const u16* __restrict__ A,
                                                  int64_t lda, const u16* __restrict__ Bt, int64_t ldb, EpiArgs e) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t m0 = (int64_t)blockIdx.x * kRowsPerBlock + wv * 16;
  const int n0 = blockIdx.y * (16 * NT);
  const int64_t kb = (int64_t)blockIdx.z * kc, ke = min(K, kb + kc);
  const int r = lane & 15, g = lane >> 4;
  f4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
  const int64_t am = m0 + r;
  const bool a_ok = am < M;
  const u16* ap = A + (a_ok ? am : 0) * lda + 8 * g;
  // row n0 + 16 t + r of Bt sits 16 t ldb elements past this lane's base row
  const u16* bb = Bt + (int64_t)(n0 + r) * ldb + 8 * g;
  const int64_t bstep = 16 * ldb;
  // two k-steps per iteration: all eighteen fragment loads are in flight
  // before the first product waits on them
  int64_t k0 = kb;
  for (; k0 + 32 < ke; k0 += 64) {
    bf16x8 fa0 = {}, fa1 = {};
    if (a_ok) {
      fa0 = *reinterpret_cast<const bf16x8*>(ap + k0);
      fa1 = *reinterpret_cast<const bf16x8*>(ap + k0 + 32);
    }
    bf16x8 fb0[NT], fb1[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      fb0[t] = bf16x8{};
      fb1[t] = bf16x8{};
      if (n0 + 16 * t + r < N) {
        fb0[t] = *reinterpret_cast<const bf16x8*>(bb + t * bstep + k0);
        fb1[t] = *reinterpret_cast<const bf16x8*>(bb + t * bstep + k0 + 32);
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa0, fb0[t], acc[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa1, fb1[t], acc[t], 0, 0, 0);
  }
  if (k0 < ke) {
    bf16x8 fa = {};
    if (a_ok) fa = *reinterpret_cast<const bf16x8*>(ap + k0);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      bf16x8 fb = {};
      if (n0 + 16 * t + r < N) fb = *reinterpret_cast<const bf16x8*>(bb + t * bstep + k0);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc[t], 0, 0, 0);
    }
  }
  // output layout: lane holds column n0 + 16 t + r, rows m0 + 4 g + (0..3)
  if constexpr (EPI == kPartial) {
    float* C = e.C + (int64_t)blockIdx.z * M * e.ldc;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int n = n0 + 16 * t + r;
      if (n >= N) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t m = m0 + 4 * g + i;
        if (m < M) C[m * e.ldc + n] = acc[t][i];
      }
    }
  } else if constexpr (EPI == kOutFwd) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int n = n0 + 16 * t + r;
      if (n >= N) continue;
      const float b = e.bias[n];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t m = m0 + 4 * g + i;
        if (m < e.rows_valid) e.y[m * N + n] = acc[t][i] + b;
      }
    }
  } else if constexpr (EPI == kHiddenFwd) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int n = n0 + 16 * t + r;
      const float b = e.bias[n];
      u16 h[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t m = m0 + 4 * g + i;
        const float z = acc[t][i] + b;
        if (e.Z) e.Z[m * kW + n] = z;
        h[i] = to_bf16(z * sigmoid(z));
        e.act[m * kW + n] = h[i];
      }
      if (e.actT) {
        uint2 pk;
        pk.x = (unsigned)h[0] | ((unsigned)h[1] << 16);
        pk.y = (unsigned)h[2] | ((unsigned)h[3] << 16);
        *reinterpret_cast<uint2*>(e.actT + (int64_t)n * e.ldT + m0 + 4 * g) = pk;
      }
    }
  } else {  // kHiddenBwd: dZ = dA * silu'(Z)
    __shared__ float red[kBlock / 64][kW];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int n = n0 + 16 * t + r;
      u16 h[4];
      float cs = 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t m = m0 + 4 * g + i;
        const float z = e.Z[m * kW + n];
        const float s = sigmoid(z);
        const float d = acc[t][i] * (s * (1.0f + z * (1.0f - s)));
        cs += d;
        h[i] = to_bf16(d);
        e.act[m * kW + n] = h[i];
      }
      uint2 pk;
      pk.x = (unsigned)h[0] | ((unsigned)h[1] << 16);
      pk.y = (unsigned)h[2] | ((unsigned)h[3] << 16);
      *reinterpret_cast<uint2*>(e.actT + (int64_t)n * e.ldT + m0 + 4 * g) = pk;
      // column sum over the wave's 16 rows: lanes r, r+16, r+32, r+48
      cs += __shfl_xor(cs, 16);
      cs += __shfl_xor(cs, 32);
      if (g == 0) red[wv][n - n0] = cs;
    }
    __syncthreads();
    if (threadIdx.x < 16 * NT) {
      float s = red[0][threadIdx.x];
#pragma unroll
      for (int w = 1; w < kBlock / 64; ++w) s += red[w][threadIdx.x];
      e.colpart[(int64_t)blockIdx.x * kW + n0 + threadIdx.x] = s;
    }
  }
}

// out[g * n + i] = sum of part[z * n + i] over z in [g G, min(parts, (g+1) G)),
// z ascending.  Two rounds (G ~ sqrt(parts)) turn any number of partials into
// one sum per element in a fixed order, with every round spread over the chip.
__global__ void group_sums(const float* __restrict__ part, int64_t parts, int64_t n, int64_t G,
                           float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t groups = (parts + G - 1) / G;
  if (t >= groups * n) return;
  const int64_t g = t / n, i = t % n;
  const int64_t z1 = min(parts, (g + 1) * G);
  float s = 0.f;
  for (int64_t z = g * G; z < z1; ++z) s += part[z * n + i];
  out[t] = s;
}

// inputs: x [B][5] FP32 (row b of the batch = x[rows ? rows[b] : b]) ->
// xb [Bp][32] BF16 and, for training, xbT [8][Bp]; padding zero
__global__ void pack_inputs(int64_t B, int64_t Bp, const float* __restrict__ x, const int64_t* __restrict__ rows,
                            u16* __restrict__ xb, u16* __restrict__ xbT) {
  const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (b >= Bp) return;
  const bool live = b < B;
  const int64_t src = live ? (rows ? rows[b] : b) : 0;
  u16 h[kK1];
#pragma unroll
  for (int j = 0; j < kK1; ++j) h[j] = (live && j < kIn) ? to_bf16(x[src * kIn + j]) : (u16)0;
  uint4* dst = reinterpret_cast<uint4*>(xb + b * kK1);
#pragma unroll
  for (int v = 0; v < kK1 / 8; ++v) {
    uint4 q;
    q.x = (unsigned)h[8 * v] | ((unsigned)h[8 * v + 1] << 16);
    q.y = (unsigned)h[8 * v + 2] | ((unsigned)h[8 * v + 3] << 16);
    q.z = (unsigned)h[8 * v + 4] | ((unsigned)h[8 * v + 5] << 16);
    q.w = (unsigned)h[8 * v + 6] | ((unsigned)h[8 * v + 7] << 16);
    dst[v] = q;
  }
  if (xbT)
#pragma unroll
    for (int j = 0; j < 8; ++j) xbT[j * Bp + b] = h[j];
}

// dL/dy [B][4] FP32 -> dyb [Bp][32] BF16 and dyT [4][Bp] BF16 (padding zero),
// plus each block's column sums of dy (FP32 tree over its 256 rows) for the
// output bias gradient
__global__ __launch_bounds__(kBlock) void pack_dy(int64_t B, int64_t Bp, const float* __restrict__ dy,
                                                  u16* __restrict__ dyb, u16* __restrict__ dyT,
                                                  float* __restrict__ colpart) {
  __shared__ float red[kOut][kBlock];
  const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool live = b < B;
  float d[kOut];
#pragma unroll
  for (int j = 0; j < kOut; ++j) {
    d[j] = live ? dy[b * kOut + j] : 0.f;
    red[j][threadIdx.x] = d[j];
  }
  if (b < Bp) {
    u16 h[kOut];
#pragma unroll
    for (int j = 0; j < kOut; ++j) h[j] = to_bf16(d[j]);
    uint4* dst = reinterpret_cast<uint4*>(dyb + b * kK1);
    uint4 q;
    q.x = (unsigned)h[0] | ((unsigned)h[1] << 16);
    q.y = (unsigned)h[2] | ((unsigned)h[3] << 16);
    q.z = 0u;
    q.w = 0u;
    dst[0] = q;
    q.x = q.y = 0u;
#pragma unroll
    for (int v = 1; v < kK1 / 8; ++v) dst[v] = q;
#pragma unroll
    for (int j = 0; j < kOut; ++j) dyT[j * Bp + b] = h[j];
  }
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int j = 0; j < kOut; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < kOut) colpart[(int64_t)blockIdx.x * kOut + threadIdx.x] = red[threadIdx.x][0];
}

// master -> packed BF16 (see the layout above)
__global__ void pack_params(const float* __restrict__ p, u16* __restrict__ w) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= kPacked) return;
  float v = 0.f;
  if (i < pW2) {
    const int o = (i - pW1) / kK1, k = (i - pW1) % kK1;
    v = k < kIn ? p[oW1 + o * kIn + k] : 0.f;
  } else if (i < pW2t) {
    v = p[oW2 + (i - pW2)];
  } else if (i < pW3) {
    const int a = (i - pW2t) / kW, b = (i - pW2t) % kW;  // W2^T[a][b] = W2[b][a]
    v = p[oW2 + b * kW + a];
  } else if (i < pW3t) {
    v = p[oW3 + (i - pW3)];
  } else if (i < pW4) {
    const int a = (i - pW3t) / kW, b = (i - pW3t) % kW;
    v = p[oW3 + b * kW + a];
  } else if (i < pW4t) {
    const int o = (i - pW4) / kW, k = (i - pW4) % kW;
    v = o < kOut ? p[oW4 + o * kW + k] : 0.f;
  } else {
    const int a = (i - pW4t) / kK1, o = (i - pW4t) % kK1;  // W4^T[a][o] = W4[o][a]
    v = o < kOut ? p[oW4 + o * kW + a] : 0.f;
  }
  w[i] = to_bf16(v);
}

// loss = mean (y - t)^2 over B x 4 entries (FP64 block partials), dy = 2 (y - t) / (4 B)
__global__ __launch_bounds__(kBlock) void mse_partial(int64_t B, const float* __restrict__ y,
                                                      const float* __restrict__ t, const int64_t* __restrict__ rows,
                                                      float* __restrict__ dy, double* __restrict__ part) {
  __shared__ double lds[kBlock];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t n = B * kOut;
  double e2 = 0.0;
  if (i < n) {
    const int64_t b = i / kOut, j = i % kOut;
    const int64_t src = rows ? rows[b] : b;
    const float d = y[i] - t[src * kOut + j];
    dy[i] = 2.0f * d / (float)n;
    e2 = (double)d * (double)d;
  }
  const double s = block_sum<kBlock>(e2, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void adam_kernel(int64_t n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// per-node features: minimum-image offset from the grain centre (1/2,1/2,1/2),
// signed distance to the grain surface, porosity
__global__ void features_kernel(int64_t n, const double* __restrict__ pos, double r, double phi,
                                float* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double d0 = min_image(pos[i] - 0.5), d1 = min_image(pos[n + i] - 0.5), d2 = min_image(pos[2 * n + i] - 0.5);
  x[i * kIn + 0] = (float)d0;
  x[i * kIn + 1] = (float)d1;
  x[i * kIn + 2] = (float)d2;
  x[i * kIn + 3] = (float)(sqrt(d0 * d0 + d1 * d1 + d2 * d2) - r);
  x[i * kIn + 4] = (float)phi;
}

// node sums of P y_3 (FP64 block partials)
__global__ __launch_bounds__(kBlock) void psum_partial(int64_t n, const float* __restrict__ y, double P,
                                                       double* __restrict__ part) {
  __shared__ double lds[kBlock];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const double v = i < n ? P * (double)y[i * kOut + 3] : 0.0;
  const double s = block_sum<kBlock>(v, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// outputs -> state: v = U y_{0..2} on interior nodes and 0 on the grain,
// p = P y_3 - mean; running max |v| into vmax (integer max on the bits of
// non-negative doubles)
template <typename T>
__global__ __launch_bounds__(kBlock) void to_state_kernel(int64_t n, int64_t n_int, const float* __restrict__ y,
                                                          double U, double P, const double* __restrict__ pmean,
                                                          T* __restrict__ v, T* __restrict__ p,
                                                          double* __restrict__ vmax) {
  __shared__ double lds[kBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double mag = 0.0;
  if (i < n) {
    const bool in = i < n_int;
    double m2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      const T va = in ? (T)(U * (double)y[i * kOut + a]) : T(0);
      v[a * n + i] = va;
      m2 += (double)va * (double)va;
    }
    p[i] = (T)(P * (double)y[i * kOut + 3] - *pmean);
    mag = sqrt(m2);
  }
  if (!vmax) return;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mag = fmax(mag, __shfl_xor(mag, off));
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x / 64] = mag;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = lds[0];
    for (int t = 1; t < kBlock / 64; ++t) m = fmax(m, lds[t]);
    if (m != m) m = __builtin_inf();
    atomicMax(reinterpret_cast<unsigned long long*>(vmax), (unsigned long long)__double_as_longlong(m));
  }
}

// A seeded permutation of [0, n) evaluated pointwise: a 4-round balanced
// Feistel network on 2h-bit integers (2^(2h) >= n), whose round function is
// a 32-bit integer hash of the right half and a round key, made a permutation
// of [0, n) by cycle walking (re-applying the network until the value falls
// below n; the walk ends because the network is a bijection of [0, 2^(2h))).
__device__ __forceinline__ unsigned mix32(unsigned x) {  // integer hash (xorshift-multiply)
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__global__ void shuffle_kernel(int64_t n, int64_t count, int h, unsigned long long seed, int64_t* __restrict__ rows) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= count) return;
  const unsigned long long mask = (1ull << h) - 1;
  unsigned k[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) k[r] = mix32((unsigned)(seed >> (16 * r)) ^ (0x9e3779b9u * (r + 1)) ^ (unsigned)(seed >> 32));
  unsigned long long x = (unsigned long long)i;
  do {
    unsigned long long L = x >> h, R = x & mask;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const unsigned long long F = (unsigned long long)mix32((unsigned)R ^ k[r] ^ (unsigned)(R >> 32)) & mask;
      const unsigned long long nl = R;
      R = L ^ F;
      L = nl;
    }
    x = (L << h) | R;
  } while (x >= (unsigned long long)n);
  rows[i] = (int64_t)x;
}

__global__ void zero_double(double* x) { *x = 0.0; }
__global__ void add_double(const double* x, double* sum) { *sum += *x; }

// ------------------------------------------------------------------ host side

inline int64_t isqrt_ceil(int64_t x) {
  int64_t r = (int64_t)std::sqrt((double)x);
  while (r * r < x) ++r;
  return r < 1 ? 1 : r;
}

// out[i] = sum_z part[z][i] for i < n, z < parts, in a fixed order (two rounds
// of group sums through tmp)
void reduce_parts(hipStream_t st, const float* part, int64_t parts, int64_t n, float* out, float* tmp) {
  if (parts <= 32) {
    hipLaunchKernelGGL(group_sums, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, st, part, parts, n, parts, out);
    return;
  }
  const int64_t G = isqrt_ceil(parts), groups = (parts + G - 1) / G;
  hipLaunchKernelGGL(group_sums, dim3(grid_for(groups * n, kBlock)), dim3(kBlock), 0, st, part, parts, n, G, tmp);
  hipLaunchKernelGGL(group_sums, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, st, (const float*)tmp, groups, n,
                     groups, out);
}

inline int64_t pad_batch(int64_t B) { return (B + kRowsPerBlock - 1) / kRowsPerBlock * kRowsPerBlock; }

// batch chunk of one weight-gradient partial: at least 256 rows, and about
// 128 chunks so that the two 64-row output blocks x chunks fill the chip
inline int64_t grad_chunk(int64_t Bp) {
  int64_t c = (Bp + 127) / 128;
  c = (c + 31) / 32 * 32;
  return c < 256 ? 256 : c;
}

struct Ws {
  u16 *xb, *xbT, *a[3], *aT[3], *dyb, *dyT, *dz[2], *dzT[2];
  float *z[3], *wpart, *bpart, *tree;
  double* red;
};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// layout of the workspace for a batch of B samples (train: with everything
// the backward pass reads)
size_t carve(void* base, int64_t B, bool train, Ws* w) {
  const int64_t Bp = pad_batch(B);
  const int64_t chunks = (Bp + grad_chunk(Bp) - 1) / grad_chunk(Bp);
  char* p = reinterpret_cast<char*>(base);
  size_t at = 0;
  auto take = [&](size_t bytes) -> void* {
    void* r = p ? p + at : nullptr;
    at += align256(bytes);
    return r;
  };
  Ws t{};
  t.xb = (u16*)take(2 * (size_t)Bp * kK1);
  for (int l = 0; l < 3; ++l) t.a[l] = (u16*)take(2 * (size_t)Bp * kW);
  t.red = (double*)take(8 * ((size_t)(Bp * kOut + kBlock - 1) / kBlock + 8));
  if (train) {
    t.xbT = (u16*)take(2 * (size_t)Bp * 8);
    for (int l = 0; l < 3; ++l) t.aT[l] = (u16*)take(2 * (size_t)Bp * kW);
    for (int l = 0; l < 3; ++l) t.z[l] = (float*)take(4 * (size_t)Bp * kW);
    t.dyb = (u16*)take(2 * (size_t)Bp * kK1);
    t.dyT = (u16*)take(2 * (size_t)Bp * 8);
    for (int s = 0; s < 2; ++s) {
      t.dz[s] = (u16*)take(2 * (size_t)Bp * kW);
      t.dzT[s] = (u16*)take(2 * (size_t)Bp * kW);
    }
    t.wpart = (float*)take(4 * (size_t)chunks * kW * kW);
    t.bpart = (float*)take(4 * (size_t)(Bp / kRowsPerBlock) * kW);
    // first-round group sums: at most ceil(sqrt(parts)) + 1 rows of any reduction
    const int64_t rows = std::max(isqrt_ceil(chunks) * kW * kW, isqrt_ceil(Bp / kRowsPerBlock) * kW);
    t.tree = (float*)take(4 * (size_t)(rows + kW * kW));
  }
  if (w) *w = t;
  return at;
}

constexpr int64_t kMaxBatch = int64_t(1) << 26;  // 67M samples (int32-safe grids)

template <int NT, int EPI>
void launch_gemm(hipStream_t st, int64_t M, int N, int64_t K, int64_t kc, const u16* A, int64_t lda, const u16* Bt,
                 int64_t ldb, const EpiArgs& e) {
  const int64_t chunks = (K + kc - 1) / kc;
  dim3 grid((unsigned)((M + kRowsPerBlock - 1) / kRowsPerBlock), (unsigned)((N + 16 * NT - 1) / (16 * NT)),
            (unsigned)chunks);
  hipLaunchKernelGGL((gemm_tn<NT, EPI>), grid, dim3(kBlock), 0, st, M, N, K, kc, A, lda, Bt, ldb, e);
}

// dW [M][N] (row-major, into grad) = A^T-form product over the padded batch,
// chunked into partials and added in a fixed order
void weight_grad(hipStream_t st, const Ws& w, int64_t Bp, int M, int N, const u16* A, const u16* Bt, float* out) {
  const int64_t kc = grad_chunk(Bp), chunks = (Bp + kc - 1) / kc;
  EpiArgs e{};
  e.C = w.wpart;
  e.ldc = N;
  if (N > 16)
    launch_gemm<8, kPartial>(st, M, N, Bp, kc, A, Bp, Bt, Bp, e);
  else
    launch_gemm<1, kPartial>(st, M, N, Bp, kc, A, Bp, Bt, Bp, e);
  reduce_parts(st, w.wpart, chunks, (int64_t)M * N, out, w.tree);
}

bool shape_ok(const mpf_mlp_desc* d) {
  return d && d->in_dim == kIn && d->width == kW && d->depth == 4 && d->out_dim == kOut;
}

}  // namespace
}  // namespace mpf

using namespace mpf;

extern "C" int64_t mpf_mlp_param_count(const mpf_mlp_desc* d) { return shape_ok(d) ? kParams : -1; }
extern "C" int64_t mpf_mlp_packed_count(const mpf_mlp_desc* d) { return shape_ok(d) ? kPacked : -1; }

extern "C" size_t mpf_mlp_workspace(const mpf_mlp_desc* d, int64_t batch, int train) {
  if (!shape_ok(d) || batch < 1 || batch > kMaxBatch) return 0;
  return carve(nullptr, batch, train != 0, nullptr);
}

extern "C" int mpf_mlp_pack(const mpf_mlp_desc* d, const float* master, void* packed, void* stream) {
  if (!shape_ok(d)) return MPF_ERR_UNSUPPORTED;
  if (!master || !packed) return MPF_ERR_ARG;
  hipLaunchKernelGGL(pack_params, dim3(grid_for(kPacked, kBlock)), dim3(kBlock), 0, as_stream(stream), master,
                     (u16*)packed);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

extern "C" int mpf_mlp_forward(const mpf_mlp_desc* d, const float* master, const void* packed, const float* x,
                               const int64_t* rows, float* y, int64_t B, int train, void* ws, size_t ws_bytes,
                               void* stream) {
  if (!shape_ok(d)) return MPF_ERR_UNSUPPORTED;
  if (!master || !packed || !x || !y || B < 1 || B > kMaxBatch) return MPF_ERR_ARG;
  if (!ws || ws_bytes < mpf_mlp_workspace(d, B, train)) return MPF_ERR_WORKSPACE;
  hipStream_t st = as_stream(stream);
  Ws w;
  carve(ws, B, train != 0, &w);
  const int64_t Bp = pad_batch(B);
  const u16* P = (const u16*)packed;
  hipLaunchKernelGGL(pack_inputs, dim3(grid_for(Bp, kBlock)), dim3(kBlock), 0, st, B, Bp, x, rows, w.xb,
                     train ? w.xbT : nullptr);
  const u16* in = w.xb;
  int64_t lda = kK1;
  const int pw[3] = {pW1, pW2, pW3}, ob[3] = {ob1, ob2, ob3};
  for (int l = 0; l < 3; ++l) {
    EpiArgs e{};
    e.Z = train ? w.z[l] : nullptr;
    e.act = w.a[l];
    e.actT = train ? w.aT[l] : nullptr;
    e.ldT = Bp;
    e.bias = master + ob[l];
    launch_gemm<8, kHiddenFwd>(st, Bp, kW, lda, lda, in, lda, P + pw[l], lda, e);
    in = w.a[l];
    lda = kW;
  }
  EpiArgs e{};
  e.bias = master + ob4;
  e.y = y;
  e.rows_valid = B;
  launch_gemm<1, kOutFwd>(st, Bp, kOut, kW, kW, in, kW, P + pW4, kW, e);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

extern "C" int mpf_mlp_backward(const mpf_mlp_desc* d, const void* packed, const float* dy, float* grad, int64_t B,
                                void* ws, size_t ws_bytes, void* stream) {
  if (!shape_ok(d)) return MPF_ERR_UNSUPPORTED;
  if (!packed || !dy || !grad || B < 1 || B > kMaxBatch) return MPF_ERR_ARG;
  if (!ws || ws_bytes < mpf_mlp_workspace(d, B, 1)) return MPF_ERR_WORKSPACE;
  hipStream_t st = as_stream(stream);
  Ws w;
  carve(ws, B, true, &w);
  const int64_t Bp = pad_batch(B);
  const int64_t nblk = Bp / kRowsPerBlock;
  const u16* P = (const u16*)packed;
  const unsigned gdy = grid_for(Bp, kBlock);
  hipLaunchKernelGGL(pack_dy, dim3(gdy), dim3(kBlock), 0, st, B, Bp, dy, w.dyb, w.dyT, w.bpart);
  reduce_parts(st, w.bpart, gdy, kOut, grad + ob4, w.tree);
  // layer 4: dW4 = dy^T a3
  weight_grad(st, w, Bp, kOut, kW, w.dyT, w.aT[2], grad + oW4);
  // down through the hidden layers: dZ_l = (dZ_{l+1} W_{l+1}) * silu'(Z_l)
  const u16* dz_in = w.dyb;
  int64_t k_in = kK1;
  const u16* wt[3] = {P + pW2t, P + pW3t, P + pW4t};  // W_{l+1}^T for l = 0, 1, 2
  const int ow[3] = {oW1, oW2, oW3}, ob[3] = {ob1, ob2, ob3};
  for (int l = 2; l >= 0; --l) {
    const int s = l & 1;
    EpiArgs e{};
    e.Z = w.z[l];
    e.act = w.dz[s];
    e.actT = w.dzT[s];
    e.ldT = Bp;
    e.colpart = w.bpart;
    launch_gemm<8, kHiddenBwd>(st, Bp, kW, k_in, k_in, dz_in, k_in, wt[l], k_in, e);
    reduce_parts(st, w.bpart, nblk, kW, grad + ob[l], w.tree);
    if (l > 0)
      weight_grad(st, w, Bp, kW, kW, w.dzT[s], w.aT[l - 1], grad + ow[l]);
    else
      weight_grad(st, w, Bp, kW, kIn, w.dzT[s], w.xbT, grad + ow[0]);
    dz_in = w.dz[s];
    k_in = kW;
  }
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

extern "C" int mpf_mlp_mse(int64_t B, const float* y, const float* t, const int64_t* rows, float* dy, double* loss,
                           void* ws, size_t ws_bytes, void* stream) {
  if (!y || !t || !dy || !loss || B < 1 || B > kMaxBatch) return MPF_ERR_ARG;
  const int64_t n = B * kOut;
  const unsigned g = grid_for(n, kBlock);
  if (!ws || ws_bytes < mpf_reduce_workspace(n)) return MPF_ERR_WORKSPACE;
  hipStream_t st = as_stream(stream);
  double* part = reinterpret_cast<double*>(ws);
  hipLaunchKernelGGL(mse_partial, dim3(g), dim3(kBlock), 0, st, B, y, t, rows, dy, part);
  hipLaunchKernelGGL(finish_sum, dim3(1), dim3(kBlock), 0, st, (const double*)part, (int64_t)g, 1, 1.0 / (double)n,
                     loss);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

extern "C" int mpf_adam_step(int64_t n, float* p, const float* g, float* m, float* v, int step, float lr, float b1,
                             float b2, float eps, void* stream) {
  if (!p || !g || !m || !v || n < 1 || step < 1 || !(lr > 0.f) || !(b1 >= 0.f && b1 < 1.f) ||
      !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f))
    return MPF_ERR_ARG;
  const float c1 = (float)(1.0 - pow((double)b1, step)), c2 = (float)(1.0 - pow((double)b2, step));
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, as_stream(stream), n, p, g, m, v, lr,
                     b1, b2, eps, c1, c2);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

extern "C" int mpf_mlp_features(int64_t n, const double* pos, double r, double phi, float* x, void* stream) {
  if (!pos || !x || n < 1 || !(r >= 0.0)) return MPF_ERR_ARG;
  hipLaunchKernelGGL(features_kernel, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, as_stream(stream), n, pos, r, phi,
                     x);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

extern "C" int mpf_mlp_to_state(int64_t n, int64_t n_int, const float* y, double U, double P, int precision, void* v,
                                void* p, double* vmax, void* ws, size_t ws_bytes, void* stream) {
  if (!y || !v || !p || n < 1 || n_int < 0 || n_int > n) return MPF_ERR_ARG;
  if (!precision_ok(precision)) return MPF_ERR_ARG;
  if (!ws || ws_bytes < mpf_reduce_workspace(n)) return MPF_ERR_WORKSPACE;
  hipStream_t st = as_stream(stream);
  const unsigned g = grid_for(n, kBlock);
  double* part = reinterpret_cast<double*>(ws);
  double* mean = part + g;
  hipLaunchKernelGGL(psum_partial, dim3(g), dim3(kBlock), 0, st, n, y, P, part);
  hipLaunchKernelGGL(finish_sum, dim3(1), dim3(kBlock), 0, st, (const double*)part, (int64_t)g, 1, 1.0 / (double)n,
                     mean);
  if (vmax) hipLaunchKernelGGL(zero_double, dim3(1), dim3(1), 0, st, vmax);
  if (state_is_f32(precision))
    hipLaunchKernelGGL(to_state_kernel<float>, dim3(g), dim3(kBlock), 0, st, n, n_int, y, U, P, (const double*)mean,
                       (float*)v, (float*)p, vmax);
  else
    hipLaunchKernelGGL(to_state_kernel<double>, dim3(g), dim3(kBlock), 0, st, n, n_int, y, U, P, (const double*)mean,
                       (double*)v, (double*)p, vmax);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

extern "C" int mpf_gemm_bf16(int64_t M, int N, int64_t K, const void* A, int64_t lda, const void* Bt, int64_t ldb,
                             float* C, int64_t ldc, void* stream) {
  if (!A || !Bt || !C || M < 1 || N < 1 || K < 32 || K % 32 || lda < K || ldb < K || ldc < N || lda % 8 || ldb % 8)
    return MPF_ERR_ARG;
  if ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(Bt)) & 15) return MPF_ERR_ARG;
  EpiArgs e{};
  e.C = C;
  e.ldc = ldc;
  hipStream_t st = as_stream(stream);
  if (N > 16)
    launch_gemm<8, kPartial>(st, M, N, K, K, (const u16*)A, lda, (const u16*)Bt, ldb, e);
  else
    launch_gemm<1, kPartial>(st, M, N, K, K, (const u16*)A, lda, (const u16*)Bt, ldb, e);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

// Fused loop of training steps: everything a step launches, for n_batches
// consecutive minibatches, from one host call (a step is about 25 launches;
// issued from Python they cost more host time than the device needs for a
// 64k-sample batch).  Layout of ws: the training workspace of B, then y, dy
// [B][4] float, the loss, and the MSE partials.
static size_t train_extra(int64_t B) {
  const size_t yb = align256(4 * (size_t)B * kOut);
  return 2 * yb + 256 + align256(mpf_reduce_workspace(B * kOut));
}

extern "C" size_t mpf_mlp_train_workspace(const mpf_mlp_desc* d, int64_t B) {
  const size_t base = mpf_mlp_workspace(d, B, 1);
  return base ? base + train_extra(B) : 0;
}

extern "C" int mpf_mlp_train(const mpf_mlp_desc* d, float* master, void* packed, float* m, float* v, float* grad,
                             const float* x, const float* t, const int64_t* rows, int64_t n_batches, int64_t B,
                             int step0, float lr0, float lr_ratio, float b1, float b2, float eps, double* loss_sum,
                             void* ws, size_t ws_bytes, void* stream) {
  if (!shape_ok(d)) return MPF_ERR_UNSUPPORTED;
  if (!master || !packed || !m || !v || !grad || !x || !t || !rows || !loss_sum || n_batches < 1 || B < 1 ||
      B > kMaxBatch || step0 < 0 || !(lr0 > 0.f) || !(lr_ratio > 0.f))
    return MPF_ERR_ARG;
  if (!ws || ws_bytes < mpf_mlp_train_workspace(d, B)) return MPF_ERR_WORKSPACE;
  hipStream_t st = as_stream(stream);
  const size_t base = mpf_mlp_workspace(d, B, 1);
  char* extra = reinterpret_cast<char*>(ws) + base;
  const size_t yb = align256(4 * (size_t)B * kOut);
  float* y = reinterpret_cast<float*>(extra);
  float* dy = reinterpret_cast<float*>(extra + yb);
  double* loss = reinterpret_cast<double*>(extra + 2 * yb);
  void* red = extra + 2 * yb + 256;
  const size_t red_bytes = ws_bytes - base - 2 * yb - 256;
  hipLaunchKernelGGL(zero_double, dim3(1), dim3(1), 0, st, loss_sum);
  double lr = lr0;
  for (int64_t i = 0; i < n_batches; ++i) {
    const int64_t* r = rows + i * B;
    int rc = mpf_mlp_forward(d, master, packed, x, r, y, B, 1, ws, base, stream);
    if (!rc) rc = mpf_mlp_mse(B, y, t, r, dy, loss, red, red_bytes, stream);
    if (rc) return rc;
    hipLaunchKernelGGL(add_double, dim3(1), dim3(1), 0, st, (const double*)loss, loss_sum);
    rc = mpf_mlp_backward(d, packed, dy, grad, B, ws, base, stream);
    if (!rc) rc = mpf_adam_step(kParams, master, grad, m, v, (int)(step0 + i + 1), (float)lr, b1, b2, eps, stream);
    if (!rc) rc = mpf_mlp_pack(d, master, packed, stream);
    if (rc) return rc;
    lr *= lr_ratio;
  }
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

extern "C" int mpf_shuffle_rows(int64_t n, int64_t count, uint64_t seed, int64_t* rows, void* stream) {
  if (!rows || n < 1 || count < 0 || count > n || n > (int64_t(1) << 60)) return MPF_ERR_ARG;
  if (count == 0) return MPF_OK;
  int bits = 1;
  while ((int64_t(1) << bits) < n) ++bits;
  const int h = (bits + 1) / 2;
  hipLaunchKernelGGL(shuffle_kernel, dim3(grid_for(count, kBlock)), dim3(kBlock), 0, as_stream(stream), n, count, h,
                     (unsigned long long)seed, rows);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}
