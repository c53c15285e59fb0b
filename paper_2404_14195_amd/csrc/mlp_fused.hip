// Fused training step of the warm-start network on gfx950: forward, loss,
// backward and the weight gradients of 64-row tiles in one persistent kernel,
// activations staying in LDS and the weight-gradient sums in registers.
//
// Network and parameter layout as in mlp.hip (5 -> 128 -> 128 -> 128 -> 4,
// SiLU, master vector W_1, b_1, ..., W_4, b_4 with W [out][in], packed BF16
// copy with W and W^T).  Products are v_mfma_f32_16x16x32_bf16 (BF16
// operands, FP32 accumulation).  The forward pass keeps, per pre-activation z,
// the derivative of SiLU, sigma(z) (1 + z (1 - sigma(z))), in registers as
// FP16 (two per register; it lies in [-0.1, 1.1], where FP16 resolves
// 2^-11); the backward pass multiplies the propagated error by it and rounds
// the product to BF16 for the next products, as the layered kernels do.
//
// A block is four waves and works on tiles of 64 rows of the minibatch, one
// tile after another (tile = block, block + grid, ...).  For every product
// that produces activations the waves split the output columns (wave w owns
// columns 32w .. 32w + 31 of each 128-wide layer, all 64 rows), so each
// weight fragment is read from the caches once per block and tile, and a
// wave's pre-activations and back-propagated errors cover the same columns
// forward and backward.  For the weight gradients dW_l = dZ_l^T A_{l-1} the
// waves split the output features (rows of dW_l) and accumulate over the
// tiles in registers.  Activations are written to LDS in both orders:
// row-major [row][feature] feeds the next layer's product, feature-major
// [feature][row] feeds the weight gradients, whose reduction index is the
// row.  At the end each block writes its gradient sums (all 34,308
// parameters) and its loss sum; a second kernel adds the blocks' partials in
// a fixed order, so a step is bitwise reproducible for a given grid.
#include "common.hpp"

namespace mpf {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int kIn = 5, kW = 128, kOut = 4;
constexpr int kParams = kW * kIn + kW + 2 * (kW * kW + kW) + kOut * kW + kOut;
constexpr int oW1 = 0, ob1 = oW1 + kW * kIn, oW2 = ob1 + kW, ob2 = oW2 + kW * kW, oW3 = ob2 + kW,
              ob3 = oW3 + kW * kW, oW4 = ob3 + kW, ob4 = oW4 + kOut * kW;
constexpr int kK1 = 32;
constexpr int pW1 = 0, pW2 = pW1 + kW * kK1, pW2t = pW2 + kW * kW, pW3 = pW2t + kW * kW, pW3t = pW3 + kW * kW,
              pW4 = pW3t + kW * kW, pW4t = pW4 + 16 * kW;

constexpr int kRows = 64;          // rows of a tile
constexpr int kThreads = 256;      // four waves
constexpr int LDR = kW + 8;        // row-major 128-wide buffers (padded against bank conflicts)
constexpr int LDX = kK1 + 8;       // row-major 32-wide buffers
constexpr int LDT = kRows + 8;     // feature-major buffers [feature][64 rows]

__device__ __forceinline__ u16 to_bf16(float f) {  // round to nearest, ties to even
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (u16)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}

__device__ __forceinline__ float sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }

__device__ __forceinline__ bf16x8 frag(const u16* p) { return *reinterpret_cast<const bf16x8*>(p); }

__device__ __forceinline__ f4 mfma(const bf16x8& a, const bf16x8& b, const f4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

struct FusedArgs {
  const float* master;
  const u16* packed;
  const float* x;       // [rows][5]
  const float* t;       // [rows][4]
  const int64_t* rows;  // [B] or null
  int64_t B;
  int64_t n_tiles;
  float dy_scale;  // 2 / (4 B)
  float* part;     // [gridDim][kParams]
  double* lpart;   // [gridDim]
};

// The wave's product over 64 rows x its 32 columns: acc[mt][j] for m-tile mt
// (rows 16 mt ..) and column tile j (columns 32 w + 16 j ..), reduction over
// k in [0, K) with A row-major in LDS (leading dimension lda) and Bt [n][k]
// row-major in global memory (leading dimension ldb).
template <int K>
__device__ __forceinline__ void wave_cols(f4 (&acc)[4][2], const u16* __restrict__ A, int lda,
                                          const u16* __restrict__ Bt, int ldb, int w, int r, int g) {
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[mt][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
  for (int k0 = 0; k0 < K; k0 += 32) {
    bf16x8 b[2], a[4];
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = frag(Bt + (int64_t)(32 * w + 16 * j + r) * ldb + k0 + 8 * g);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) a[mt] = frag(A + (16 * mt + r) * lda + k0 + 8 * g);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[mt][j] = mfma(a[mt], b[j], acc[mt][j]);
  }
}

// Activation tile of the wave (pre-activation z, value h) into LDS in both
// orders; column n = 32 w + 16 j + r, rows 16 mt + 4 g + i.
__device__ __forceinline__ void store_both(const float (&h)[4][2][4], u16* __restrict__ R, u16* __restrict__ T,
                                           int w, int r, int g) {
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = 32 * w + 16 * j + r;
      u16 q[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        q[i] = to_bf16(h[mt][j][i]);
        if (R) R[(16 * mt + 4 * g + i) * LDR + n] = q[i];
      }
      uint2 pk;
      pk.x = (unsigned)q[0] | ((unsigned)q[1] << 16);
      pk.y = (unsigned)q[2] | ((unsigned)q[3] << 16);
      *reinterpret_cast<uint2*>(T + n * LDT + 16 * mt + 4 * g) = pk;
    }
}

// dW[o][in] += sum over the tile's rows of dZ^T[o][row] X^T[in][row]: the
// wave's output rows o = 32 w + 16 mt + ..., NT column tiles, A = dZ^T and
// Bt = X^T feature-major in LDS.
template <int NT>
__device__ __forceinline__ void wave_wgrad(f4 (&acc)[2][NT], const u16* __restrict__ AT,
                                           const u16* __restrict__ BT, int w, int r, int g) {
#pragma unroll 1
  for (int k0 = 0; k0 < kRows; k0 += 32) {
    bf16x8 a[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) a[mt] = frag(AT + (32 * w + 16 * mt + r) * LDT + k0 + 8 * g);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const bf16x8 b = frag(BT + (16 * nt + r) * LDT + k0 + 8 * g);
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) acc[mt][nt] = mfma(a[mt], b, acc[mt][nt]);
    }
  }
}

typedef _Float16 h2 __attribute__((ext_vector_type(2)));

// SiLU of the wave's pre-activations acc + bias: values into h, derivatives
// into sp (FP16 pairs: rows 4 g + 2 p, 4 g + 2 p + 1).
__device__ __forceinline__ void silu_fwd(const f4 (&acc)[4][2], const float* __restrict__ bias, float (&h)[4][2][4],
                                         h2 (&sp)[4][2][2], int w, int r) {
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const float b = bias[32 * w + 16 * j + r];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        float d[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const float z = acc[mt][j][2 * q + e] + b;
          const float sg = sigmoid(z);
          h[mt][j][2 * q + e] = z * sg;
          d[e] = sg * (1.0f + z * (1.0f - sg));
        }
        sp[mt][j][q] = h2{(_Float16)d[0], (_Float16)d[1]};
      }
  }
}

// dZ = dA * silu'(Z) from the accumulators; per-lane column sums of dZ into
// cs[j] (bias gradient); the result to LDS in both orders (R may be null).
__device__ __forceinline__ void backprop_silu(const f4 (&acc)[4][2], const h2 (&sp)[4][2][2], float (&cs)[2],
                                              u16* __restrict__ R, u16* __restrict__ T, int w, int r, int g) {
  float d[4][2][4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        d[mt][j][i] = acc[mt][j][i] * (float)sp[mt][j][i >> 1][i & 1];
        cs[j] += d[mt][j][i];
      }
  store_both(d, R, T, w, r, g);
}

__global__ __launch_bounds__(kThreads, 1) void mlp_fused_step(FusedArgs a) {
  __shared__ __align__(16) u16 s_xr[kRows * LDX];   // X [row][32]
  __shared__ __align__(16) u16 s_xt[kK1 * LDT];     // X^T [32][row]
  __shared__ __align__(16) u16 s_r0[kRows * LDR];   // H1, H3, then dZ2 (row-major)
  __shared__ __align__(16) u16 s_r1[kRows * LDR];   // H2, then dZ3
  __shared__ __align__(16) u16 s_t1[kW * LDT];      // H1^T
  __shared__ __align__(16) u16 s_t2[kW * LDT];      // H2^T
  __shared__ __align__(16) u16 s_t3[kW * LDT];      // H3^T
  __shared__ __align__(16) u16 s_dzt[kW * LDT];     // dZ^T of the current layer
  __shared__ __align__(16) u16 s_dyr[kRows * LDX];  // dL/dy [row][32] (columns >= 4 zero)
  __shared__ __align__(16) u16 s_dyt[16 * LDT];     // dL/dy^T [16][row] (rows >= 4 zero)
  __shared__ float s_red[4][kW];
  __shared__ double s_loss[kThreads / 64];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const u16* P = a.packed;
  const float* M = a.master;

  // gradient sums of this block (registers, all tiles)
  f4 gW1[2][2], gW2[2][8], gW3[2][8], gW4[2];
  float cs1[2] = {0.f, 0.f}, cs2[2] = {0.f, 0.f}, cs3[2] = {0.f, 0.f}, cs4 = 0.f;
  double loss = 0.0;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    gW4[i] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 2; ++j) gW1[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 8; ++j) gW2[i][j] = gW3[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  }
  // padding columns of X and dL/dy stay zero for every tile
  for (int e = tid; e < kRows * LDX; e += kThreads) s_xr[e] = s_dyr[e] = 0;
  for (int e = tid; e < kK1 * LDT; e += kThreads) s_xt[e] = 0;
  for (int e = tid; e < 16 * LDT; e += kThreads) s_dyt[e] = 0;
  __syncthreads();

  for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
    const int64_t base = tile * kRows;
    // ---- inputs: rows beyond the batch are zero
    if (tid < kRows) {
      const int64_t b = base + tid;
      const bool live = b < a.B;
      const int64_t src = live ? (a.rows ? a.rows[b] : b) : 0;
#pragma unroll
      for (int f = 0; f < kIn; ++f) {
        const u16 h = live ? to_bf16(a.x[src * kIn + f]) : (u16)0;
        s_xr[tid * LDX + f] = h;
        s_xt[f * LDT + tid] = h;
      }
    }
    __syncthreads();
    h2 sp1[4][2][2], sp2[4][2][2], sp3[4][2][2];
    f4 acc[4][2];
    // ---- forward: three hidden layers
    {
      float h[4][2][4];
      wave_cols<kK1>(acc, s_xr, LDX, P + pW1, kK1, w, r, g);
      silu_fwd(acc, M + ob1, h, sp1, w, r);
      store_both(h, s_r0, s_t1, w, r, g);
      __syncthreads();
      wave_cols<kW>(acc, s_r0, LDR, P + pW2, kW, w, r, g);
      silu_fwd(acc, M + ob2, h, sp2, w, r);
      store_both(h, s_r1, s_t2, w, r, g);
      __syncthreads();
      wave_cols<kW>(acc, s_r1, LDR, P + pW3, kW, w, r, g);
      silu_fwd(acc, M + ob3, h, sp3, w, r);
      store_both(h, s_r0, s_t3, w, r, g);
      __syncthreads();
    }
    // ---- output layer and loss: wave w takes rows 16 w .. 16 w + 15
    {
      f4 y = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k0 = 0; k0 < kW; k0 += 32)
        y = mfma(frag(s_r0 + (16 * w + r) * LDR + k0 + 8 * g), frag(P + pW4 + r * kW + k0 + 8 * g), y);
      // lane: column r (output r < 4), rows 16 w + 4 g + i
      const float b4 = r < kOut ? M[ob4 + r] : 0.f;
      u16 q[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * w + 4 * g + i;
        const int64_t bb = base + row;
        float dy = 0.f;
        if (r < kOut && bb < a.B) {
          const int64_t src = a.rows ? a.rows[bb] : bb;
          const float d = y[i] + b4 - a.t[src * kOut + r];
          loss += (double)d * (double)d;
          dy = d * a.dy_scale;
        }
        cs4 += dy;
        q[i] = to_bf16(dy);
        if (r < 16) s_dyr[row * LDX + r] = q[i];
      }
      uint2 pk;
      pk.x = (unsigned)q[0] | ((unsigned)q[1] << 16);
      pk.y = (unsigned)q[2] | ((unsigned)q[3] << 16);
      *reinterpret_cast<uint2*>(s_dyt + r * LDT + 16 * w + 4 * g) = pk;
    }
    __syncthreads();
    // ---- layer 3: dZ3 = (dy W4) * silu'(Z3); dW4 += dy^T H3
    wave_cols<kK1>(acc, s_dyr, LDX, P + pW4t, kK1, w, r, g);
    backprop_silu(acc, sp3, cs3, s_r1, s_dzt, w, r, g);
    {
#pragma unroll
      for (int k0 = 0; k0 < kRows; k0 += 32) {
        const bf16x8 aa = frag(s_dyt + r * LDT + k0 + 8 * g);
#pragma unroll
        for (int j = 0; j < 2; ++j) gW4[j] = mfma(aa, frag(s_t3 + (32 * w + 16 * j + r) * LDT + k0 + 8 * g), gW4[j]);
      }
    }
    __syncthreads();
    // ---- layer 2: dW3 += dZ3^T H2; dZ2 = (dZ3 W3) * silu'(Z2)
    wave_wgrad<8>(gW3, s_dzt, s_t2, w, r, g);
    wave_cols<kW>(acc, s_r1, LDR, P + pW3t, kW, w, r, g);
    __syncthreads();  // dZ3 is consumed; its buffers take dZ2
    backprop_silu(acc, sp2, cs2, s_r0, s_dzt, w, r, g);
    __syncthreads();
    // ---- layer 1: dW2 += dZ2^T H1; dZ1 = (dZ2 W2) * silu'(Z1); dW1 += dZ1^T X
    wave_wgrad<8>(gW2, s_dzt, s_t1, w, r, g);
    wave_cols<kW>(acc, s_r0, LDR, P + pW2t, kW, w, r, g);
    __syncthreads();
    backprop_silu(acc, sp1, cs1, nullptr, s_dzt, w, r, g);
    __syncthreads();
    wave_wgrad<2>(gW1, s_dzt, s_xt, w, r, g);
    __syncthreads();  // the next tile overwrites every buffer
  }

  // ---- this block's partial gradient, in the master layout
  float* out = a.part + (int64_t)blockIdx.x * kParams;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = 32 * w + 16 * mt + 4 * g + i;
#pragma unroll
      for (int nt = 0; nt < 8; ++nt) {
        out[oW2 + o * kW + 16 * nt + r] = gW2[mt][nt][i];
        out[oW3 + o * kW + 16 * nt + r] = gW3[mt][nt][i];
      }
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
        if (16 * nt + r < kIn) out[oW1 + o * kIn + 16 * nt + r] = gW1[mt][nt][i];
    }
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = 4 * g + i;
      if (o < kOut) out[oW4 + o * kW + 32 * w + 16 * j + r] = gW4[j][i];
    }
  // bias sums: each lane holds column sums over its rows; add the four row
  // groups g (lanes r, r + 16, r + 32, r + 48)
  auto colsum = [&](float v) {
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
  };
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const float s1 = colsum(cs1[j]), s2 = colsum(cs2[j]), s3 = colsum(cs3[j]);
    if (g == 0) {
      out[ob1 + 32 * w + 16 * j + r] = s1;
      out[ob2 + 32 * w + 16 * j + r] = s2;
      out[ob3 + 32 * w + 16 * j + r] = s3;
    }
  }
  const float s4 = colsum(cs4);  // output column r over the wave's rows
  if (g == 0) s_red[w][r] = s4;
  // loss: FP64 over the block
  double l = loss;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
  if (lane == 0) s_loss[w] = l;
  __syncthreads();
  if (tid < kOut) out[ob4 + tid] = s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
  if (tid == 0) a.lpart[blockIdx.x] = s_loss[0] + s_loss[1] + s_loss[2] + s_loss[3];
}

// grad[p] = sum over blocks of part[blk][p], blocks in ascending order;
// loss = sum of the blocks' loss sums / (4 B)
__global__ void fused_reduce(const float* __restrict__ part, int nblk, float* __restrict__ grad,
                             const double* __restrict__ lpart, double inv_n, double* __restrict__ loss,
                             double* __restrict__ loss_sum) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < kParams) {
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * kParams + p];
    grad[p] = s;
  }
  if (p == 0) {
    double l = 0.0;
    for (int b = 0; b < nblk; ++b) l += lpart[b];
    l *= inv_n;
    if (loss) *loss = l;
    if (loss_sum) *loss_sum += l;
  }
}

__global__ void zero_d(double* x) { *x = 0.0; }

constexpr int64_t kMaxBatch = int64_t(1) << 26;

int grid_blocks(int64_t n_tiles) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
  }
  return (int)(n_tiles < cus ? n_tiles : cus);
}

bool shape_ok(const mpf_mlp_desc* d) {
  return d && d->in_dim == kIn && d->width == kW && d->depth == 4 && d->out_dim == kOut;
}

}  // namespace
}  // namespace mpf

using namespace mpf;

extern "C" size_t mpf_mlp_fused_workspace(const mpf_mlp_desc* d, int64_t B) {
  if (!shape_ok(d) || B < 1 || B > kMaxBatch) return 0;
  const int64_t tiles = (B + kRows - 1) / kRows;
  const int64_t nblk = tiles < 1024 ? tiles : 1024;  // more than any device's compute units
  return (size_t)nblk * (kParams * sizeof(float) + sizeof(double)) + 512;
}

extern "C" int mpf_mlp_grad_fused(const mpf_mlp_desc* d, const float* master, const void* packed, const float* x,
                                  const float* t, const int64_t* rows, int64_t B, float* grad, double* loss,
                                  void* ws, size_t ws_bytes, void* stream) {
  if (!shape_ok(d)) return MPF_ERR_UNSUPPORTED;
  if (!master || !packed || !x || !t || !grad || B < 1 || B > kMaxBatch) return MPF_ERR_ARG;
  if (!ws || ws_bytes < mpf_mlp_fused_workspace(d, B)) return MPF_ERR_WORKSPACE;
  hipStream_t st = as_stream(stream);
  const int64_t tiles = (B + kRows - 1) / kRows;
  const int nblk = grid_blocks(tiles);
  double* lpart = reinterpret_cast<double*>(ws);
  float* part = reinterpret_cast<float*>(reinterpret_cast<char*>(ws) + ((nblk * sizeof(double) + 255) / 256) * 256);
  FusedArgs fa{master, (const u16*)packed, x, t, rows, B, tiles, (float)(2.0 / (4.0 * (double)B)), part, lpart};
  hipLaunchKernelGGL(mlp_fused_step, dim3(nblk), dim3(kThreads), 0, st, fa);
  hipLaunchKernelGGL(fused_reduce, dim3((kParams + 255) / 256), dim3(256), 0, st, (const float*)part, nblk, grad,
                     (const double*)lpart, 1.0 / (4.0 * (double)B), loss, (double*)nullptr);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

extern "C" int mpf_mlp_train_fused(const mpf_mlp_desc* d, float* master, void* packed, float* m, float* v,
                                   float* grad, const float* x, const float* t, const int64_t* rows,
                                   int64_t n_batches, int64_t B, int step0, float lr0, float lr_ratio, float b1,
                                   float b2, float eps, double* loss_sum, void* ws, size_t ws_bytes, void* stream) {
  if (!shape_ok(d)) return MPF_ERR_UNSUPPORTED;
  if (!master || !packed || !m || !v || !grad || !x || !t || !rows || !loss_sum || n_batches < 1 || B < 1 ||
      B > kMaxBatch || step0 < 0 || !(lr0 > 0.f) || !(lr_ratio > 0.f))
    return MPF_ERR_ARG;
  if (!ws || ws_bytes < mpf_mlp_fused_workspace(d, B)) return MPF_ERR_WORKSPACE;
  hipStream_t st = as_stream(stream);
  const int64_t tiles = (B + kRows - 1) / kRows;
  const int nblk = grid_blocks(tiles);
  double* lpart = reinterpret_cast<double*>(ws);
  float* part = reinterpret_cast<float*>(reinterpret_cast<char*>(ws) + ((nblk * sizeof(double) + 255) / 256) * 256);
  hipLaunchKernelGGL(zero_d, dim3(1), dim3(1), 0, st, loss_sum);
  double lr = lr0;
  for (int64_t i = 0; i < n_batches; ++i) {
    FusedArgs fa{master, (const u16*)packed, x, t, rows + i * B, B, tiles, (float)(2.0 / (4.0 * (double)B)), part,
                 lpart};
    hipLaunchKernelGGL(mlp_fused_step, dim3(nblk), dim3(kThreads), 0, st, fa);
    hipLaunchKernelGGL(fused_reduce, dim3((kParams + 255) / 256), dim3(256), 0, st, (const float*)part, nblk, grad,
                       (const double*)lpart, 1.0 / (4.0 * (double)B), (double*)nullptr, loss_sum);
    int rc = mpf_adam_step(kParams, master, grad, m, v, (int)(step0 + i + 1), (float)lr, b1, b2, eps, stream);
    if (!rc) rc = mpf_mlp_pack(d, master, packed, stream);
    if (rc) return rc;
    lr *= lr_ratio;
  }
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}
