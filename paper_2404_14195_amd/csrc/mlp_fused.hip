// Fused training step of the warm-start network on gfx950: forward, loss,
// backward and the weight gradients of 64-row tiles in one persistent kernel,
// activations staying in LDS, the weights and the weight-gradient sums in
// registers.
//
// Network and parameter layout as in mlp.hip (5 -> 128 -> 128 -> 128 -> 4,
// SiLU, master vector W_1, b_1, ..., W_4, b_4 with W [out][in], packed BF16
// copy with W and W^T).  Products are v_mfma_f32_16x16x32_bf16 (BF16
// operands, FP32 accumulation).  The forward pass keeps, per pre-activation z,
// the derivative of SiLU, sigma(z) (1 + z (1 - sigma(z))), in registers as
// FP16 (two per register; it lies in [-0.1, 1.1], where FP16 resolves
// 2^-11); the backward pass multiplies the propagated error by it and rounds
// the product to BF16 for the next products, as the layered kernels do.
// sigma is evaluated with the hardware base-2 exponential and reciprocal
// (about 1 ulp each, far below the BF16 rounding of every operand).
//
// A block is eight waves, one block per compute unit (activations and the
// small weights take 150 KB of LDS), so each SIMD runs two waves that hide
// each other's LDS and MFMA latencies.  The block works on tiles of 64 rows
// of the minibatch, one tile after another (tile = block, block + grid, ...).
// For every product that produces activations the waves split the output
// columns (wave w owns columns 16w .. 16w + 15 of each 128-wide layer, all 64
// rows), so a wave needs only its 16 rows of each weight matrix: it keeps its
// fragments of the two 128 x 128 forward products in registers (32 registers,
// loaded once), loads those of the two backward products (W^T) into a third
// set one phase before their use (they come from the L2 cache, which all
// blocks share), and the three small matrices (W_1, W_4, W_4^T) sit in LDS.
// A wave's pre-activations and back-propagated errors cover the same columns
// forward and backward.  For the weight gradients dW_l = dZ_l^T A_{l-1} the
// waves split the output features (rows of dW_l) the same way and accumulate
// over the tiles in registers (dW_2, dW_3) or in LDS (the small dW_1, dW_4).
// Activations are written to LDS in both orders: row-major [row][feature]
// feeds the next layer's product, feature-major [feature][row] feeds the
// weight gradients, whose reduction index is the row.  The next tile's inputs
// and targets are loaded while the current tile is computed.  At the end
// each block writes its gradient sums (all 34,308 parameters) and its loss
// sum; a second kernel adds the blocks' partials in a fixed order (and, in
// the training loop, applies the Adam update and refreshes the BF16 copy), so
// a step is bitwise reproducible for a given grid.
#include "common.hpp"

namespace mpf {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int kIn = 5, kW = 128, kOut = 4;
constexpr int kParams = kW * kIn + kW + 2 * (kW * kW + kW) + kOut * kW + kOut;
constexpr int oW1 = 0, ob1 = oW1 + kW * kIn, oW2 = ob1 + kW, ob2 = oW2 + kW * kW, oW3 = ob2 + kW,
              ob3 = oW3 + kW * kW, oW4 = ob3 + kW, ob4 = oW4 + kOut * kW;
constexpr int kK1 = 32;
constexpr int pW1 = 0, pW2 = pW1 + kW * kK1, pW2t = pW2 + kW * kW, pW3 = pW2t + kW * kW, pW3t = pW3 + kW * kW,
              pW4 = pW3t + kW * kW, pW4t = pW4 + 16 * kW;

constexpr int kRows = 64;              // rows of a tile
constexpr int kWaves = 8;              // waves per block
constexpr int kThreads = kWaves * 64;  // 512
constexpr int LDR = kW + 8;            // row-major 128-wide buffers (padded against bank conflicts)
constexpr int LDX = kK1 + 8;           // row-major 32-wide buffers
constexpr int LDT = kRows + 8;         // feature-major buffers [feature][64 rows]
constexpr int LDW4 = kW + 8;           // W4's rows in LDS (padded like the activations)

// W1 and W4^T ([128][32]) sit in LDS unpadded, each row's four 16-byte
// pieces rotated by (row / 4) mod 4, so that the 16 rows of a fragment read
// cover all 64 banks.
__device__ __forceinline__ int swz(int row, int piece) { return row * kK1 + 8 * (piece ^ ((row >> 2) & 3)); }

// BF16 of two floats, round to nearest even (v_cvt_pk_bf16_f32); low half a
__device__ __forceinline__ unsigned bf16_pair(float a, float b) {
  const bf16x2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(unsigned, v);
}

__device__ __forceinline__ float sigmoid(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

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

// The wave's B fragments of one 128-deep product: rows 16 w + r of Bt
// [n][128], k-steps of 32 (lane group g holds k = 32 s + 8 g .. + 7).
__device__ __forceinline__ void load_cols(bf16x8 (&b)[4], const u16* __restrict__ Bt, int w, int r, int g) {
#pragma unroll
  for (int s = 0; s < 4; ++s) b[s] = frag(Bt + (16 * w + r) * kW + 32 * s + 8 * g);
}

// The wave's product over 64 rows x its 16 columns: acc[mt] for m-tile mt
// (rows 16 mt ..), reduction over KS k-steps, A row-major in LDS (leading
// dimension lda), B fragments b[s].
template <int KS>
__device__ __forceinline__ void wave_cols(f4 (&acc)[4], const u16* __restrict__ A, int lda, const bf16x8 (&b)[KS],
                                          int r, int g) {
  // m-tile by m-tile, so that the epilogue of one m-tile can overlap the
  // products of the next
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    bf16x8 a[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) a[s] = frag(A + (16 * mt + r) * lda + 32 * s + 8 * g);
    acc[mt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < KS; ++s) acc[mt] = mfma(a[s], b[s], acc[mt]);
  }
}

// The same product for a single k-step with Bt [n][32] in LDS (swizzled).
__device__ __forceinline__ void wave_cols_lds(f4 (&acc)[4], const u16* __restrict__ A, int lda,
                                              const u16* __restrict__ Bt, int w, int r, int g) {
  const bf16x8 b[1] = {frag(Bt + swz(16 * w + r, g))};
  wave_cols<1>(acc, A, lda, b, r, g);
}

// Activation tile of the wave (value h) into LDS in both orders; column
// n = 16 w + r, rows 16 mt + 4 g + i.
__device__ __forceinline__ void store_both(const float (&h)[4][4], u16* __restrict__ R, u16* __restrict__ T, int w,
                                           int r, int g) {
  const int n = 16 * w + r;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    uint2 pk;
    pk.x = bf16_pair(h[mt][0], h[mt][1]);
    pk.y = bf16_pair(h[mt][2], h[mt][3]);
    if (R) {
      u16* c = R + (16 * mt + 4 * g) * LDR + n;
      c[0] = (u16)pk.x;
      c[LDR] = (u16)(pk.x >> 16);
      c[2 * LDR] = (u16)pk.y;
      c[3 * LDR] = (u16)(pk.y >> 16);
    }
    *reinterpret_cast<uint2*>(T + n * LDT + 16 * mt + 4 * g) = pk;
  }
}

// dW[o][in] += sum over the tile's rows of dZ^T[o][row] X^T[in][row]: the
// wave's output rows o = 16 w + ..., NT column tiles, A = dZ^T and Bt = X^T
// feature-major in LDS.
template <int NT>
__device__ __forceinline__ void wave_wgrad(f4 (&acc)[NT], const u16* __restrict__ AT, const u16* __restrict__ BT,
                                           int w, int r, int g) {
#pragma unroll
  for (int k0 = 0; k0 < kRows; k0 += 32) {
    const bf16x8 a = frag(AT + (16 * w + r) * LDT + k0 + 8 * g);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = mfma(a, frag(BT + (16 * nt + r) * LDT + k0 + 8 * g), acc[nt]);
  }
}

typedef _Float16 h2 __attribute__((ext_vector_type(2)));

// SiLU of the wave's pre-activations acc + bias: values into h, derivatives
// into sp (FP16 pairs: rows 4 g + 2 q, 4 g + 2 q + 1 of m-tile mt).
__device__ __forceinline__ void silu_fwd(const f4 (&acc)[4], float bias, float (&h)[4][4], h2 (&sp)[4][2]) {
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      float d[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const float z = acc[mt][2 * q + e] + bias;
        const float sg = sigmoid(z);
        const float hv = z * sg;
        h[mt][2 * q + e] = hv;
        d[e] = fmaf(hv, 1.0f - sg, sg);  // sigma (1 + z (1 - sigma))
      }
      sp[mt][q] = h2{(_Float16)d[0], (_Float16)d[1]};
    }
}

// dZ = dA * silu'(Z) from the accumulators; the lane's column sum of dZ into
// cs (bias gradient); the result to LDS in both orders (R may be null).
__device__ __forceinline__ void backprop_silu(const f4 (&acc)[4], const h2 (&sp)[4][2], float& cs,
                                              u16* __restrict__ R, u16* __restrict__ T, int w, int r, int g) {
  float d[4][4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      d[mt][i] = acc[mt][i] * (float)sp[mt][i >> 1][i & 1];
      cs += d[mt][i];
    }
  store_both(d, R, T, w, r, g);
}

__global__ __launch_bounds__(kThreads, 1) void mlp_fused_step(FusedArgs a) {
  __shared__ __align__(16) u16 s_xr[2][kRows * LDX];  // X [row][32], two tiles (staged one ahead)
  __shared__ __align__(16) u16 s_xt[2][kK1 * LDT];    // X^T [32][row]
  __shared__ __align__(16) u16 s_r0[kRows * LDR];   // H1, H3, then dZ2 (row-major)
  __shared__ __align__(16) u16 s_r1[kRows * LDR];   // H2, then dZ3
  __shared__ __align__(16) u16 s_t1[kW * LDT];      // H1^T
  __shared__ __align__(16) u16 s_t2[kW * LDT];      // H2^T
  __shared__ __align__(16) u16 s_t3[kW * LDT];      // H3^T, then dZ2^T
  __shared__ __align__(16) u16 s_dzt[kW * LDT];     // dZ3^T, then dZ1^T
  __shared__ __align__(16) u16 s_dyr[kRows * LDX];  // dL/dy [row][32] (columns >= 4 zero)
  __shared__ __align__(16) u16 s_dyt[16 * LDT];     // dL/dy^T [16][row] (rows >= 4 zero)
  __shared__ __align__(16) u16 s_w1[kW * kK1];      // W1 [128][32] (inputs padded to 32), swizzled
  __shared__ __align__(16) u16 s_w4t[kW * kK1];     // W4^T [128][32] (outputs padded to 32), swizzled
  __shared__ __align__(16) u16 s_w4[16 * LDW4];     // W4 [16][128] (outputs padded to 16)
  __shared__ float s_tg[2][kRows][kOut];            // the tiles' targets
  __shared__ float s_gw1[kW][kIn];                  // dW1 sums over the tiles
  __shared__ float s_gw4[kOut][kW];                 // dW4 sums over the tiles
  __shared__ float s_red[4][16];
  __shared__ double s_loss[kWaves];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const u16* P = a.packed;
  const float* M = a.master;

  // this wave's fragments of the two 128 x 128 forward products, for every
  // tile; the three small matrices go to LDS
  bf16x8 w2[4], w3[4], wb[4];
  load_cols(w2, P + pW2, w, r, g);
  load_cols(w3, P + pW3, w, r, g);
  for (int e = tid; e < kW * kK1 / 8; e += kThreads) {  // 16-byte pieces, four per row
    const int row = e / (kK1 / 8), c = e % (kK1 / 8);
    *reinterpret_cast<uint4*>(s_w1 + swz(row, c)) = reinterpret_cast<const uint4*>(P + pW1)[e];
    *reinterpret_cast<uint4*>(s_w4t + swz(row, c)) = reinterpret_cast<const uint4*>(P + pW4t)[e];
  }
  for (int e = tid; e < 16 * kW / 8; e += kThreads) {  // sixteen per row
    const int row = e / (kW / 8), c = e % (kW / 8);
    *reinterpret_cast<uint4*>(s_w4 + row * LDW4 + 8 * c) = reinterpret_cast<const uint4*>(P + pW4)[e];
  }
  const float bias1 = M[ob1 + 16 * w + r], bias2 = M[ob2 + 16 * w + r], bias3 = M[ob3 + 16 * w + r];
  const float b4 = r < kOut ? M[ob4 + r] : 0.f;

  // gradient sums of this block (registers, all tiles)
  f4 gW2[8], gW3[8];
  float cs1 = 0.f, cs2 = 0.f, cs3 = 0.f, cs4 = 0.f;
  double loss = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) gW2[j] = gW3[j] = f4{0.f, 0.f, 0.f, 0.f};
  // padding columns of X and dL/dy stay zero for every tile
  for (int e = tid; e < kRows * LDX; e += kThreads) s_xr[0][e] = s_xr[1][e] = s_dyr[e] = 0;
  for (int e = tid; e < kK1 * LDT; e += kThreads) s_xt[0][e] = s_xt[1][e] = 0;
  for (int e = tid; e < 16 * LDT; e += kThreads) s_dyt[e] = 0;
  // the small gradients (dW1: 5 real input columns, dW4: 4 real output rows)
  // are summed in LDS, each entry by the one lane that computes it
  for (int e = tid; e < kW * kIn; e += kThreads) (&s_gw1[0][0])[e] = 0.f;
  for (int e = tid; e < kOut * kW; e += kThreads) (&s_gw4[0][0])[e] = 0.f;

  // the first wave loads a tile's inputs and targets (rows beyond the batch
  // are zero) two tiles ahead and the row indices three tiles ahead, so that
  // no load waits for another inside the loop, and stages the next tile's
  // inputs into the second LDS buffer at the end of the current tile
  float xin[kIn], tin[kOut];
  int64_t src_next = -1;  // row three tiles ahead (two after the fetch), -1 beyond the batch
  auto index = [&](int64_t tile) -> int64_t {
    const int64_t b = tile * kRows + tid;
    return b < a.B ? (a.rows ? a.rows[b] : b) : -1;
  };
  auto fetch = [&](int64_t src) {
#pragma unroll
    for (int f = 0; f < kIn; ++f) xin[f] = src >= 0 ? a.x[src * kIn + f] : 0.f;
#pragma unroll
    for (int o = 0; o < kOut; ++o) tin[o] = src >= 0 ? a.t[src * kOut + o] : 0.f;
  };
  // a tile's inputs into the LDS buffer xb (the first wave)
  auto stage = [&](int xb) {
#pragma unroll
    for (int f = 0; f < kIn; ++f) {
      const u16 h = (u16)bf16_pair(xin[f], 0.f);
      s_xr[xb][tid * LDX + f] = h;
      s_xt[xb][f * LDT + tid] = h;
    }
#pragma unroll
    for (int o = 0; o < kOut; ++o) s_tg[xb][tid][o] = tin[o];
  };
  __syncthreads();  // the zeroed buffers before the first staging
  if (tid < kRows) {
    fetch(index(blockIdx.x));
    stage(0);
    fetch(index(blockIdx.x + gridDim.x));
    src_next = index(blockIdx.x + 2 * (int64_t)gridDim.x);
  }
  __syncthreads();

  int xb = 0;  // the LDS input buffer of the current tile
  for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x, xb ^= 1) {
    const int64_t base = tile * kRows;
    const u16* xr = s_xr[xb];
    const u16* xt = s_xt[xb];
    h2 sp1[4][2], sp2[4][2], sp3[4][2];
    f4 acc[4];
    // ---- forward: three hidden layers
    {
      float h[4][4];
      wave_cols_lds(acc, xr, LDX, s_w1, w, r, g);
      silu_fwd(acc, bias1, h, sp1);
      store_both(h, s_r0, s_t1, w, r, g);
      __syncthreads();
      wave_cols<4>(acc, s_r0, LDR, w2, r, g);
      silu_fwd(acc, bias2, h, sp2);
      store_both(h, s_r1, s_t2, w, r, g);
      __syncthreads();
      wave_cols<4>(acc, s_r1, LDR, w3, r, g);
      silu_fwd(acc, bias3, h, sp3);
      store_both(h, s_r0, s_t3, w, r, g);
      __syncthreads();
    }
    load_cols(wb, P + pW3t, w, r, g);  // for layer 2 of the backward pass
    // ---- output layer and loss: waves 0-3, wave w takes rows 16 w .. 16 w + 15
    if (w < 4) {
      f4 y = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 4; ++s)
        y = mfma(frag(s_r0 + (16 * w + r) * LDR + 32 * s + 8 * g), frag(s_w4 + r * LDW4 + 32 * s + 8 * g), y);
      // lane: column r (output r < 4), rows 16 w + 4 g + i
      float dyv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * w + 4 * g + i;
        float dy = 0.f;
        if (r < kOut && base + row < a.B) {
          const float d = y[i] + b4 - s_tg[xb][row][r];
          loss += (double)d * (double)d;
          dy = d * a.dy_scale;
        }
        cs4 += dy;
        dyv[i] = dy;
      }
      uint2 pk;
      pk.x = bf16_pair(dyv[0], dyv[1]);
      pk.y = bf16_pair(dyv[2], dyv[3]);
      u16* c = s_dyr + (16 * w + 4 * g) * LDX + r;
      c[0] = (u16)pk.x;
      c[LDX] = (u16)(pk.x >> 16);
      c[2 * LDX] = (u16)pk.y;
      c[3 * LDX] = (u16)(pk.y >> 16);
      *reinterpret_cast<uint2*>(s_dyt + r * LDT + 16 * w + 4 * g) = pk;
    }
    __syncthreads();
    // ---- layer 3: dZ3 = (dy W4) * silu'(Z3); dW4 += dy^T H3 (columns 16 w ..)
    wave_cols_lds(acc, s_dyr, LDX, s_w4t, w, r, g);
    backprop_silu(acc, sp3, cs3, s_r1, s_dzt, w, r, g);
    {
      f4 t4 = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k0 = 0; k0 < kRows; k0 += 32)
        t4 = mfma(frag(s_dyt + r * LDT + k0 + 8 * g), frag(s_t3 + (16 * w + r) * LDT + k0 + 8 * g), t4);
      if (g == 0)  // output rows 4 g + i < 4
#pragma unroll
        for (int i = 0; i < kOut; ++i) s_gw4[i][16 * w + r] += t4[i];
    }
    __syncthreads();
    // ---- layer 2: dW3 += dZ3^T H2; dZ2 = (dZ3 W3) * silu'(Z2)
    // (dZ2 goes to buffers nobody reads in this phase: s_r0, whose H3 the
    // output layer consumed, and s_t3, whose H3^T the dW4 product consumed)
    wave_wgrad<8>(gW3, s_dzt, s_t2, w, r, g);
    wave_cols<4>(acc, s_r1, LDR, wb, r, g);
    load_cols(wb, P + pW2t, w, r, g);  // for layer 1
    backprop_silu(acc, sp2, cs2, s_r0, s_t3, w, r, g);
    __syncthreads();
    // ---- layer 1: dW2 += dZ2^T H1; dZ1 = (dZ2 W2) * silu'(Z1) (dZ1^T into
    // s_dzt, whose dZ3^T the dW3 product of the previous phase consumed)
    wave_wgrad<8>(gW2, s_t3, s_t1, w, r, g);
    wave_cols<4>(acc, s_r0, LDR, wb, r, g);
    backprop_silu(acc, sp1, cs1, nullptr, s_dzt, w, r, g);
    __syncthreads();
    // ---- dW1 += dZ1^T X; the next tile's inputs into the other buffer
    {
      f4 t1[1] = {f4{0.f, 0.f, 0.f, 0.f}};
      wave_wgrad<1>(t1, s_dzt, xt, w, r, g);  // input columns r < 16, of which 5 are real
      if (r < kIn)
#pragma unroll
        for (int i = 0; i < 4; ++i) s_gw1[16 * w + 4 * g + i][r] += t1[0][i];
    }
    if (tid < kRows) {
      stage(xb ^ 1);
      fetch(src_next);
      src_next = index(tile + 3 * (int64_t)gridDim.x);
    }
    __syncthreads();  // the next tile overwrites the activation buffers
  }

  // ---- this block's partial gradient, in the master layout
  float* out = a.part + (int64_t)blockIdx.x * kParams;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int o = 16 * w + 4 * g + i;
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) {
      out[oW2 + o * kW + 16 * nt + r] = gW2[nt][i];
      out[oW3 + o * kW + 16 * nt + r] = gW3[nt][i];
    }
  }
  // bias sums: each lane holds its column's sum over its rows; add the four
  // row groups g (lanes r, r + 16, r + 32, r + 48)
  auto colsum = [&](float v) {
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
  };
  const float s1 = colsum(cs1), s2 = colsum(cs2), s3 = colsum(cs3), s4 = colsum(cs4);
  if (g == 0) {
    out[ob1 + 16 * w + r] = s1;
    out[ob2 + 16 * w + r] = s2;
    out[ob3 + 16 * w + r] = s3;
    if (w < 4) s_red[w][r] = s4;  // output column r over the wave's rows
  }
  // loss: FP64 over the block
  double l = loss;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
  if (lane == 0) s_loss[w] = l;
  __syncthreads();  // also: the LDS sums of dW1 and dW4 are complete
  for (int e = tid; e < kW * kIn; e += kThreads) out[oW1 + e] = (&s_gw1[0][0])[e];
  for (int e = tid; e < kOut * kW; e += kThreads) out[oW4 + e] = (&s_gw4[0][0])[e];
  if (tid < kOut) out[ob4 + tid] = s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
  if (tid == 0) {
    double t = 0.0;
    for (int q = 0; q < kWaves; ++q) t += s_loss[q];
    a.lpart[blockIdx.x] = t;
  }
}

// grad[p] = sum over blocks of part[blk][p] in a fixed order: a block of the
// reduction takes 64 parameters (one per lane, so every load of a wave is 256
// contiguous bytes); its 16 waves add consecutive sixteenths of the blocks'
// partials in ascending order, then wave 0 adds the 16 sums in order.  loss =
// sum of the blocks' loss sums / (4 B).  With UPDATE the same thread then
// takes the Adam step of parameter p (the arithmetic of mpf_adam_step) and
// writes its BF16 copies (those of mpf_mlp_pack; the zero padding of the
// packed copy is never touched).
constexpr int kRedCols = 64, kRedRows = 16;

struct AdamArg {
  float* master;
  float* m;
  float* v;
  u16* packed;
  float lr, b1, b2, eps, c1, c2;
};

template <bool UPDATE>
__global__ __launch_bounds__(kRedCols* kRedRows) void fused_reduce(const float* __restrict__ part, int nblk,
                                                                   float* __restrict__ grad,
                                                                   const double* __restrict__ lpart, double inv_n,
                                                                   double* __restrict__ loss,
                                                                   double* __restrict__ loss_sum, AdamArg ad) {
  __shared__ float s[kRedRows][kRedCols + 1];
  const int c = threadIdx.x % kRedCols, rr = threadIdx.x / kRedCols;
  const int p = blockIdx.x * kRedCols + c;
  const int per = (nblk + kRedRows - 1) / kRedRows;
  const int b0 = rr * per, b1 = min(nblk, b0 + per);
  float acc = 0.f;
  if (p < kParams) {
    constexpr int U = 8;  // loads in flight
    int b = b0;
    for (; b + U <= b1; b += U) {
      float q[U];
#pragma unroll
      for (int u = 0; u < U; ++u) q[u] = part[(int64_t)(b + u) * kParams + p];
#pragma unroll
      for (int u = 0; u < U; ++u) acc += q[u];
    }
    for (; b < b1; ++b) acc += part[(int64_t)b * kParams + p];
  }
  s[rr][c] = acc;
  __syncthreads();
  if (rr == 0 && p < kParams) {
    float gsum = s[0][c];
#pragma unroll
    for (int q = 1; q < kRedRows; ++q) gsum += s[q][c];
    grad[p] = gsum;
    if constexpr (UPDATE) {
      const float mi = ad.b1 * ad.m[p] + (1.f - ad.b1) * gsum;
      const float vi = ad.b2 * ad.v[p] + (1.f - ad.b2) * gsum * gsum;
      ad.m[p] = mi;
      ad.v[p] = vi;
      const float x = ad.master[p] - ad.lr * (mi / ad.c1) / (sqrtf(vi / ad.c2) + ad.eps);
      ad.master[p] = x;
      const u16 h = (u16)bf16_pair(x, 0.f);
      if (p < ob1) {
        ad.packed[pW1 + (p - oW1) / kIn * kK1 + (p - oW1) % kIn] = h;
      } else if (p >= oW2 && p < ob2) {
        const int o = (p - oW2) / kW, i = (p - oW2) % kW;
        ad.packed[pW2 + o * kW + i] = h;
        ad.packed[pW2t + i * kW + o] = h;
      } else if (p >= oW3 && p < ob3) {
        const int o = (p - oW3) / kW, i = (p - oW3) % kW;
        ad.packed[pW3 + o * kW + i] = h;
        ad.packed[pW3t + i * kW + o] = h;
      } else if (p >= oW4 && p < ob4) {
        const int o = (p - oW4) / kW, i = (p - oW4) % kW;
        ad.packed[pW4 + o * kW + i] = h;
        ad.packed[pW4t + i * kK1 + o] = h;
      }
    }
  }
  if (blockIdx.x == 0) {
    // the blocks' loss sums: thread t takes blocks t, t + 1024, ... in
    // order, then a fixed pairwise tree
    __shared__ double sl[kRedCols * kRedRows];
    double l = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kRedCols * kRedRows) l += lpart[b];
    sl[threadIdx.x] = l;
    __syncthreads();
    for (int h = kRedCols * kRedRows / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) sl[threadIdx.x] += sl[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const double t = sl[0] * inv_n;
      if (loss) *loss = t;
      if (loss_sum) *loss_sum += t;
    }
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
  hipLaunchKernelGGL(fused_reduce<false>, dim3((kParams + kRedCols - 1) / kRedCols), dim3(kRedCols * kRedRows), 0,
                     st, (const float*)part, nblk, grad, (const double*)lpart, 1.0 / (4.0 * (double)B), loss,
                     (double*)nullptr, AdamArg{});
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
  if (!(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f)) return MPF_ERR_ARG;
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
    // Adam's bias corrections as mpf_adam_step forms them
    const int step = (int)(step0 + i + 1);
    const AdamArg ad{master, m, v, (u16*)packed, (float)lr, b1, b2, eps,
                     (float)(1.0 - pow((double)b1, step)), (float)(1.0 - pow((double)b2, step))};
    hipLaunchKernelGGL(fused_reduce<true>, dim3((kParams + kRedCols - 1) / kRedCols), dim3(kRedCols * kRedRows), 0,
                       st, (const float*)part, nblk, grad, (const double*)lpart, 1.0 / (4.0 * (double)B),
                       (double*)nullptr, loss_sum, ad);
    lr *= lr_ratio;
  }
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}
