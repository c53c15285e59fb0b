// Meshless TRT lattice Boltzmann steps (Sec. 2.2) on gfx950.
//
// State: populations shifted by their lattice weight, f~_k = f_k - w_k, stored
// node-major as records of qp values (qp = 20 for D3Q19, 16 for D3Q15; the
// padding entries stay zero), so one neighbour's populations arrive with a
// few 16-byte loads from one or two cache lines.  The shift makes FP32 storage usable: the forcing term per
// step is about 1e-9 of f_k, below FP32 resolution of f_k itself but not of
// the deviation f~_k.  The equilibrium and the TRT split are written for the
// shifted values directly (w_k = w_{opp(k)}, so the shift cancels in f - f^eq).
//
// A step is one fused pass per node tile: gather-stream the post-collision
// populations of the stencil (Eq. LBM_streaming with interpolation weights of
// Eq. operatorApprox), bounce back the unknown populations of surface nodes
// (Eq. interpolated_bounceback_mlbm; which ones are unknown is a per-node bit
// mask, built once by lbm_unknown), then collide (Eqs. macro_var, feq,
// LBM_collision, force_lbm) and write the next post-collision state.  Weights
// stream coalesced from [k][j][node].
//
// Compensated FP32 state (MPF_F32_KAHAN): next to the FP32 records f lives a
// caller-owned FP32 record comp per node, so the state is f + comp.  The
// column loop is the FP32 one (neighbours contribute their FP32 records);
// the tile's epilogue adds the node's own comp through its rest population
// and its self column (W_k0 comp_k) in FP64, bounces back and collides in
// FP64, and splits the result into the FP32 value and the FP32 remainder.
// An update smaller than half an ulp of f then moves comp instead of being
// rounded away every step, which is what stalls a plain FP32 state short of
// its fixed point.
#include <type_traits>

#include "common.hpp"

namespace mpf {
namespace {

constexpr int kBlock = 256;

template <typename T>
struct Prm {
  T itp, itm;  // 1/tau+, 1/tau-
  T g0, g1, g2;
};

// Record length of a node's populations in the node-major layout.
template <int Q>
struct Pad;
template <>
struct Pad<19> {
  static constexpr int QP = 20;
};
template <>
struct Pad<15> {
  static constexpr int QP = 16;
};

template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int n = 4;
};
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int n = 2;
};

// TRT collision of one node's shifted populations, in place.  Returns the
// flags bits of the node: MPF_FLAG_NONFINITE for a non-finite density or
// velocity, MPF_FLAG_LIMIT for |u|^2 >= 1/3 (the lattice speed of sound).
template <typename T, int Q>
__device__ __forceinline__ uint32_t collide(T (&f)[Q], const Prm<T>& pr) {
  using L = Lattice<Q>;
  T drho = T(0), j0 = T(0), j1 = T(0), j2 = T(0);
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    drho += f[k];
    if (L::ex[k]) j0 += L::ex[k] > 0 ? f[k] : -f[k];
    if (L::ey[k]) j1 += L::ey[k] > 0 ? f[k] : -f[k];
    if (L::ez[k]) j2 += L::ez[k] > 0 ? f[k] : -f[k];
  }
  const T rho = T(1) + drho;
  const T ir = T(1) / rho;
  const T u0 = j0 * ir, u1 = j1 * ir, u2 = j2 * ir;
  const T uu = u0 * u0 + u1 * u1 + u2 * u2;
  const T F0 = rho * pr.g0, F1 = rho * pr.g1, F2 = rho * pr.g2;
  // x - x is 0 for a finite x and NaN otherwise
  const uint32_t bits = !(drho - drho == T(0) && uu - uu == T(0)) ? MPF_FLAG_NONFINITE
                                                                  : (uu >= T(1) / T(3) ? MPF_FLAG_LIMIT : 0u);
  // each opposite pair (k, kb) is relaxed together and in place: the TRT
  // update of f_k involves only f_k and f_kb, so no full f^eq, F or output
  // arrays stay live (fewer registers for the FP64 state)
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const int kb = lat_opp(k);
    if (kb < k) continue;
    const T wk = (T)lat_w<Q>(k);
    const T eu = T(L::ex[k]) * u0 + T(L::ey[k]) * u1 + T(L::ez[k]) * u2;
    const T ebu = T(L::ex[kb]) * u0 + T(L::ey[kb]) * u1 + T(L::ez[kb]) * u2;
    // f^eq_k - w_k = w_k (drho + rho (3 eu + 4.5 eu^2 - 1.5 uu))
    const T feq = wk * (drho + rho * (T(3) * eu + T(4.5) * eu * eu - T(1.5) * uu));
    const T feqb = wk * (drho + rho * (T(3) * ebu + T(4.5) * ebu * ebu - T(1.5) * uu));
    const T Fk = T(3) * wk * (T(L::ex[k]) * F0 + T(L::ey[k]) * F1 + T(L::ez[k]) * F2);
    const T Fkb = T(3) * wk * (T(L::ex[kb]) * F0 + T(L::ey[kb]) * F1 + T(L::ez[kb]) * F2);
    const T fk = f[k], fb = f[kb];
    const T fp = T(0.5) * (fk + fb), fm = T(0.5) * (fk - fb);
    const T ep = T(0.5) * (feq + feqb), em = T(0.5) * (feq - feqb);
    f[k] = fk - (fp - ep) * pr.itp - (fm - em) * pr.itm + Fk;
    if (kb != k) {
      const T fmb = T(0.5) * (fb - fk), emb = T(0.5) * (feqb - feq);
      f[kb] = fb - (fp - ep) * pr.itp - (fmb - emb) * pr.itm + Fkb;
    }
  }
  return bits;
}

// The compensated state collides and streams in FP64.
template <typename T, bool KAHAN>
struct Compute {
  using type = T;
};
template <>
struct Compute<float, true> {
  using type = double;
};

// Record of QP values at rec (16-byte aligned) into r[].
template <typename T, int QP>
__device__ __forceinline__ void load_rec(const T* __restrict__ rec, T (&r)[QP]) {
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::n;
  const V* p = reinterpret_cast<const V*>(rec);
#pragma unroll
  for (int v = 0; v < QP / VN; ++v) {
    V x = p[v];
    if constexpr (VN == 4) {
      r[4 * v] = x.x; r[4 * v + 1] = x.y; r[4 * v + 2] = x.z; r[4 * v + 3] = x.w;
    } else {
      r[2 * v] = x.x; r[2 * v + 1] = x.y;
    }
  }
}

template <typename T, int QP>
__device__ __forceinline__ void store_rec(T* __restrict__ rec, const T (&r)[QP]) {
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::n;
  V* p = reinterpret_cast<V*>(rec);
#pragma unroll
  for (int v = 0; v < QP / VN; ++v) {
    V x;
    if constexpr (VN == 4) {
      x.x = r[4 * v]; x.y = r[4 * v + 1]; x.z = r[4 * v + 2]; x.w = r[4 * v + 3];
    } else {
      x.x = r[2 * v]; x.y = r[2 * v + 1];
    }
    p[v] = x;
  }
}

// hi = fl32(x), lo = fl32(x - hi): the FP32 pair of a compensated value.
template <int QP>
__device__ __forceinline__ void split_store(const double (&x)[QP], float* __restrict__ hi_rec,
                                            float* __restrict__ lo_rec) {
  float hi[QP], lo[QP];
#pragma unroll
  for (int k = 0; k < QP; ++k) {
    hi[k] = (float)x[k];
    lo[k] = (float)(x[k] - (double)hi[k]);
  }
  store_rec<float, QP>(hi_rec, hi);
  store_rec<float, QP>(lo_rec, lo);
}

__device__ __forceinline__ void raise_flags(uint32_t* flags, uint32_t bits) {
  if (flags && bits) atomicOr(flags, bits);
}

// src may equal dst: each thread reads and writes only its own node.  With
// a compensation record comp (compensated state; CT = double) the node's
// value is src + comp, collided in FP64 and split back into dst and comp.
template <typename T, typename CT, int Q>
__global__ __launch_bounds__(kBlock) void lbm_collide(int64_t n, const T* src, T* dst, T* comp, Prm<CT> pr,
                                                      uint32_t* flags) {
  constexpr int QP = Pad<Q>::QP;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  CT f[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) f[k] = (CT)src[i * QP + k] + (comp ? (CT)comp[i * QP + k] : CT(0));
  raise_flags(flags, collide<CT, Q>(f, pr));
  if constexpr (sizeof(CT) != sizeof(T)) {
    double x[QP];
#pragma unroll
    for (int k = 0; k < QP; ++k) x[k] = k < Q ? (double)f[k] : 0.0;
    split_store<QP>(x, dst + i * QP, comp + i * QP);
  } else {
#pragma unroll
    for (int k = 0; k < Q; ++k) dst[i * QP + k] = f[k];
  }
}

// Blocks take 64-node tiles; hardware hands workgroups to the 8 XCDs round
// robin, so block b works on tile (b % 8) * (G / 8) + b / 8 and each XCD's L2
// sees one contiguous (Morton-ordered, hence compact) range of nodes.
constexpr int kTile = 64;
constexpr int kXcd = 8;
// Waves per 64-node tile in the step kernel: 8, and 6 for FP32 weights with
// an FP64 state (6 % faster on a 581k-node cell, equal on a 71k-node one;
// FP32 and FP64 are fastest at 8 on both).
template <typename TW, typename T>
constexpr int step_waves() { return sizeof(TW) == 4 && sizeof(T) == 8 ? 6 : 8; }

__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t G) { return (b % kXcd) * (G / kXcd) + b / kXcd; }

inline unsigned tiles_grid(int64_t n) {
  int64_t t = (n + kTile - 1) / kTile;
  t = (t + kXcd - 1) / kXcd * kXcd;
  return (unsigned)t;
}

// One step for a tile of 64 nodes (lane = node).  The waves of the
// block (step_waves) take the stencil columns in turn; for each column a lane loads its
// neighbour's whole population record with 16-byte loads and accumulates all
// q - 1 moving populations against the coalesced weights.  The partial sums
// meet in LDS and are added in a fixed order by the first wave, which then
// applies bounce-back and the collision and writes the tile.  The column loop
// is deliberately not unrolled (unrolling cost 30-60 % of the step time).
// STREAM_W selects non-temporal weight loads.  Weights that fit the 256 MB
// Infinity Cache are read from it on every step after the first, and
// streaming them then costs 6-50 %; weights far larger than it are read from
// HBM anyway, and streaming them keeps the gathered population records in the
// caches (6 % faster at 1.26-2.5 GB of weights, all precisions).
// The tile plan of the LDS-staged gather (HALO): count[t] distinct stencil
// nodes of tile t, listed ascending in halo[t][0, count), and every stencil
// entry as its 16-bit position in its tile's list.
struct TileArg {
  const int32_t* count;
  const int32_t* halo;
  const uint16_t* lidx;
  int h_cap;
};

// LDS of the step kernel: the waves' partial sums, and with HALO first the
// tile's halo records (the partial sums reuse that space afterwards).
template <typename TW, typename T, int Q>
constexpr size_t step_part_bytes() { return sizeof(T) * step_waves<TW, T>() * (Q - 1) * kTile; }

// The compensated state's FP64 epilogue would take 94 VGPRs (two 8-wave
// blocks per CU); capped at 80 (three blocks, a few values spilled in the
// epilogue) the step is 6-7 % faster on the 71k and 581k-node cells.  The
// staged FP64 kernel is bounded the other way (at most four waves per SIMD):
// with its LDS sized at launch the compiler would otherwise aim at an
// occupancy that its two blocks per CU never reach and cut its registers.
template <typename TW, typename T, int Q, bool COLLIDE, bool STREAM_W, bool KAHAN, bool HALO>
__global__ __launch_bounds__((step_waves<TW, T>() * kWave))
__attribute__((amdgpu_waves_per_eu(KAHAN ? 6 : 1, (sizeof(TW) == 8 && HALO) ? 4 : 8))) void lbm_step(
    int64_t n, int64_t n_int, int nl, const int32_t* __restrict__ sten, const TW* __restrict__ W,
    const uint32_t* __restrict__ unknown, const T* __restrict__ src, T* __restrict__ dst, T* __restrict__ comp,
    Prm<typename Compute<T, KAHAN>::type> pr, uint32_t* __restrict__ flags, TileArg tp) {
  using CT = typename Compute<T, KAHAN>::type;
  constexpr int QP = Pad<Q>::QP;
  constexpr int NW = step_waves<TW, T>();
  // Without HALO the partial sums sit in a static array: the compiler then
  // knows the LDS bound on occupancy and spends the registers it leaves on
  // loads in flight (with dynamic LDS it aims at an occupancy the launch
  // cannot reach, and the FP64 step slows by up to 25 %).
  unsigned char* lds_raw;
  if constexpr (HALO) {
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    lds_raw = lds_dyn;
  } else {
    __shared__ __align__(16) unsigned char lds_fixed[step_part_bytes<TW, T, Q>()];
    lds_raw = lds_fixed;
  }
  T(*part)[Q - 1][kTile] = reinterpret_cast<T(*)[Q - 1][kTile]>(lds_raw);
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile * kTile >= n) return;  // whole block
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const int64_t i = tile * kTile + lane;
  const bool live = i < n;
  const int64_t ic = live ? i : n - 1;
  const int64_t ks = (int64_t)nl * n;  // population stride in W
  T* recs = reinterpret_cast<T*>(lds_raw);
  if constexpr (HALO) {
    // the tile's halo records into LDS, 16 bytes per thread per pass:
    // consecutive threads take consecutive pieces of ascending records
    using V = typename Vec16<T>::type;
    constexpr int NV = QP / Vec16<T>::n;
    const int cnt = tp.count[tile];
    const int32_t* hl = tp.halo + tile * tp.h_cap;
    V* dstv = reinterpret_cast<V*>(recs);
    for (int c = threadIdx.x; c < cnt * NV; c += NW * kWave) {
      const int r = c / NV;
      dstv[c] = reinterpret_cast<const V*>(src + (int64_t)hl[r] * QP)[c - r * NV];
    }
    __syncthreads();
  }
  T acc[Q];
#pragma unroll
  for (int k = 0; k < Q; ++k) acc[k] = T(0);
#pragma unroll 1
  for (int j = wv; j < nl; j += NW) {
    const int64_t at = (int64_t)j * n + ic;
    T r[QP];
    if constexpr (HALO) {
      load_rec<T, QP>(recs + (int)tp.lidx[at] * QP, r);
    } else {
      const int64_t s = sten[at];
      load_rec<T, QP>(src + s * QP, r);
    }
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      const TW* wk = W + (k - 1) * ks + at;
      TW w;
      if constexpr (STREAM_W) w = __builtin_nontemporal_load(wk);
      else w = *wk;
      acc[k] += (T)w * r[k];
    }
  }
  if constexpr (HALO) __syncthreads();  // every wave is done with the records before they are overwritten
#pragma unroll
  for (int k = 1; k < Q; ++k) part[wv][k - 1][lane] = acc[k];
  __syncthreads();
  if (wv != 0 || !live) return;
  CT f[QP];
  f[0] = (CT)src[ic * QP];
  if constexpr (KAHAN) f[0] += (CT)comp[ic * QP];
#pragma unroll
  for (int k = 1; k < Q; ++k) {
    CT sum = (CT)part[0][k - 1][lane];
#pragma unroll
    for (int w = 1; w < NW; ++w) sum += (CT)part[w][k - 1][lane];
    // the node's own remainder through its self column (column 0)
    if constexpr (KAHAN) sum += (CT)W[(k - 1) * ks + ic] * (CT)comp[ic * QP + k];
    f[k] = sum;
  }
#pragma unroll
  for (int k = Q; k < QP; ++k) f[k] = CT(0);
  if (i >= n_int) {
    // unknown populations take their opposite's streamed value; both
    // members of a pair may be unknown (then they swap)
    const uint32_t mask = unknown[i - n_int];
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      const int kb = lat_opp(k);
      if (k < kb) {
        const CT a = f[k], b = f[kb];
        if (mask >> k & 1u) f[k] = b;
        if (mask >> kb & 1u) f[kb] = a;
      }
    }
  }
  if (COLLIDE) {
    CT c[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) c[k] = f[k];
    raise_flags(flags, collide<CT, Q>(c, pr));
#pragma unroll
    for (int k = 0; k < Q; ++k) f[k] = c[k];
  }
  if constexpr (KAHAN) {
    split_store<QP>(f, dst + i * QP, comp + i * QP);
  } else {
    store_rec<T, QP>(dst + i * QP, f);
  }
}

template <typename T, int Q>
__global__ __launch_bounds__(kBlock) void lbm_init(int64_t n, T* __restrict__ f, double rho, double u0, double u1,
                                                   double u2) {
  using L = Lattice<Q>;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  constexpr int QP = Pad<Q>::QP;
  const double uu = u0 * u0 + u1 * u1 + u2 * u2;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const double eu = L::ex[k] * u0 + L::ey[k] * u1 + L::ez[k] * u2;
    const double wk = lat_w<Q>(k);
    f[i * QP + k] = (T)(wk * ((rho - 1.0) + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu)));
  }
#pragma unroll
  for (int k = Q; k < QP; ++k) f[i * QP + k] = T(0);
}

// Equilibrium populations of given macroscopic fields in physical units, the
// inverse of lbm_moments: u_lb = v / vs, rho = 1 + 3 p / vs^2.
template <typename T, int Q>
__global__ __launch_bounds__(kBlock) void lbm_init_fields(int64_t n, const double* __restrict__ v,
                                                          const double* __restrict__ p, double vs,
                                                          T* __restrict__ f) {
  using L = Lattice<Q>;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  constexpr int QP = Pad<Q>::QP;
  const double u0 = v[i] / vs, u1 = v[n + i] / vs, u2 = v[2 * n + i] / vs;
  const double drho = 3.0 * p[i] / (vs * vs), rho = 1.0 + drho;
  const double uu = u0 * u0 + u1 * u1 + u2 * u2;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    const double eu = L::ex[k] * u0 + L::ey[k] * u1 + L::ez[k] * u2;
    f[i * QP + k] = (T)(lat_w<Q>(k) * (drho + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu)));
  }
#pragma unroll
  for (int k = Q; k < QP; ++k) f[i * QP + k] = T(0);
}

template <typename T, int Q>
__global__ __launch_bounds__(kBlock) void lbm_moments(int64_t n, const T* __restrict__ f, const T* __restrict__ comp,
                                                      double vs, double* __restrict__ v, double* __restrict__ p) {
  using L = Lattice<Q>;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double drho = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
#pragma unroll
  for (int k = 0; k < Q; ++k) {
    // the compensated state is hi + lo, added in FP64
    const double fk = (double)f[i * Pad<Q>::QP + k] + (comp ? (double)comp[i * Pad<Q>::QP + k] : 0.0);
    drho += fk;
    j0 += L::ex[k] * fk;
    j1 += L::ey[k] * fk;
    j2 += L::ez[k] * fk;
  }
  const double rho = 1.0 + drho;
  v[i] = vs * j0 / rho;
  v[n + i] = vs * j1 / rho;
  v[2 * n + i] = vs * j2 / rho;
  if (p) p[i] = vs * vs * drho / 3.0;
}

// Unknown populations of boundary node b as a bit mask (bit k: population k).
// Normal rule (Sec. 2.2): e_k . n_b > 0, the departure point lies on the solid
// side of the tangent plane.  Solid rule (Sec. 3.3, the touching limit): the
// departure point x_b - dx e_k itself lies inside a grain, the grain being the
// ball of radius r around the cell centre or one of its periodic images; the
// nearest image is taken per axis (offset rint(p - 1/2)).  The products by
// e_k are exact (e_k in {-1, 0, 1}^3) and the squared distance is rounded
// operation by operation (contraction into fused multiply-adds is off in this
// kernel), so the decision matches a plain FP64 evaluation.
template <int Q>
__global__ __launch_bounds__(kBlock) void lbm_unknown(int64_t nb, int64_t n, int64_t n_int,
                                                      const double* __restrict__ pos,
                                                      const double* __restrict__ nrm, int rule, double dx, double r,
                                                      uint32_t* __restrict__ unknown) {
#pragma clang fp contract(off)
  using L = Lattice<Q>;
  const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (b >= nb) return;
  uint32_t mask = 0;
  if (rule == MPF_UNKNOWN_NORMAL) {
    const double nx = nrm[b], ny = nrm[nb + b], nz = nrm[2 * nb + b];
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      const double en = (double)L::ex[k] * nx + (double)L::ey[k] * ny + (double)L::ez[k] * nz;
      if (en > 0.0) mask |= 1u << k;
    }
  } else {
    const int64_t i = n_int + b;
    const double x[3] = {pos[i], pos[n + i], pos[2 * n + i]};
    const double r2 = r * r;
#pragma unroll
    for (int k = 1; k < Q; ++k) {
      const double e[3] = {(double)L::ex[k], (double)L::ey[k], (double)L::ez[k]};
      double d2 = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double p = x[a] - dx * e[a];
        const double c = 0.5 + rint(p - 0.5);
        const double d = p - c;
        d2 = a == 0 ? d * d : d2 + d * d;
      }
      if (d2 < r2) mask |= 1u << k;
    }
  }
  unknown[b] = mask;
}

// Weight arrays above this size are streamed (non-temporal loads): twice the
// Infinity Cache, between the measured points where caching wins (0.31 GB)
// and where streaming wins (1.26 GB).
constexpr double kStreamWeightsBytes = 512.0 * 1024 * 1024;

// LDS staging is used when the largest halo fits this many bytes of
// records: 64 KiB for FP32 records keeps three 8-wave blocks per CU at the
// step kernel's register use (halos of up to 819 records); the FP64 kernel
// holds two blocks per CU at its register use anyway, so 80 KiB (512 records)
// costs it no occupancy (the refined clouds here: about 350 on average, 500
// at most; on the 71k-node cell its step drops from 88.9 to 74.8 us).  The
// mixed kernel (FP32 weights, FP64 state) keeps 64 KiB: staged at 80 KiB it
// was slower (50.2 -> 55.4 us).
template <typename TW, typename T>
constexpr size_t halo_lds_bytes() { return sizeof(T) == 8 && sizeof(TW) == 8 ? 80 * 1024 : 64 * 1024; }

template <typename TW, typename T, int Q, bool STREAM_W, bool KAHAN, bool HALO>
void launch_steps(int64_t n, int64_t n_int, int nl, const int32_t* sten, const TW* W, const uint32_t* unknown,
                  T* f, T* ft, T* comp, T* cur, int n_steps, const Prm<typename Compute<T, KAHAN>::type>& pr,
                  uint32_t* flags, const TileArg& tp, size_t lds, hipStream_t st) {
  const unsigned gt = tiles_grid(n);
  const dim3 blk(step_waves<TW, T>() * kWave);
  for (int s = 0; s < n_steps - 1; ++s) {
    T* nxt = cur == f ? ft : f;
    hipLaunchKernelGGL((lbm_step<TW, T, Q, true, STREAM_W, KAHAN, HALO>), dim3(gt), blk, lds, st, n, n_int, nl,
                       sten, W, unknown, (const T*)cur, nxt, comp, pr, flags, tp);
    cur = nxt;
  }
  hipLaunchKernelGGL((lbm_step<TW, T, Q, false, STREAM_W, KAHAN, HALO>), dim3(gt), blk, lds, st, n, n_int, nl, sten,
                     W, unknown, (const T*)cur, f, comp, pr, flags, tp);
}

template <typename TW, typename T, int Q, bool KAHAN>
int run(const mpf_lbm_params* prm, int64_t n, int64_t n_int, int nl, const int32_t* sten, const TW* W,
        const uint32_t* unknown, const mpf_tiles* tiles, T* f, T* ft, T* comp, uint32_t* flags, int n_steps,
        hipStream_t st) {
  using CT = typename Compute<T, KAHAN>::type;
  Prm<CT> pr{(CT)(1.0 / prm->tau_plus), (CT)(1.0 / prm->tau_minus), (CT)prm->g_lb[0], (CT)prm->g_lb[1],
             (CT)prm->g_lb[2]};
  const unsigned g = grid_for(n, kBlock);
  // collide so that after n_steps - 1 fused passes the current state sits in
  // ft, and the last (stream-only) pass lands in f
  T* cur = (n_steps - 1) % 2 == 0 ? ft : f;
  hipLaunchKernelGGL((lbm_collide<T, CT, Q>), dim3(g), dim3(kBlock), 0, st, n, (const T*)f, cur, comp, pr, flags);
  constexpr int QP = Pad<Q>::QP;
  const size_t part = step_part_bytes<TW, T, Q>();
  const size_t halo_bytes = tiles ? (size_t)tiles->h_max * QP * sizeof(T) : 0;
  const bool halo = tiles && halo_bytes <= halo_lds_bytes<TW, T>();
  const TileArg tp{tiles ? tiles->count : nullptr, tiles ? tiles->halo : nullptr, tiles ? tiles->lidx : nullptr,
                   tiles ? tiles->h_cap : 0};
  const size_t lds = halo ? (halo_bytes > part ? halo_bytes : part) : 0;  // else static
  const bool stream_w = (double)(Q - 1) * nl * n * sizeof(TW) > kStreamWeightsBytes;
  if (halo) {
    if (stream_w)
      launch_steps<TW, T, Q, true, KAHAN, true>(n, n_int, nl, sten, W, unknown, f, ft, comp, cur, n_steps, pr, flags,
                                                tp, lds, st);
    else
      launch_steps<TW, T, Q, false, KAHAN, true>(n, n_int, nl, sten, W, unknown, f, ft, comp, cur, n_steps, pr,
                                                 flags, tp, lds, st);
  } else {
    if (stream_w)
      launch_steps<TW, T, Q, true, KAHAN, false>(n, n_int, nl, sten, W, unknown, f, ft, comp, cur, n_steps, pr,
                                                 flags, tp, lds, st);
    else
      launch_steps<TW, T, Q, false, KAHAN, false>(n, n_int, nl, sten, W, unknown, f, ft, comp, cur, n_steps, pr,
                                                  flags, tp, lds, st);
  }
  MPF_LAUNCH_CHECK();
  return check_flags(flags, st);
}

// Populations are double for MPF_F64 and MPF_MIXED, float for MPF_F32 and
// MPF_F32_KAHAN.
template <int Q, typename F>
int with_state(int precision, F&& fn) {
  if (state_is_f32(precision)) return fn(float{});
  if (precision == MPF_F64 || precision == MPF_MIXED) return fn(double{});
  return MPF_ERR_ARG;
}

template <typename F>
int with_q(int q, F&& fn) {
  if (q == 19) return fn(std::integral_constant<int, 19>{});
  if (q == 15) return fn(std::integral_constant<int, 15>{});
  return MPF_ERR_ARG;
}

}  // namespace
}  // namespace mpf

extern "C" int mpf_lbm_init(const mpf_lbm_params* prm, int64_t n, double rho, const double* u_host, void* f,
                            void* stream) {
  using namespace mpf;
  if (!prm || !f || !u_host || n < 1) return MPF_ERR_ARG;
  hipStream_t st = as_stream(stream);
  const unsigned g = grid_for(n, kBlock);
  const double u0 = u_host[0], u1 = u_host[1], u2 = u_host[2];
  return with_q(prm->q, [&](auto qc) {
    constexpr int Q = decltype(qc)::value;
    return with_state<Q>(prm->precision, [&](auto t) {
      using T = decltype(t);
      hipLaunchKernelGGL((lbm_init<T, Q>), dim3(g), dim3(kBlock), 0, st, n, (T*)f, rho, u0, u1, u2);
      MPF_LAUNCH_CHECK();
      return MPF_OK;
    });
  });
}

extern "C" int mpf_lbm_init_fields(const mpf_lbm_params* prm, int64_t n, const double* v, const double* p,
                                   double vel_scale, void* f, void* stream) {
  using namespace mpf;
  if (!prm || !f || !v || !p || n < 1 || !(vel_scale > 0.0)) return MPF_ERR_ARG;
  hipStream_t st = as_stream(stream);
  const unsigned g = grid_for(n, kBlock);
  return with_q(prm->q, [&](auto qc) {
    constexpr int Q = decltype(qc)::value;
    return with_state<Q>(prm->precision, [&](auto t) {
      using T = decltype(t);
      hipLaunchKernelGGL((lbm_init_fields<T, Q>), dim3(g), dim3(kBlock), 0, st, n, v, p, vel_scale, (T*)f);
      MPF_LAUNCH_CHECK();
      return MPF_OK;
    });
  });
}

extern "C" int mpf_lbm_run(const mpf_lbm_params* prm, int64_t n, int64_t n_int, int nl, const int32_t* sten,
                           const void* W, const uint32_t* unknown, const mpf_tiles* tiles, void* f, void* f_tmp,
                           void* comp, uint32_t* flags, int n_steps, void* stream) {
  using namespace mpf;
  if (!prm || !sten || !W || !f || !f_tmp || n < 1 || n_int < 0 || n_int > n || nl < 1 || n_steps < 0)
    return MPF_ERR_ARG;
  if (n > n_int && !unknown) return MPF_ERR_ARG;
  if (!(prm->tau_plus > 0.5) || !(prm->tau_minus > 0.5)) return MPF_ERR_ARG;
  if (!precision_ok(prm->precision)) return MPF_ERR_ARG;
  if ((prm->precision == MPF_F32_KAHAN) != (comp != nullptr)) return MPF_ERR_ARG;
  if (tiles && (!tiles->count || !tiles->halo || !tiles->lidx || tiles->h_cap < 64 || tiles->h_max < 1 ||
                tiles->h_max > tiles->h_cap || (tiles->tile != 0 && tiles->tile != kTile)))
    return MPF_ERR_ARG;
  if (n_steps == 0) return MPF_OK;
  hipStream_t st = as_stream(stream);
  return with_q(prm->q, [&](auto qc) {
    constexpr int Q = decltype(qc)::value;
    if (prm->precision == MPF_F64)
      return run<double, double, Q, false>(prm, n, n_int, nl, sten, (const double*)W, unknown, tiles, (double*)f,
                                           (double*)f_tmp, nullptr, flags, n_steps, st);
    if (prm->precision == MPF_MIXED)
      return run<float, double, Q, false>(prm, n, n_int, nl, sten, (const float*)W, unknown, tiles, (double*)f,
                                          (double*)f_tmp, nullptr, flags, n_steps, st);
    if (prm->precision == MPF_F32_KAHAN)
      return run<float, float, Q, true>(prm, n, n_int, nl, sten, (const float*)W, unknown, tiles, (float*)f, (float*)f_tmp,
                                        (float*)comp, flags, n_steps, st);
    return run<float, float, Q, false>(prm, n, n_int, nl, sten, (const float*)W, unknown, tiles, (float*)f, (float*)f_tmp,
                                       nullptr, flags, n_steps, st);
  });
}

extern "C" int mpf_lbm_unknown(int q, int64_t n, int64_t n_int, const double* pos, const double* nrm, int rule,
                               double dx, double r, uint32_t* unknown, void* stream) {
  using namespace mpf;
  if (n < 1 || n_int < 0 || n_int > n) return MPF_ERR_ARG;
  const int64_t nb = n - n_int;
  if (nb == 0) return MPF_OK;
  if (!unknown) return MPF_ERR_ARG;
  if (rule == MPF_UNKNOWN_NORMAL) {
    if (!nrm) return MPF_ERR_ARG;
  } else if (rule == MPF_UNKNOWN_SOLID) {
    if (!pos || !(dx > 0.0 && dx < 0.5) || !(r > 0.0)) return MPF_ERR_ARG;
  } else {
    return MPF_ERR_ARG;
  }
  hipStream_t st = as_stream(stream);
  const unsigned g = grid_for(nb, kBlock);
  return with_q(q, [&](auto qc) {
    constexpr int Q = decltype(qc)::value;
    hipLaunchKernelGGL((lbm_unknown<Q>), dim3(g), dim3(kBlock), 0, st, nb, n, n_int, pos, nrm, rule, dx, r, unknown);
    MPF_LAUNCH_CHECK();
    return MPF_OK;
  });
}

extern "C" int mpf_lbm_moments(const mpf_lbm_params* prm, int64_t n, const void* f, const void* comp,
                               double vel_scale, double* v, double* p, void* stream) {
  using namespace mpf;
  if (!prm || !f || !v || n < 1) return MPF_ERR_ARG;
  if (comp && prm->precision != MPF_F32_KAHAN) return MPF_ERR_ARG;
  hipStream_t st = as_stream(stream);
  const unsigned g = grid_for(n, kBlock);
  return with_q(prm->q, [&](auto qc) {
    constexpr int Q = decltype(qc)::value;
    return with_state<Q>(prm->precision, [&](auto t) {
      using T = decltype(t);
      hipLaunchKernelGGL((lbm_moments<T, Q>), dim3(g), dim3(kBlock), 0, st, n, (const T*)f, (const T*)comp,
                         vel_scale, v, p);
      MPF_LAUNCH_CHECK();
      return MPF_OK;
    });
  });
}
