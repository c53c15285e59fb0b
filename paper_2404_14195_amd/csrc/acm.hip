// Artificial-compressibility Navier-Stokes steps (Sec. 2.3, Eqs.
// MNS_intermediate, MNS_pressure, MNS_velocity, MNS_C) on gfx950.
//
// Every pass is a stencil apply: weights and stencil indices are stored
// [op][j][node], field values are gathered through the caches (nodes are
// Morton ordered; a run keeps v and v' as node records [n][4], so a gathered
// velocity is one record).  A step is 1 + 3 n_p dependent passes:
//   predictor  (interior)     v' from v: 4 operators x 3 components
//   n_p x { pressure (interior)  p -= dt C^2 rho div v
//           neumann  (boundary)  p_b from dp/dn = 0, in place (its stencil
//                                holds only interior neighbours)
//           velocity (interior)  v = v' - dt/rho grad p, max |v| }
// With the entropically damped pressure equation (Sec. 2.3 names it as the
// remedy for the oscillations of Sec. 3.6) the pressure pass also gathers p:
//   p <- p + dt (-C^2 rho div v - v . grad p + nu lap p),
// reading the old pressure and writing a second buffer (Jacobi); the buffers
// alternate from pass to pass.
// C is never stored: each pressure pass derives it from the running max |v|
// (device double, updated with an integer atomicMax on the bit pattern, which
// orders non-negative doubles), so no host round trip enters a step.
//
// Compensated FP32 state (MPF_F32_KAHAN): every interior value carries an
// FP32 compensation term (v and v' as records [n][4] beside the value
// records, p as a plain array), gathered by nobody but its own node.  The
// predictor adds dt R to v_hi + v_lo, the pressure pass -coef div v to
// p_hi + p_lo, the velocity pass -dt/rho grad p to v'_hi + v'_lo, each with
// the error-free two-sum of Knuth, so that an increment below half an ulp of
// the FP32 value moves lo instead of vanishing; the stencil sums themselves
// read the FP32 values only, as in MPF_F32.
//
// Each node's stencil sum is split over LPN adjacent lanes (lane sl takes
// columns sl, sl + LPN, ...) and closed with a fixed butterfly, which shortens
// the chain of dependent gathers per lane.  One launch per pass: measured on
// the 8k-node cell, a persistent cooperative kernel with grid barriers between
// passes and a replayed HIP graph were both slower than plain launches once
// the gather chain was split 8 ways (126 -> 50 us per step).
#include "common.hpp"
#include "graph.hpp"

namespace mpf {
namespace {

constexpr int kBlock = 256;
constexpr int kTile = 64;  // nodes per tile of a plan that does not say (mpf_tile_plan)
// cells whose long runs replay a captured graph: on the 8k-node cell the
// step drops 8 % (41.0 -> 37.8 us FP32), on the 71k-node one it is 1 % slower
constexpr int64_t kGraphNodes = 50000;
constexpr int kGraphSteps = 16;

template <int LPN, typename T>
__device__ __forceinline__ T group_sum(T x) {
#pragma unroll
  for (int off = LPN / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// body(j) for the columns j = j0 + sl, j0 + sl + LPN, ... below nl, in
// ascending order; fully unrolled when the stencil size is a compile-time
// constant, so every lane issues all its index, weight and gather loads early.
template <int LPN, int NLC, typename Body>
__device__ __forceinline__ void columns(int nl, int j0, int sl, Body&& body) {
  if constexpr (NLC > 0) {
#pragma unroll
    for (int t = 0; t < (NLC + LPN - 1) / LPN; ++t) {
      const int j = j0 + sl + t * LPN;
      if (j < NLC) body(j);
    }
  } else {
    for (int j = j0 + sl; j < nl; j += LPN) body(j);
  }
}

// Velocity records [n][4] = (x, y, z, 0): a gathered neighbour costs one
// 16-byte (FP32) or two 16-byte (FP64) loads from one line instead of three
// loads from three lines of a [3][n] layout.
template <typename T>
struct Rec;
template <>
struct Rec<float> {
  using type = float4;
};
template <>
struct Rec<double> {
  using type = double4;
};

template <typename T>
__device__ __forceinline__ typename Rec<T>::type load4(const T* __restrict__ R, int64_t i) {
  return reinterpret_cast<const typename Rec<T>::type*>(R)[i];
}

template <typename T>
__device__ __forceinline__ void store4(T* __restrict__ R, int64_t i, T x, T y, T z) {
  typename Rec<T>::type r;
  r.x = x;
  r.y = y;
  r.z = z;
  r.w = T(0);
  reinterpret_cast<typename Rec<T>::type*>(R)[i] = r;
}

template <typename T>
__global__ void to_records(int64_t n, const T* __restrict__ v, T* __restrict__ R) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) store4(R, i, v[i], v[n + i], v[2 * n + i]);
}

template <typename T>
__global__ void from_records(int64_t n, const T* __restrict__ R, T* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const auto r = load4(R, i);
  v[i] = r.x;
  v[n + i] = r.y;
  v[2 * n + i] = r.z;
}

template <typename T, typename TW>
struct Fields {
  int64_t n, n_int, nb;
  int nl;
  const int32_t* sten;
  const TW* w;  // [4][nl][n]
  const int32_t* sn;
  const TW* wn;  // [nl][nb]
  T* V;         // [n][4] velocity records (x, y, z, 0), the run's working copy of v
  T* p;         // [n] the caller's pressure
  T* P1;        // [n] second pressure buffer (damped pressure equation only)
  T* VP;        // [n][4] v' records
  T* VL;        // [n][4] compensation of V (compensated state only, else null)
  T* VPL;       // [n][4] compensation of VP
  T* PL;        // [n] compensation of p (the caller's comp row 3)
  double* vmax;
  uint32_t* flags;  // or null
  T nu, dt, dt_rho, g0, g1, g2;
  double dtd, rho, beta, v_ref;
  double dt_h;  // dt / h_min for the Courant check, 0 for none
};

// Knuth's two-sum: s + e == a + b exactly, s = fl(a + b).  Only additions, so
// no contraction into fused multiply-adds can change it.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// The node functions read a stencil neighbour's velocity record or pressure
// through gv(at) / gp(at), at = j n + i the stencil entry: from memory
// through the caches (sten), or from the tile's halo in LDS (staged).
template <typename T, typename TW, int LPN, int NLC, bool KAHAN, typename GV>
__device__ __forceinline__ void predictor_node(const Fields<T, TW>& F, int64_t i, int sl, GV&& gv) {
  const int nl = NLC ? NLC : F.nl;  // a constant for the common stencil size
  const int64_t n = F.n, os = (int64_t)nl * n;
  T d[3][4];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int o = 0; o < 4; ++o) d[a][o] = T(0);
  columns<LPN, NLC>(nl, 0, sl, [&](int j) {
    const int64_t at = (int64_t)j * n + i;
    const T wx = (T)F.w[at], wy = (T)F.w[os + at], wz = (T)F.w[2 * os + at], wl = (T)F.w[3 * os + at];
    const auto r = gv(at);  // one node's velocity: one record, one or two vector loads
    const T u[3] = {r.x, r.y, r.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      d[a][0] += wx * u[a];
      d[a][1] += wy * u[a];
      d[a][2] += wz * u[a];
      d[a][3] += wl * u[a];
    }
  });
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int o = 0; o < 4; ++o) d[a][o] = group_sum<LPN>(d[a][o]);
  if (sl == 0) {
    const auto ri = load4(F.V, i);
    const T vi[3] = {ri.x, ri.y, ri.z};
    const T g[3] = {F.g0, F.g1, F.g2};
    T out[3];
    if constexpr (KAHAN) {
      const auto rl = load4(F.VL, i);
      const T lo[3] = {rl.x, rl.y, rl.z};
      T ol[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const T adv = vi[0] * d[a][0] + vi[1] * d[a][1] + vi[2] * d[a][2];
        two_sum(vi[a], lo[a] + F.dt * (F.nu * d[a][3] - adv + g[a]), out[a], ol[a]);
      }
      store4(F.VPL, i, ol[0], ol[1], ol[2]);
    } else {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const T adv = vi[0] * d[a][0] + vi[1] * d[a][1] + vi[2] * d[a][2];
        out[a] = vi[a] + F.dt * (F.nu * d[a][3] - adv + g[a]);
      }
    }
    store4(F.VP, i, out[0], out[1], out[2]);
  }
}

template <typename T, typename TW, int LPN, int NLC, bool KAHAN, typename GV>
__device__ __forceinline__ void pressure_node(const Fields<T, TW>& F, const T* pin, T* pout, T coef, int64_t i,
                                              int sl, GV&& gv) {
  const int nl = NLC ? NLC : F.nl;  // a constant for the common stencil size
  const int64_t n = F.n, os = (int64_t)nl * n;
  T div = T(0);
  columns<LPN, NLC>(nl, 0, sl, [&](int j) {
    const int64_t at = (int64_t)j * n + i;
    const auto r = gv(at);
    div += (T)F.w[at] * r.x + (T)F.w[os + at] * r.y + (T)F.w[2 * os + at] * r.z;
  });
  div = group_sum<LPN>(div);
  if (sl != 0) return;
  if constexpr (KAHAN) {
    T hi, lo;
    two_sum(pin[i], F.PL[i] - coef * div, hi, lo);
    pout[i] = hi;
    F.PL[i] = lo;
  } else {
    pout[i] = pin[i] - coef * div;  // in place (pin == pout) for the plain method
  }
}

// The damped pressure equation: p_new = p - coef div v - dt v_i . grad p + dt nu lap p.
template <typename T, typename TW, int LPN, int NLC, bool KAHAN, typename GV, typename GP>
__device__ __forceinline__ void pressure_edac_node(const Fields<T, TW>& F, const T* __restrict__ vsrc,
                                                   const T* __restrict__ pin, T* __restrict__ pout, T coef,
                                                   int64_t i, int sl, GV&& gv, GP&& gp) {
  const int nl = NLC ? NLC : F.nl;
  const int64_t n = F.n, os = (int64_t)nl * n;
  T div = T(0), gx = T(0), gy = T(0), gz = T(0), lp = T(0);
  columns<LPN, NLC>(nl, 0, sl, [&](int j) {
    const int64_t at = (int64_t)j * n + i;
    const T wx = (T)F.w[at], wy = (T)F.w[os + at], wz = (T)F.w[2 * os + at], wl = (T)F.w[3 * os + at];
    const auto r = gv(at);
    const T ps = gp(at);
    div += wx * r.x + wy * r.y + wz * r.z;
    gx += wx * ps;
    gy += wy * ps;
    gz += wz * ps;
    lp += wl * ps;
  });
  div = group_sum<LPN>(div);
  gx = group_sum<LPN>(gx);
  gy = group_sum<LPN>(gy);
  gz = group_sum<LPN>(gz);
  lp = group_sum<LPN>(lp);
  if (sl == 0) {
    const auto ri = load4(vsrc, i);
    const T adv = ri.x * gx + ri.y * gy + ri.z * gz;
    if constexpr (KAHAN) {
      T hi, lo;
      two_sum(pin[i], F.PL[i] - coef * div + F.dt * (F.nu * lp - adv), hi, lo);
      pout[i] = hi;
      F.PL[i] = lo;
    } else {
      pout[i] = pin[i] - coef * div + F.dt * (F.nu * lp - adv);
    }
  }
}

template <typename T, typename TW, int LPN, int NLC>
__device__ __forceinline__ void neumann_node(const Fields<T, TW>& F, T* P, int64_t b, int sl) {
  const int nl = NLC ? NLC : F.nl;  // a constant for the common stencil size
  T s = T(0);
  columns<LPN, NLC>(nl, 1, sl, [&](int j) {
    const int64_t at = (int64_t)j * F.nb + b;
    s += (T)F.wn[at] * P[F.sn[at]];
  });
  s = group_sum<LPN>(s);
  if (sl == 0) P[F.n_int + b] = -s / (T)F.wn[b];
}

// returns |v_i| (valid in every lane of the node's group)
template <typename T, typename TW, int LPN, int NLC, bool KAHAN, typename GP>
__device__ __forceinline__ double velocity_node(const Fields<T, TW>& F, int64_t i, int sl, GP&& gpres) {
  const int nl = NLC ? NLC : F.nl;  // a constant for the common stencil size
  const int64_t n = F.n, os = (int64_t)nl * n;
  T gp[3] = {T(0), T(0), T(0)};
  columns<LPN, NLC>(nl, 0, sl, [&](int j) {
    const int64_t at = (int64_t)j * n + i;
    const T ps = gpres(at);
    gp[0] += (T)F.w[at] * ps;
    gp[1] += (T)F.w[os + at] * ps;
    gp[2] += (T)F.w[2 * os + at] * ps;
  });
  double m2 = 0.0;
  const auto rp = load4(F.VP, i);
  const T vpi[3] = {rp.x, rp.y, rp.z};
  T va[3];
  if constexpr (KAHAN) {
    const auto rl = load4(F.VPL, i);
    const T lo[3] = {rl.x, rl.y, rl.z};
    T vl[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      gp[a] = group_sum<LPN>(gp[a]);
      two_sum(vpi[a], lo[a] - F.dt_rho * gp[a], va[a], vl[a]);
      m2 += (double)va[a] * (double)va[a];
    }
    if (sl == 0) store4(F.VL, i, vl[0], vl[1], vl[2]);
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      gp[a] = group_sum<LPN>(gp[a]);
      va[a] = vpi[a] - F.dt_rho * gp[a];
      m2 += (double)va[a] * (double)va[a];
    }
  }
  if (sl == 0) store4(F.V, i, va[0], va[1], va[2]);
  return sqrt(m2);
}

// C from the running max; the first thread of the launch also raises flags
// bit 1 when the pressure waves' Courant number C dt / h_min exceeds 1.
template <typename T, typename TW>
__device__ __forceinline__ T coupling_coef(const Fields<T, TW>& F) {
  const double vm = *F.vmax;
  const double C = F.beta * (vm > F.v_ref ? vm : F.v_ref);
  if (F.flags && F.dt_h > 0.0 && blockIdx.x == 0 && threadIdx.x == 0 && C * F.dt_h > 1.0)
    atomicOr(F.flags, MPF_FLAG_LIMIT);
  return (T)(F.dtd * (C * C) * F.rho);
}

// Block max of |v| into the running max (exact, so any order gives the same).
// A NaN magnitude is taken as +inf before the reduction (fmax would drop it),
// so a non-finite state always shows up as C = inf, and as flags bit 0.
__device__ __forceinline__ void block_max_into(double mag, double* lds, double* vmax, uint32_t* flags) {
  if (!(mag <= __builtin_huge_val())) mag = __builtin_huge_val();
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mag = fmax(mag, __shfl_xor(mag, off));
  if ((threadIdx.x & (kWave - 1)) == 0) lds[threadIdx.x / kWave] = mag;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = lds[0];
    for (int t = 1; t < (int)(blockDim.x / kWave); ++t) m = fmax(m, lds[t]);
    if (flags && !(m < __builtin_huge_val())) atomicOr(flags, MPF_FLAG_NONFINITE);
    atomicMax(reinterpret_cast<unsigned long long*>(vmax), (unsigned long long)__double_as_longlong(m));
  }
  __syncthreads();
}

// ---------------------------------------------------------------- one launch per pass

template <typename T, typename TW, int LPN, int NLC, bool KAHAN>
__global__ __launch_bounds__(kBlock) void k_predictor(Fields<T, TW> F) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = g / LPN;
  if (i >= F.n_int) return;  // whole LPN groups exit together
  predictor_node<T, TW, LPN, NLC, KAHAN>(F, i, (int)(g % LPN), [&](int64_t at) { return load4(F.V, F.sten[at]); });
}

template <typename T, typename TW, int LPN, int NLC, bool KAHAN>
__global__ __launch_bounds__(kBlock) void k_pressure(Fields<T, TW> F, const T* __restrict__ vsrc, T* P) {
  const T coef = coupling_coef(F);
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = g / LPN;
  if (i >= F.n_int) return;
  pressure_node<T, TW, LPN, NLC, KAHAN>(F, P, P, coef, i, (int)(g % LPN),
                                        [&](int64_t at) { return load4(vsrc, F.sten[at]); });
}

template <typename T, typename TW, int LPN, int NLC, bool KAHAN>
__global__ __launch_bounds__(kBlock) void k_pressure_edac(Fields<T, TW> F, const T* __restrict__ vsrc,
                                                          const T* __restrict__ pin, T* __restrict__ pout) {
  const T coef = coupling_coef(F);
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = g / LPN;
  if (i >= F.n_int) return;
  pressure_edac_node<T, TW, LPN, NLC, KAHAN>(F, vsrc, pin, pout, coef, i, (int)(g % LPN),
                                             [&](int64_t at) { return load4(vsrc, F.sten[at]); },
                                             [&](int64_t at) { return pin[F.sten[at]]; });
}

template <typename T, typename TW, int LPN, int NLC>
__global__ __launch_bounds__(kBlock) void k_neumann(Fields<T, TW> F, T* P) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g == 0) *F.vmax = 0.0;  // the pressure pass has consumed it; the velocity pass rebuilds it
  const int64_t b = g / LPN;
  if (b >= F.nb) return;
  neumann_node<T, TW, LPN, NLC>(F, P, b, (int)(g % LPN));
}

template <typename T, typename TW, int LPN, int NLC, bool KAHAN>
__global__ __launch_bounds__(kBlock) void k_velocity(Fields<T, TW> F, const T* __restrict__ P) {
  __shared__ double red[kBlock / kWave];
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t i = g / LPN;
  double mag = 0.0;
  if (i < F.n_int)
    mag = velocity_node<T, TW, LPN, NLC, KAHAN>(F, i, (int)(g % LPN), [&](int64_t at) { return P[F.sten[at]]; });
  block_max_into(mag, red, F.vmax, F.flags);
}

// ---------------------------------------------------------------- LDS-staged gather
// A tile of the tile plan is 64 consecutive nodes (mpf_tile_plan): one wave
// at one lane per node, two waves at two.  The tile's threads first copy its
// halo (the tile's distinct stencil nodes, ascending) from the gathered field
// into LDS with contiguous loads, then read every neighbour value from LDS
// through its 16-bit position lidx[j][i].  The summation order is that of the
// cached gather, so results are the same bit for bit.

struct Halo {
  const int32_t* count;
  const int32_t* halo;
  const uint16_t* lidx;
  int h_cap;
  int h_max;
  int tile;  // nodes per tile: 64, 128 or 256
};

// the tile's halo values of src into dst (this tile's LDS), four entries per
// thread in flight; the tile's gt threads share the copy (entries past the
// halo load a valid one and are not stored; named temporaries, so that
// nothing is placed in scratch)
template <typename R>
__device__ __forceinline__ void stage_halo(const Halo& H, int64_t tile, const R* __restrict__ src, R* dst, int t,
                                           int gt) {
  const int cnt = H.count[tile];
  const int32_t* hl = H.halo + tile * H.h_cap;
  for (int c0 = t; c0 < cnt; c0 += 4 * gt) {
    const int c1 = c0 + gt, c2 = c0 + 2 * gt, c3 = c0 + 3 * gt;
    const int i0 = hl[c0];
    const int i1 = hl[c1 < cnt ? c1 : c0];
    const int i2 = hl[c2 < cnt ? c2 : c0];
    const int i3 = hl[c3 < cnt ? c3 : c0];
    const R v0 = src[i0], v1 = src[i1], v2 = src[i2], v3 = src[i3];
    dst[c0] = v0;
    if (c1 < cnt) dst[c1] = v1;
    if (c2 < cnt) dst[c2] = v2;
    if (c3 < cnt) dst[c3] = v3;
  }
}

// Thread layout of a staged pass with LPN lanes per node: a tile of ts nodes
// (64, 128 or 256, ts LPN <= kBlock) is gt = ts LPN consecutive threads; a
// block holds kBlock / gt tiles, each with h_max halo values in LDS.
template <int LPN>
struct StagedIdx {
  int64_t g, i, tile;
  int sl, t, slot, gt;
  __device__ explicit StagedIdx(int ts) {
    const int lg = __builtin_ctz((unsigned)ts);  // ts is a power of two
    gt = ts * LPN;
    g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    i = g / LPN;
    sl = (int)(g % LPN);
    tile = i >> lg;
    t = threadIdx.x & (gt - 1);
    slot = threadIdx.x >> (lg + (LPN == 2 ? 1 : 0));
  }
};

template <typename T, typename TW, int LPN, int NLC, bool KAHAN>
__global__ __launch_bounds__(kBlock) void k_predictor_st(Fields<T, TW> F, Halo H) {
  using R = typename Rec<T>::type;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const StagedIdx<LPN> x(H.tile);
  R* hv = reinterpret_cast<R*>(lds_raw) + x.slot * H.h_max;
  if (x.tile * H.tile < F.n_int) stage_halo(H, x.tile, reinterpret_cast<const R*>(F.V), hv, x.t, x.gt);
  __syncthreads();
  if (x.i >= F.n_int) return;
  predictor_node<T, TW, LPN, NLC, KAHAN>(F, x.i, x.sl, [&](int64_t at) { return hv[H.lidx[at]]; });
}

template <typename T, typename TW, int LPN, int NLC, bool KAHAN>
__global__ __launch_bounds__(kBlock) void k_pressure_st(Fields<T, TW> F, const T* __restrict__ vsrc, T* P, Halo H) {
  using R = typename Rec<T>::type;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const T coef = coupling_coef(F);
  const StagedIdx<LPN> x(H.tile);
  R* hv = reinterpret_cast<R*>(lds_raw) + x.slot * H.h_max;
  if (x.tile * H.tile < F.n_int) stage_halo(H, x.tile, reinterpret_cast<const R*>(vsrc), hv, x.t, x.gt);
  __syncthreads();
  if (x.i >= F.n_int) return;
  pressure_node<T, TW, LPN, NLC, KAHAN>(F, P, P, coef, x.i, x.sl, [&](int64_t at) { return hv[H.lidx[at]]; });
}

template <typename T, typename TW, int LPN, int NLC, bool KAHAN>
__global__ __launch_bounds__(kBlock) void k_pressure_edac_st(Fields<T, TW> F, const T* __restrict__ vsrc,
                                                             const T* __restrict__ pin, T* __restrict__ pout,
                                                             Halo H) {
  using R = typename Rec<T>::type;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const T coef = coupling_coef(F);
  const StagedIdx<LPN> x(H.tile);
  const int tiles = kBlock / x.gt;
  R* hv = reinterpret_cast<R*>(lds_raw) + x.slot * H.h_max;
  T* hp = reinterpret_cast<T*>(reinterpret_cast<R*>(lds_raw) + tiles * H.h_max) + x.slot * H.h_max;
  if (x.tile * H.tile < F.n_int) {
    stage_halo(H, x.tile, reinterpret_cast<const R*>(vsrc), hv, x.t, x.gt);
    stage_halo(H, x.tile, pin, hp, x.t, x.gt);
  }
  __syncthreads();
  if (x.i >= F.n_int) return;
  pressure_edac_node<T, TW, LPN, NLC, KAHAN>(F, vsrc, pin, pout, coef, x.i, x.sl,
                                             [&](int64_t at) { return hv[H.lidx[at]]; },
                                             [&](int64_t at) { return hp[H.lidx[at]]; });
}

template <typename T, typename TW, int LPN, int NLC, bool KAHAN>
__global__ __launch_bounds__(kBlock) void k_velocity_st(Fields<T, TW> F, const T* __restrict__ P, Halo H) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ double red[kBlock / kWave];
  const StagedIdx<LPN> x(H.tile);
  T* hp = reinterpret_cast<T*>(lds_raw) + x.slot * H.h_max;
  if (x.tile * H.tile < F.n_int) stage_halo(H, x.tile, P, hp, x.t, x.gt);
  __syncthreads();
  double mag = 0.0;
  if (x.i < F.n_int)
    mag = velocity_node<T, TW, LPN, NLC, KAHAN>(F, x.i, x.sl, [&](int64_t at) { return hp[H.lidx[at]]; });
  block_max_into(mag, red, F.vmax, F.flags);
}

template <typename T>
__global__ void copy_field(int64_t n, const T* __restrict__ src, T* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

template <typename T>
__global__ void fill_zero(T* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] = T(0);
}

// Lanes per node when the caller leaves the choice to the library, from a
// sweep over cells of 2k to 1.8M nodes (N_L = 30, every precision).  Only a
// pass too small to fill the chip gains from splitting each stencil 8 ways
// (the dependent gather chain of one node is then the bound); from a few
// tens of thousands of nodes on, the split's idle lanes and butterflies cost
// more than they hide, and one lane per node wins (FP32 on 1.8M nodes: 1.43
// vs 1.54 ms at 2 lanes; all precisions at 71k and 219k nodes, 2.4x over 8
// lanes at 219k).  FP64 state records (32 bytes per gathered node) prefer 2
// lanes again on the largest cells (1.8M nodes: 2.52 vs 2.69 ms FP64).
template <typename T>
int default_lanes(int64_t n_int) {
  if (n_int <= 12000) return 8;
  if (n_int <= 50000) return 2;
  if (sizeof(T) == sizeof(double) && n_int > 500000) return 2;
  return 1;
}

// The staged passes (H from the tile plan; LDS: each of the block's
// kBlock / (64 LPN) tiles holds h_max halo values).
template <typename T, typename TW, int LPN, int NLC, bool KAHAN>
int run_staged(Fields<T, TW>& F, const Halo& H, int n_steps, int n_p, bool edac, hipStream_t st) {
  using R = typename Rec<T>::type;
  const unsigned gi = grid_for(F.n_int * LPN, kBlock), gb = grid_for(F.nb * LPN, kBlock);
  const size_t tiles = kBlock / (H.tile * LPN);
  const size_t lv = tiles * H.h_max * sizeof(R), lp = tiles * H.h_max * sizeof(T);
  T* cur = F.p;
  for (int s = 0; s < n_steps; ++s) {
    hipLaunchKernelGGL((k_predictor_st<T, TW, LPN, NLC, KAHAN>), dim3(gi), dim3(kBlock), lv, st, F, H);
    for (int it = 0; it < n_p; ++it) {
      const T* vsrc = it == 0 ? F.VP : F.V;
      if (edac) {
        T* nxt = cur == F.p ? F.P1 : F.p;
        hipLaunchKernelGGL((k_pressure_edac_st<T, TW, LPN, NLC, KAHAN>), dim3(gi), dim3(kBlock), lv + lp, st, F,
                           vsrc, (const T*)cur, nxt, H);
        cur = nxt;
      } else {
        hipLaunchKernelGGL((k_pressure_st<T, TW, LPN, NLC, KAHAN>), dim3(gi), dim3(kBlock), lv, st, F, vsrc, cur, H);
      }
      hipLaunchKernelGGL((k_neumann<T, TW, LPN, NLC>), dim3(gb), dim3(kBlock), 0, st, F, cur);
      hipLaunchKernelGGL((k_velocity_st<T, TW, LPN, NLC, KAHAN>), dim3(gi), dim3(kBlock), lp, st, F, (const T*)cur,
                         H);
    }
  }
  if (cur != F.p)
    hipLaunchKernelGGL(copy_field<T>, dim3(grid_for(F.n, kBlock)), dim3(kBlock), 0, st, F.n, (const T*)cur, F.p);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

// Staging is used with one or two lanes per node when the block's halos fit:
// its tiles' velocity records and pressures (the damped pressure pass holds
// both) in 64 KiB: halos of up to 819 nodes for FP32 at one lane (four tiles
// per block) and for FP64 at two (two tiles), 1,638 for FP32 at two lanes,
// 409 for FP64 at one (the refined clouds here: about 350 on average, 573 at
// most at N_L = 30, up to 1,100 at N_L = 50).
constexpr size_t kAcmHaloLds = 64 * 1024;

template <typename T>
bool halo_fits(int lanes, int h_max, int tile) {
  using R = typename Rec<T>::type;
  return (lanes == 1 || lanes == 2) && tile * lanes <= kBlock &&
         (size_t)(kBlock / (tile * lanes)) * (size_t)h_max * (sizeof(R) + sizeof(T)) <= kAcmHaloLds;
}

template <typename T, typename TW, int LPN, int NLC, bool KAHAN>
int run_launches(Fields<T, TW>& F, const Halo* H, int n_steps, int n_p, bool edac, hipStream_t st) {
  if constexpr (LPN <= 2) {
    if (H && halo_fits<T>(LPN, H->h_max, H->tile))
      return run_staged<T, TW, LPN, NLC, KAHAN>(F, *H, n_steps, n_p, edac, st);
  }
  const unsigned gi = grid_for(F.n_int * LPN, kBlock), gb = grid_for(F.nb * LPN, kBlock);
  T* cur = F.p;  // the pressure of the current iteration (alternates with F.P1 when damped)
  for (int s = 0; s < n_steps; ++s) {
    hipLaunchKernelGGL((k_predictor<T, TW, LPN, NLC, KAHAN>), dim3(gi), dim3(kBlock), 0, st, F);
    for (int it = 0; it < n_p; ++it) {
      const T* vsrc = it == 0 ? F.VP : F.V;
      if (edac) {
        T* nxt = cur == F.p ? F.P1 : F.p;
        hipLaunchKernelGGL((k_pressure_edac<T, TW, LPN, NLC, KAHAN>), dim3(gi), dim3(kBlock), 0, st, F, vsrc,
                           (const T*)cur, nxt);
        cur = nxt;
      } else {
        hipLaunchKernelGGL((k_pressure<T, TW, LPN, NLC, KAHAN>), dim3(gi), dim3(kBlock), 0, st, F, vsrc, cur);
      }
      hipLaunchKernelGGL((k_neumann<T, TW, LPN, NLC>), dim3(gb), dim3(kBlock), 0, st, F, cur);
      hipLaunchKernelGGL((k_velocity<T, TW, LPN, NLC, KAHAN>), dim3(gi), dim3(kBlock), 0, st, F, (const T*)cur);
    }
  }
  if (cur != F.p)
    hipLaunchKernelGGL(copy_field<T>, dim3(grid_for(F.n, kBlock)), dim3(kBlock), 0, st, F.n, (const T*)cur, F.p);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

// stencils of 30 nodes (the measured size) and of 25 (the paper's choice in
// its convergence study) get fully unrolled column loops, which lets every
// lane issue all its index, weight and gather loads early
template <typename T, typename TW, int LPN, bool KAHAN>
int launch_nl(Fields<T, TW>& F, const Halo* H, int n_steps, int n_p, bool edac, hipStream_t st) {
  if (F.nl == 30) return run_launches<T, TW, LPN, 30, KAHAN>(F, H, n_steps, n_p, edac, st);
  if (F.nl == 25) return run_launches<T, TW, LPN, 25, KAHAN>(F, H, n_steps, n_p, edac, st);
  return run_launches<T, TW, LPN, 0, KAHAN>(F, H, n_steps, n_p, edac, st);
}

template <typename T, typename TW, bool KAHAN>
int launch_lanes(Fields<T, TW>& F, const Halo* H, int lanes, int n_steps, int n_p, bool edac, hipStream_t st) {
  switch (lanes) {
    case 1: return launch_nl<T, TW, 1, KAHAN>(F, H, n_steps, n_p, edac, st);
    case 2: return launch_nl<T, TW, 2, KAHAN>(F, H, n_steps, n_p, edac, st);
    case 4: return launch_nl<T, TW, 4, KAHAN>(F, H, n_steps, n_p, edac, st);
    case 8: return launch_nl<T, TW, 8, KAHAN>(F, H, n_steps, n_p, edac, st);
    default: return launch_nl<T, TW, 16, KAHAN>(F, H, n_steps, n_p, edac, st);
  }
}

// comp (compensated state only): [4][n] floats, v_lo rows 0-2 and p_lo row 3
template <typename T, typename TW>
int run(const mpf_acm_params* prm, int64_t n, int64_t n_int, int nl, const int32_t* sten, const TW* w,
        const int32_t* sn, const TW* wn, const mpf_tiles* tiles, T* v, T* p, T* comp, double* vmax, uint32_t* flags,
        int n_steps, void* ws, hipStream_t st) {
  Fields<T, TW> F;
  F.n = n; F.n_int = n_int; F.nb = n - n_int; F.nl = nl;
  F.sten = sten; F.w = w; F.sn = sn; F.wn = wn; F.p = p;
  F.V = reinterpret_cast<T*>(ws);
  F.VP = F.V + 4 * n;
  F.P1 = F.VP + 4 * n;
  F.VL = comp ? F.P1 + n : nullptr;
  F.VPL = comp ? F.VL + 4 * n : nullptr;
  F.PL = comp ? comp + 3 * n : nullptr;
  F.vmax = vmax;
  F.flags = flags;
  F.nu = (T)prm->nu; F.dt = (T)prm->dt; F.dt_rho = (T)(prm->dt / prm->rho);
  F.g0 = (T)prm->g[0]; F.g1 = (T)prm->g[1]; F.g2 = (T)prm->g[2];
  F.dtd = prm->dt; F.rho = prm->rho; F.beta = prm->beta; F.v_ref = prm->v_ref;
  F.dt_h = prm->h_min > 0.0 ? prm->dt / prm->h_min : 0.0;
  // the run works on node records: v [3][n] -> V [n][4] now and back at the
  // end (likewise the compensation of v); v' is zero on the boundary for the
  // whole run
  const unsigned gn = grid_for(n, kBlock);
  hipLaunchKernelGGL(to_records<T>, dim3(gn), dim3(kBlock), 0, st, n, (const T*)v, F.V);
  hipLaunchKernelGGL(fill_zero<T>, dim3(grid_for(4 * n, kBlock)), dim3(kBlock), 0, st, F.VP, 4 * n);
  if (comp) {
    hipLaunchKernelGGL(to_records<T>, dim3(gn), dim3(kBlock), 0, st, n, (const T*)comp, F.VL);
    hipLaunchKernelGGL(fill_zero<T>, dim3(grid_for(4 * n, kBlock)), dim3(kBlock), 0, st, F.VPL, 4 * n);
  }
  const bool edac = prm->edac != 0;
  Halo hd{};
  const Halo* H = nullptr;
  if (tiles) {
    hd = Halo{tiles->count, tiles->halo, tiles->lidx, tiles->h_cap, tiles->h_max, tiles->tile ? tiles->tile : kTile};
    H = &hd;
  }
  int lanes = prm->lanes;
  if (lanes == 0) {
    lanes = default_lanes<T>(n_int);
    // a one-lane pass whose halos do not fit LDS gathers through the caches;
    // two lanes per node halve the tiles per block, and staged they beat it
    if (H && lanes == 1 && !halo_fits<T>(1, H->h_max, H->tile) && halo_fits<T>(2, H->h_max, H->tile)) lanes = 2;
  }
  // a step is 1 + 3 n_p launches; on cells of up to kGraphNodes nodes their
  // launch overhead is a large part of the step, and long runs replay a
  // captured graph of kGraphSteps steps
  auto steps = [&](int k, hipStream_t s) {
    if constexpr (sizeof(T) == sizeof(float))  // the compensated state is FP32
      return comp ? launch_lanes<T, TW, true>(F, H, lanes, k, prm->n_p, edac, s)
                  : launch_lanes<T, TW, false>(F, H, lanes, k, prm->n_p, edac, s);
    else
      return launch_lanes<T, TW, false>(F, H, lanes, k, prm->n_p, edac, s);
  };
  const int rc = run_steps(n_steps, n <= kGraphNodes ? kGraphSteps : 0, steps, st);
  if (rc) return rc;
  hipLaunchKernelGGL(from_records<T>, dim3(gn), dim3(kBlock), 0, st, n, (const T*)F.V, v);
  if (comp) hipLaunchKernelGGL(from_records<T>, dim3(gn), dim3(kBlock), 0, st, n, (const T*)F.VL, comp);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

}  // namespace
}  // namespace mpf

extern "C" int mpf_acm_dt(double h_min, double nu, double* dt_host) {
  if (!dt_host || !(h_min > 0.0) || !(nu > 0.0)) return MPF_ERR_ARG;
  *dt_host = 0.1 * h_min * h_min / (2.0 * nu);
  return MPF_OK;
}

extern "C" size_t mpf_acm_workspace(int64_t n, int precision) {
  if (n < 1) return 256;
  // V and V' records [n][4], a second pressure [n]; compensated: also the
  // compensation records of V and V' [n][4] each
  if (precision == MPF_F32_KAHAN) return 17 * (size_t)n * sizeof(float) + 256;
  const size_t es = precision == MPF_F32 ? sizeof(float) : sizeof(double);
  return 9 * (size_t)n * es + 256;
}

extern "C" int mpf_acm_run(const mpf_acm_params* prm, int64_t n, int64_t n_int, int nl, const int32_t* sten,
                           const void* w, const int32_t* sn, const void* wn, const mpf_tiles* tiles, void* v, void* p,
                           void* comp, double* vmax, uint32_t* flags, int n_steps, void* ws, size_t ws_bytes,
                           void* stream) {
  using namespace mpf;
  if (!prm || !sten || !w || !v || !p || !vmax || n < 1 || n_int < 0 || n_int > n || nl < 2 || n_steps < 0 ||
      prm->n_p < 1 || !(prm->dt > 0.0) || !(prm->rho > 0.0) || !(prm->h_min >= 0.0))
    return MPF_ERR_ARG;
  if (n > n_int && (!sn || !wn)) return MPF_ERR_ARG;
  const int prec = prm->precision;
  if (prec != MPF_F64 && prec != MPF_F32 && prec != MPF_MIXED && prec != MPF_F32_KAHAN) return MPF_ERR_ARG;
  if ((prec == MPF_F32_KAHAN) != (comp != nullptr)) return MPF_ERR_ARG;
  if (prm->edac != 0 && prm->edac != 1) return MPF_ERR_ARG;
  if (prm->lanes != 0 && prm->lanes != 1 && prm->lanes != 2 && prm->lanes != 4 && prm->lanes != 8 &&
      prm->lanes != 16)
    return MPF_ERR_ARG;
  if (tiles && (!tiles->count || !tiles->halo || !tiles->lidx || tiles->h_cap < 64 || tiles->h_max < 1 ||
                tiles->h_max > tiles->h_cap ||
                (tiles->tile != 0 && tiles->tile != 64 && tiles->tile != 128 && tiles->tile != 256)))
    return MPF_ERR_ARG;
  if (!ws || ws_bytes < mpf_acm_workspace(n, prec)) return MPF_ERR_WORKSPACE;
  if (n_steps == 0) return MPF_OK;
  hipStream_t st = as_stream(stream);
  int rc;
  if (prec == MPF_F64)
    rc = run<double, double>(prm, n, n_int, nl, sten, (const double*)w, sn, (const double*)wn, tiles, (double*)v,
                             (double*)p, nullptr, vmax, flags, n_steps, ws, st);
  else if (prec == MPF_MIXED)
    rc = run<double, float>(prm, n, n_int, nl, sten, (const float*)w, sn, (const float*)wn, tiles, (double*)v,
                            (double*)p, nullptr, vmax, flags, n_steps, ws, st);
  else
    rc = run<float, float>(prm, n, n_int, nl, sten, (const float*)w, sn, (const float*)wn, tiles, (float*)v,
                           (float*)p, (float*)comp, vmax, flags, n_steps, ws, st);
  if (rc) return rc;
  return check_flags(flags, st);
}
