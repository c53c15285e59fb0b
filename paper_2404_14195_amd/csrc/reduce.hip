// Permeability and drag reductions (Eqs. k_definition, stress_tensor_force,
// integration_force) and the library's host-side helpers.
//
// Sums are deterministic: every block reduces its items with a fixed-shape
// tree into one partial, and one block then adds the partials in a fixed
// order, so a rerun gives the same bits.  All accumulation is FP64 whatever
// the precision of the fields.
#include <mutex>

#include "common.hpp"

namespace mpf {

constexpr int kRBlock = 256;

__global__ __launch_bounds__(256) void finish_sum(const double* __restrict__ part, int64_t n, int stride,
                                                  double scale, double* __restrict__ out) {
  __shared__ double lds[256];
  double acc = 0.0;
  for (int64_t t = threadIdx.x; t < n; t += 256) acc += part[t * stride];
  double s = block_sum<256>(acc, lds);
  if (threadIdx.x == 0) *out = s * scale;
}

namespace {

template <typename T>
__global__ __launch_bounds__(kRBlock) void flux_partial(int64_t ns, int nl, const int32_t* __restrict__ idx,
                                                        const double* __restrict__ sw, const T* __restrict__ vx,
                                                        double* __restrict__ part) {
  __shared__ double lds[kRBlock];
  const int64_t s = (int64_t)blockIdx.x * kRBlock + threadIdx.x;
  double v = 0.0;
  if (s < ns) {
    for (int j = 0; j < nl; ++j) {
      const int64_t at = (int64_t)j * ns + s;
      v += sw[at] * (double)vx[idx[at]];
    }
  }
  const double b = block_sum<kRBlock>(v, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = b;
}

template <typename T>
__global__ __launch_bounds__(kRBlock) void sum_partial(int64_t n, const T* __restrict__ x,
                                                       double* __restrict__ part) {
  __shared__ double lds[kRBlock];
  const int64_t i = (int64_t)blockIdx.x * kRBlock + threadIdx.x;
  const double b = block_sum<kRBlock>(i < n ? (double)x[i] : 0.0, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = b;
}

// Traction sigma n at boundary node b, summed per block into part[3][nblk]
// (part may be NULL); when t_out is given, also written per node as
// t_out[3][nb], with the centred pressure in pc_out[nb].
template <typename T>
__global__ __launch_bounds__(kRBlock) void drag_partial(int64_t n, const T* __restrict__ v, const T* __restrict__ p,
                                                        int64_t nb, int nl, const int32_t* __restrict__ sb,
                                                        const double* __restrict__ wg,
                                                        const double* __restrict__ nrm,
                                                        const double* __restrict__ pmean, double rho_nu,
                                                        double* __restrict__ part, int64_t nblk,
                                                        double* __restrict__ t_out, double* __restrict__ pc_out) {
  __shared__ double lds[kRBlock];
  const int64_t b = (int64_t)blockIdx.x * kRBlock + threadIdx.x;
  double t[3] = {0.0, 0.0, 0.0};
  if (b < nb) {
    double G[3][3];  // G[c][a] = d v_c / d x_a
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < 3; ++a) G[c][a] = 0.0;
    const int64_t os = (int64_t)nl * nb;
    for (int j = 0; j < nl; ++j) {
      const int64_t at = (int64_t)j * nb + b;
      const int s = sb[at];
      const double u[3] = {(double)v[s], (double)v[n + s], (double)v[2 * n + s]};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double wa = wg[a * os + at];
#pragma unroll
        for (int c = 0; c < 3; ++c) G[c][a] += wa * u[c];
      }
    }
    const double pp = (double)p[sb[b]] - *pmean;
    const double nv[3] = {nrm[b], nrm[nb + b], nrm[2 * nb + b]};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double s = -pp * nv[c];
#pragma unroll
      for (int a = 0; a < 3; ++a) s += rho_nu * (G[c][a] + G[a][c]) * nv[a];
      t[c] = s;
    }
    if (t_out) {
#pragma unroll
      for (int c = 0; c < 3; ++c) t_out[c * nb + b] = t[c];
      pc_out[b] = pp;
    }
  }
  if (!part) return;  // block-uniform: the map alone needs no sums
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double bsum = block_sum<kRBlock>(t[c], lds);
    if (threadIdx.x == 0) part[c * nblk + blockIdx.x] = bsum;
  }
}

}  // namespace
}  // namespace mpf

using namespace mpf;

extern "C" size_t mpf_reduce_workspace(int64_t n_items) {
  const int64_t nblk = n_items > 0 ? (n_items + kRBlock - 1) / kRBlock : 1;
  return (size_t)(3 * nblk + 8) * sizeof(double) + 256;
}

namespace mpf {
namespace {
template <typename T>
__global__ void scale_kernel(int64_t n, T* __restrict__ x, T c) {
  const int64_t i = (int64_t)blockIdx.x * kRBlock + threadIdx.x;
  if (i < n) x[i] *= c;
}
}  // namespace
}  // namespace mpf

extern "C" int mpf_scale(int64_t n, void* x, int precision, double c, void* stream) {
  using namespace mpf;
  if (!x || n < 0) return MPF_ERR_ARG;
  if (precision != MPF_F64 && !state_is_f32(precision)) return MPF_ERR_ARG;
  if (n == 0) return MPF_OK;
  hipStream_t st = as_stream(stream);
  if (precision == MPF_F64)
    hipLaunchKernelGGL(scale_kernel<double>, dim3(grid_for(n, kRBlock)), dim3(kRBlock), 0, st, n, (double*)x, c);
  else
    hipLaunchKernelGGL(scale_kernel<float>, dim3(grid_for(n, kRBlock)), dim3(kRBlock), 0, st, n, (float*)x, (float)c);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

extern "C" int mpf_flux_planes(int64_t ns, int nl, const int32_t* s_idx, const double* s_w, const void* vx,
                               int precision, int64_t n_all, double* q_out, void* ws, size_t ws_bytes,
                               void* stream) {
  if (!q_out || ns < 0 || n_all < 1 || nl < 1 || (ns > 0 && (!s_idx || !s_w || !vx))) return MPF_ERR_ARG;
  if (!precision_ok(precision)) return MPF_ERR_ARG;
  if (!ws || ws_bytes < mpf_reduce_workspace(ns)) return MPF_ERR_WORKSPACE;
  hipStream_t st = as_stream(stream);
  double* part = reinterpret_cast<double*>(ws);
  const unsigned g = grid_for(ns, kRBlock);
  if (!state_is_f32(precision))
    hipLaunchKernelGGL(flux_partial<double>, dim3(g), dim3(kRBlock), 0, st, ns, nl, s_idx, s_w, (const double*)vx,
                       part);
  else
    hipLaunchKernelGGL(flux_partial<float>, dim3(g), dim3(kRBlock), 0, st, ns, nl, s_idx, s_w, (const float*)vx,
                       part);
  hipLaunchKernelGGL(finish_sum, dim3(1), dim3(256), 0, st, (const double*)part, (int64_t)g, 1, 1.0 / (double)n_all,
                     q_out);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

extern "C" int mpf_drag(int64_t n, const void* v, const void* p, int precision, int64_t nb, int nl,
                        const int32_t* sb, const double* wg, const double* nrm, double rho, double nu, double dA,
                        double* F_out, void* ws, size_t ws_bytes, void* stream) {
  if (!v || !p || !F_out || n < 1 || nb < 0 || nl < 1 || (nb > 0 && (!sb || !wg || !nrm))) return MPF_ERR_ARG;
  if (!precision_ok(precision)) return MPF_ERR_ARG;
  if (!ws || ws_bytes < mpf_reduce_workspace(n > nb ? n : nb)) return MPF_ERR_WORKSPACE;
  hipStream_t st = as_stream(stream);
  double* part = reinterpret_cast<double*>(ws);
  const int64_t nmax = n > nb ? n : nb;
  const int64_t cap = (nmax + kRBlock - 1) / kRBlock;
  double* pmean = part + 3 * cap;
  // node mean of p
  const unsigned gn = grid_for(n, kRBlock);
  if (!state_is_f32(precision))
    hipLaunchKernelGGL(sum_partial<double>, dim3(gn), dim3(kRBlock), 0, st, n, (const double*)p, part);
  else
    hipLaunchKernelGGL(sum_partial<float>, dim3(gn), dim3(kRBlock), 0, st, n, (const float*)p, part);
  hipLaunchKernelGGL(finish_sum, dim3(1), dim3(256), 0, st, (const double*)part, (int64_t)gn, 1, 1.0 / (double)n,
                     pmean);
  // tractions
  const unsigned gb = grid_for(nb, kRBlock);
  if (!state_is_f32(precision))
    hipLaunchKernelGGL(drag_partial<double>, dim3(gb), dim3(kRBlock), 0, st, n, (const double*)v, (const double*)p,
                       nb, nl, sb, wg, nrm, (const double*)pmean, rho * nu, part, (int64_t)gb, nullptr, nullptr);
  else
    hipLaunchKernelGGL(drag_partial<float>, dim3(gb), dim3(kRBlock), 0, st, n, (const float*)v, (const float*)p, nb,
                       nl, sb, wg, nrm, (const double*)pmean, rho * nu, part, (int64_t)gb, nullptr, nullptr);
  for (int c = 0; c < 3; ++c)
    hipLaunchKernelGGL(finish_sum, dim3(1), dim3(256), 0, st, (const double*)(part + c * gb), (int64_t)gb, 1, dA,
                       F_out + c);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

extern "C" int mpf_traction(int64_t n, const void* v, const void* p, int precision, int64_t nb, int nl,
                            const int32_t* sb, const double* wg, const double* nrm, double rho, double nu,
                            double* t_out, double* pc_out, void* ws, size_t ws_bytes, void* stream) {
  if (!v || !p || n < 1 || nb < 0 || nl < 1 || (nb > 0 && (!sb || !wg || !nrm || !t_out || !pc_out)))
    return MPF_ERR_ARG;
  if (!precision_ok(precision)) return MPF_ERR_ARG;
  if (!ws || ws_bytes < mpf_reduce_workspace(n > nb ? n : nb)) return MPF_ERR_WORKSPACE;
  if (nb == 0) return MPF_OK;
  hipStream_t st = as_stream(stream);
  double* part = reinterpret_cast<double*>(ws);
  const int64_t nmax = n > nb ? n : nb;
  const int64_t cap = (nmax + kRBlock - 1) / kRBlock;
  double* pmean = part + 3 * cap;
  const unsigned gn = grid_for(n, kRBlock);
  if (!state_is_f32(precision))
    hipLaunchKernelGGL(sum_partial<double>, dim3(gn), dim3(kRBlock), 0, st, n, (const double*)p, part);
  else
    hipLaunchKernelGGL(sum_partial<float>, dim3(gn), dim3(kRBlock), 0, st, n, (const float*)p, part);
  hipLaunchKernelGGL(finish_sum, dim3(1), dim3(256), 0, st, (const double*)part, (int64_t)gn, 1, 1.0 / (double)n,
                     pmean);
  const unsigned gb = grid_for(nb, kRBlock);
  if (!state_is_f32(precision))
    hipLaunchKernelGGL(drag_partial<double>, dim3(gb), dim3(kRBlock), 0, st, n, (const double*)v, (const double*)p,
                       nb, nl, sb, wg, nrm, (const double*)pmean, rho * nu, nullptr, (int64_t)gb, t_out, pc_out);
  else
    hipLaunchKernelGGL(drag_partial<float>, dim3(gb), dim3(kRBlock), 0, st, n, (const float*)v, (const float*)p, nb,
                       nl, sb, wg, nrm, (const double*)pmean, rho * nu, nullptr, (int64_t)gb, t_out, pc_out);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

extern "C" const char* mpf_strerror(int code) {
  switch (code) {
    case MPF_OK: return "ok";
    case MPF_ERR_ARG: return "invalid argument";
    case MPF_ERR_HIP: return "HIP runtime error";
    case MPF_ERR_UNSUPPORTED: return "unsupported configuration (no kernel built for it)";
    case MPF_ERR_DIVERGED: return "the run's flags word was set (non-finite state or stability limit exceeded)";
    case MPF_ERR_WORKSPACE: return "workspace missing or too small";
    default: return "unknown error code";
  }
}

extern "C" int mpf_version(void) { return 20000; }

extern "C" int mpf_sc_cell(double r, double* porosity_host, double* area_host) {
  if (!(r >= 0.0 && r < 0.7071067811865475) || !porosity_host || !area_host) return MPF_ERR_ARG;
  const double pi = 3.141592653589793;
  double vs = 4.0 / 3.0 * pi * r * r * r, a = 4.0 * pi * r * r;
  if (r > 0.5) {  // six caps of height r - 1/2 leave the cell
    const double hc = r - 0.5;
    vs -= 6.0 * pi * hc * hc * (3.0 * r - hc) / 3.0;
    a -= 6.0 * 2.0 * pi * r * hc;
  }
  *porosity_host = 1.0 - vs;
  *area_host = a;
  return MPF_OK;
}

extern "C" int mpf_lbm_units_of(double h_min, double nu, double tau_plus, double magic, const double* g_host,
                                mpf_lbm_units* out) {
  if (!out || !g_host || !(h_min > 0.0) || !(nu > 0.0) || !(tau_plus > 0.5) || !(magic > 0.0)) return MPF_ERR_ARG;
  const double dx = 0.5 * h_min;               // streaming distance, Sec. 2.2
  const double nu_lb = (tau_plus - 0.5) / 3.0;  // Eq. lbm_viscosity
  const double dt = nu_lb * dx * dx / nu;       // Eq. conversion_factors: nu = nu_lb dx^2 / dt
  out->dx = dx;
  out->dt = dt;
  out->nu_lb = nu_lb;
  out->tau_minus = 0.5 + magic / (tau_plus - 0.5);  // Lambda = (tau+ - 1/2)(tau- - 1/2)
  out->vel_scale = dx / dt;
  for (int a = 0; a < 3; ++a) out->g_lb[a] = g_host[a] * dt * dt / dx;
  return MPF_OK;
}

extern "C" int mpf_permeability(double q, double nu, const double* g_host, double d, double* k_host) {
  if (!g_host || !k_host || !(nu > 0.0) || !(d > 0.0)) return MPF_ERR_ARG;
  const double g = sqrt(g_host[0] * g_host[0] + g_host[1] * g_host[1] + g_host[2] * g_host[2]);
  if (!(g > 0.0)) return MPF_ERR_ARG;
  *k_host = q * nu / (g * d * d);
  return MPF_OK;
}

extern "C" int mpf_drag_coefficient(double Fx, double r, double phi, double q, double mu, double* K_host) {
  if (!K_host || !(r > 0.0) || !(phi > 0.0) || q == 0.0 || !(mu > 0.0)) return MPF_ERR_ARG;
  *K_host = Fx / (6.0 * 3.141592653589793 * r * phi * q * mu);
  return MPF_OK;
}

namespace mpf {
namespace {
// Residual monitors: per block the max of |v - v_prev| and of |v| (exact in
// any order; a NaN wins) and the sum of (div v)^2 by a fixed tree.
__device__ __forceinline__ double nan_max(double a, double b) { return (a != a || b != b) ? (a + b) : fmax(a, b); }

template <typename T, typename TW>
__global__ __launch_bounds__(kRBlock) void residual_partial(int64_t n, int64_t n_int, int nl,
                                                            const int32_t* __restrict__ sten,
                                                            const TW* __restrict__ w, const T* __restrict__ v,
                                                            const T* __restrict__ vp, double* __restrict__ part,
                                                            int64_t nblk) {
  __shared__ double lds[kRBlock];
  const int64_t i = (int64_t)blockIdx.x * kRBlock + threadIdx.x;
  double dmax = 0.0, vmag = 0.0, d2 = 0.0;
  if (i < n_int) {
    const double vi[3] = {(double)v[i], (double)v[n + i], (double)v[2 * n + i]};
    vmag = sqrt(vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]);
    if (vp) {
      const double e[3] = {vi[0] - (double)vp[i], vi[1] - (double)vp[n + i], vi[2] - (double)vp[2 * n + i]};
      dmax = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    }
    const int64_t os = (int64_t)nl * n;
    double div = 0.0;
    for (int j = 0; j < nl; ++j) {
      const int64_t at = (int64_t)j * n + i;
      const int64_t s = sten[at];
      div += (double)w[at] * (double)v[s] + (double)w[os + at] * (double)v[n + s] +
             (double)w[2 * os + at] * (double)v[2 * n + s];
    }
    d2 = div * div;
  }
  const double bsum = block_sum<kRBlock>(d2, lds);
  lds[threadIdx.x] = dmax;
  __syncthreads();
  for (int st = kRBlock / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) lds[threadIdx.x] = nan_max(lds[threadIdx.x], lds[threadIdx.x + st]);
    __syncthreads();
  }
  const double bdmax = lds[0];
  __syncthreads();
  lds[threadIdx.x] = vmag;
  __syncthreads();
  for (int st = kRBlock / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) lds[threadIdx.x] = nan_max(lds[threadIdx.x], lds[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = bdmax;
    part[nblk + blockIdx.x] = lds[0];
    part[2 * nblk + blockIdx.x] = bsum;
  }
}

__global__ __launch_bounds__(256) void residual_finish(const double* __restrict__ part, int64_t nblk, int64_t n_int,
                                                       double* __restrict__ out) {
  __shared__ double lds[256];
  double m0 = 0.0, m1 = 0.0, acc = 0.0;
  for (int64_t t = threadIdx.x; t < nblk; t += 256) {
    m0 = nan_max(m0, part[t]);
    m1 = nan_max(m1, part[nblk + t]);
    acc += part[2 * nblk + t];
  }
  const double s = block_sum<256>(acc, lds);
  lds[threadIdx.x] = m0;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) lds[threadIdx.x] = nan_max(lds[threadIdx.x], lds[threadIdx.x + st]);
    __syncthreads();
  }
  const double r0 = lds[0];
  __syncthreads();
  lds[threadIdx.x] = m1;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) lds[threadIdx.x] = nan_max(lds[threadIdx.x], lds[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = r0;
    out[1] = lds[0];
    out[2] = n_int > 0 ? sqrt(s / (double)n_int) : 0.0;
  }
}
}  // namespace
}  // namespace mpf

extern "C" int mpf_residual(int64_t n, int64_t n_int, int nl, const int32_t* sten, const void* w, const void* v,
                            const void* v_prev, int precision, double* out, void* ws, size_t ws_bytes,
                            void* stream) {
  if (!out || !v || n < 1 || n_int < 0 || n_int > n || nl < 1 || (n_int > 0 && (!sten || !w))) return MPF_ERR_ARG;
  if (!precision_ok(precision)) return MPF_ERR_ARG;
  if (!ws || ws_bytes < mpf_reduce_workspace(n)) return MPF_ERR_WORKSPACE;
  hipStream_t st = as_stream(stream);
  double* part = reinterpret_cast<double*>(ws);
  const unsigned g = grid_for(n_int, kRBlock);
  if (precision == MPF_F64)
    hipLaunchKernelGGL((residual_partial<double, double>), dim3(g), dim3(kRBlock), 0, st, n, n_int, nl, sten,
                       (const double*)w, (const double*)v, (const double*)v_prev, part, (int64_t)g);
  else if (precision == MPF_MIXED)
    hipLaunchKernelGGL((residual_partial<double, float>), dim3(g), dim3(kRBlock), 0, st, n, n_int, nl, sten,
                       (const float*)w, (const double*)v, (const double*)v_prev, part, (int64_t)g);
  else
    hipLaunchKernelGGL((residual_partial<float, float>), dim3(g), dim3(kRBlock), 0, st, n, n_int, nl, sten,
                       (const float*)w, (const float*)v, (const float*)v_prev, part, (int64_t)g);
  hipLaunchKernelGGL(residual_finish, dim3(1), dim3(256), 0, st, (const double*)part, (int64_t)g, n_int, out);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

// ---------------------------------------------------------------- pointwise difference
namespace mpf {
namespace {
constexpr int kMaxLevels = 16;
struct Levels {
  double t[kMaxLevels];
};

__global__ void zero_counts(int64_t* c, int n) {
  if (threadIdx.x < (unsigned)n) c[threadIdx.x] = 0;
}

// delta_i = |va_i - vb_i| / |vb_i| (FP64), and per block the number of
// counted nodes above each level, added to counts with integer atomics (exact
// in any order).
template <typename TA, typename TB>
__global__ __launch_bounds__(kRBlock) void pointwise_kernel(int64_t n, const TA* __restrict__ va,
                                                            const TB* __restrict__ vb, double* __restrict__ delta,
                                                            double* __restrict__ dv, int64_t n_count, int n_levels,
                                                            Levels lv, int64_t* __restrict__ counts) {
  __shared__ int cnt[kMaxLevels];
  if (threadIdx.x < kMaxLevels) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kRBlock + threadIdx.x;
  if (i < n) {
    const double d0 = (double)va[i] - (double)vb[i];
    const double d1 = (double)va[n + i] - (double)vb[n + i];
    const double d2 = (double)va[2 * n + i] - (double)vb[2 * n + i];
    const double b0 = vb[i], b1 = vb[n + i], b2 = vb[2 * n + i];
    const double num = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    const double den = sqrt(b0 * b0 + b1 * b1 + b2 * b2);
    const double d = den > 0.0 ? num / den : (num > 0.0 ? __builtin_huge_val() : 0.0);
    if (delta) delta[i] = d;
    if (dv) dv[i] = num;
    if (i < n_count)
      for (int l = 0; l < n_levels; ++l)
        if (d > lv.t[l]) atomicAdd(&cnt[l], 1);
  }
  __syncthreads();
  if (counts && threadIdx.x < (unsigned)n_levels && cnt[threadIdx.x])
    atomicAdd(reinterpret_cast<unsigned long long*>(counts + threadIdx.x), (unsigned long long)cnt[threadIdx.x]);
}

template <typename TA, typename TB>
void launch_pointwise(int64_t n, const void* va, const void* vb, double* delta, double* dv, int64_t n_count,
                      int n_levels, const Levels& lv, int64_t* counts, hipStream_t st) {
  hipLaunchKernelGGL((pointwise_kernel<TA, TB>), dim3(grid_for(n, kRBlock)), dim3(kRBlock), 0, st, n,
                     (const TA*)va, (const TB*)vb, delta, dv, n_count, n_levels, lv, counts);
}
}  // namespace
}  // namespace mpf

extern "C" int mpf_pointwise(int64_t n, const void* va, int prec_a, const void* vb, int prec_b, double* delta,
                             double* dv, int64_t n_count, int n_levels, const double* levels_host, int64_t* counts,
                             void* stream) {
  using namespace mpf;
  if (n < 1 || !va || !vb || !precision_ok(prec_a) || !precision_ok(prec_b)) return MPF_ERR_ARG;
  if (n_levels < 0 || n_levels > kMaxLevels || n_count < 0 || n_count > n) return MPF_ERR_ARG;
  if (n_levels > 0 && (!levels_host || !counts)) return MPF_ERR_ARG;
  Levels lv{};
  for (int l = 0; l < n_levels; ++l) lv.t[l] = levels_host[l];
  hipStream_t st = as_stream(stream);
  if (n_levels > 0) hipLaunchKernelGGL(zero_counts, dim3(1), dim3(kMaxLevels), 0, st, counts, n_levels);
  const bool fa = state_is_f32(prec_a), fb = state_is_f32(prec_b);
  if (fa && fb) launch_pointwise<float, float>(n, va, vb, delta, dv, n_count, n_levels, lv, counts, st);
  else if (fa) launch_pointwise<float, double>(n, va, vb, delta, dv, n_count, n_levels, lv, counts, st);
  else if (fb) launch_pointwise<double, float>(n, va, vb, delta, dv, n_count, n_levels, lv, counts, st);
  else launch_pointwise<double, double>(n, va, vb, delta, dv, n_count, n_levels, lv, counts, st);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

// ---------------------------------------------------------------- allocation-free flux
// Block partial sums of mpf_flux_planes_noalloc live in a static device array
// instead of a caller workspace.  Host code never passes the array's name to
// a kernel (on the host it is only a stand-in symbol): its device address is
// looked up once per device with hipGetSymbolAddress, with that device
// current, and kept in scratch_dev.
namespace mpf {
namespace {
constexpr int64_t kScratchPartials = 8192;  // 64 KiB of partials: 2^21 samples
static __device__ __align__(256) double scratch[kScratchPartials];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

int scratch_dev(double** out) {
  int dev = 0;
  MPF_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return MPF_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    MPF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return MPF_ERR_HIP;
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return MPF_OK;
}
}  // namespace
}  // namespace mpf

extern "C" int64_t mpf_flux_planes_noalloc_max(void) { return mpf::kScratchPartials * mpf::kRBlock; }

extern "C" int mpf_flux_planes_noalloc(int64_t ns, int nl, const int32_t* s_idx, const double* s_w, const void* vx,
                                       int precision, int64_t n_all, double* q_out, void* stream) {
  using namespace mpf;
  if (!q_out || ns < 0 || n_all < 1 || nl < 1 || (ns > 0 && (!s_idx || !s_w || !vx))) return MPF_ERR_ARG;
  if (!precision_ok(precision)) return MPF_ERR_ARG;
  if (ns > mpf_flux_planes_noalloc_max()) return MPF_ERR_WORKSPACE;
  double* part = nullptr;
  const int rc = scratch_dev(&part);
  if (rc) return rc;
  hipStream_t st = as_stream(stream);
  const unsigned g = grid_for(ns, kRBlock);  // every partial [0, g) is written before it is read
  if (!state_is_f32(precision))
    hipLaunchKernelGGL(flux_partial<double>, dim3(g), dim3(kRBlock), 0, st, ns, nl, s_idx, s_w, (const double*)vx,
                       part);
  else
    hipLaunchKernelGGL(flux_partial<float>, dim3(g), dim3(kRBlock), 0, st, ns, nl, s_idx, s_w, (const float*)vx,
                       part);
  hipLaunchKernelGGL(finish_sum, dim3(1), dim3(256), 0, st, (const double*)part, (int64_t)g, 1, 1.0 / (double)n_all,
                     q_out);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}
