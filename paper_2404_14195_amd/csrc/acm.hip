// Artificial-compressibility Navier-Stokes steps (Sec. 2.3, Eqs.
// MNS_intermediate, MNS_pressure, MNS_velocity, MNS_C) on gfx950.
//
// Every pass is an HBM-bound stencil apply: one thread per node walks its
// nl stencil columns; weights and stencil indices are stored [op][j][node]
// so the 64 lanes of a wave read consecutive addresses, while the gathered
// field values come from the caches (nodes are Morton ordered).  A step is
// 1 + 3 n_p dependent passes:
//   predictor  (interior)     v' from v: 4 operators x 3 components
//   n_p x { pressure (interior)  p -= dt C^2 rho div v
//           neumann  (boundary)  p_b from dp/dn = 0, in place (its stencil
//                                holds only interior neighbours)
//           velocity (interior)  v = v' - dt/rho grad p, max |v| }
// C is never stored: each pressure pass derives it from the running max |v|
// (device double, updated with an integer atomicMax on the bit pattern, which
// orders non-negative doubles), so no host round trip enters a step.
#include "common.hpp"

namespace mpf {
namespace {

constexpr int kBlock = 256;

template <typename T>
__global__ __launch_bounds__(kBlock) void acm_predictor(int64_t n, int64_t n_int, int nl,
                                                        const int32_t* __restrict__ sten, const T* __restrict__ w,
                                                        const T* __restrict__ v, T* __restrict__ vp, T nu, T dt,
                                                        T g0, T g1, T g2) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n_int) return;
  const int64_t os = (int64_t)nl * n;  // operator stride in w
  T d[3][4];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int o = 0; o < 4; ++o) d[a][o] = T(0);
  for (int j = 0; j < nl; ++j) {
    const int64_t at = (int64_t)j * n + i;
    const int s = sten[at];
    const T wx = w[at], wy = w[os + at], wz = w[2 * os + at], wl = w[3 * os + at];
    const T u[3] = {v[s], v[n + s], v[2 * n + s]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      d[a][0] += wx * u[a];
      d[a][1] += wy * u[a];
      d[a][2] += wz * u[a];
      d[a][3] += wl * u[a];
    }
  }
  const T vi[3] = {v[i], v[n + i], v[2 * n + i]};
  const T g[3] = {g0, g1, g2};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const T adv = vi[0] * d[a][0] + vi[1] * d[a][1] + vi[2] * d[a][2];
    vp[a * n + i] = vi[a] + dt * (nu * d[a][3] - adv + g[a]);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void acm_pressure(int64_t n, int64_t n_int, int nl,
                                                       const int32_t* __restrict__ sten, const T* __restrict__ w,
                                                       const T* __restrict__ v, T* __restrict__ p,
                                                       const double* __restrict__ vmax, double dt, double rho,
                                                       double beta, double v_ref) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n_int) return;
  const double vm = *vmax;
  const double C = beta * (vm > v_ref ? vm : v_ref);
  const T coef = (T)(dt * (C * C) * rho);
  const int64_t os = (int64_t)nl * n;
  T div = T(0);
  for (int j = 0; j < nl; ++j) {
    const int64_t at = (int64_t)j * n + i;
    const int s = sten[at];
    div += w[at] * v[s] + w[os + at] * v[n + s] + w[2 * os + at] * v[2 * n + s];
  }
  p[i] -= coef * div;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void acm_neumann(int64_t n_int, int64_t nb, int nl,
                                                      const int32_t* __restrict__ sn, const T* __restrict__ wn,
                                                      T* __restrict__ p, double* __restrict__ vmax) {
  const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (b == 0) *vmax = 0.0;  // the pressure pass has consumed it; the velocity pass rebuilds it
  if (b >= nb) return;
  T s = T(0);
  for (int j = 1; j < nl; ++j) {
    const int64_t at = (int64_t)j * nb + b;
    s += wn[at] * p[sn[at]];
  }
  p[n_int + b] = -s / wn[b];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void acm_velocity(int64_t n, int64_t n_int, int nl,
                                                       const int32_t* __restrict__ sten, const T* __restrict__ w,
                                                       const T* __restrict__ vp, const T* __restrict__ p,
                                                       T* __restrict__ v, T dt_rho,
                                                       unsigned long long* __restrict__ vmax_bits) {
  __shared__ double red[kBlock / kWave];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double mag = 0.0;
  if (i < n_int) {
    const int64_t os = (int64_t)nl * n;
    T gp[3] = {T(0), T(0), T(0)};
    for (int j = 0; j < nl; ++j) {
      const int64_t at = (int64_t)j * n + i;
      const T ps = p[sten[at]];
      gp[0] += w[at] * ps;
      gp[1] += w[os + at] * ps;
      gp[2] += w[2 * os + at] * ps;
    }
    double m2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T va = vp[a * n + i] - dt_rho * gp[a];
      v[a * n + i] = va;
      m2 += (double)va * (double)va;
    }
    mag = sqrt(m2);
  }
  // block max; the max is exact, so any reduction order gives the same value
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mag = fmax(mag, __shfl_xor(mag, off));
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = mag;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int t = 1; t < kBlock / kWave; ++t) m = fmax(m, red[t]);
    if (m != m) m = __builtin_inf();  // a non-finite state shows up as C = inf
    atomicMax(vmax_bits, (unsigned long long)__double_as_longlong(m));
  }
}

template <typename T>
__global__ void fill_zero(T* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] = T(0);
}

template <typename T>
int run(const mpf_acm_params* prm, int64_t n, int64_t n_int, int nl, const int32_t* sten, const T* w,
        const int32_t* sn, const T* wn, T* v, T* p, double* vmax, int n_steps, void* ws, hipStream_t st) {
  const int64_t nb = n - n_int;
  T* vp = reinterpret_cast<T*>(ws);
  const unsigned gi = grid_for(n_int, kBlock), gb = grid_for(nb, kBlock);
  // v' is zero on the boundary for the whole run
  for (int a = 0; a < 3; ++a) {
    if (nb > 0) hipLaunchKernelGGL(fill_zero<T>, dim3(gb), dim3(kBlock), 0, st, vp + a * n + n_int, nb);
  }
  const T nu = (T)prm->nu, dt = (T)prm->dt, dt_rho = (T)(prm->dt / prm->rho);
  for (int s = 0; s < n_steps; ++s) {
    hipLaunchKernelGGL(acm_predictor<T>, dim3(gi), dim3(kBlock), 0, st, n, n_int, nl, sten, w, v, vp, nu, dt,
                       (T)prm->g[0], (T)prm->g[1], (T)prm->g[2]);
    for (int it = 0; it < prm->n_p; ++it) {
      hipLaunchKernelGGL(acm_pressure<T>, dim3(gi), dim3(kBlock), 0, st, n, n_int, nl, sten, w,
                         (const T*)(it == 0 ? vp : v), p, vmax, prm->dt, prm->rho, prm->beta, prm->v_ref);
      hipLaunchKernelGGL(acm_neumann<T>, dim3(gb), dim3(kBlock), 0, st, n_int, nb, nl, sn, wn, p, vmax);
      hipLaunchKernelGGL(acm_velocity<T>, dim3(gi), dim3(kBlock), 0, st, n, n_int, nl, sten, w, (const T*)vp,
                         (const T*)p, v, dt_rho, reinterpret_cast<unsigned long long*>(vmax));
    }
  }
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

}  // namespace
}  // namespace mpf

extern "C" size_t mpf_acm_workspace(int64_t n, int precision) {
  const size_t es = precision == MPF_F32 ? sizeof(float) : sizeof(double);
  return n > 0 ? 3 * (size_t)n * es + 256 : 256;
}

extern "C" int mpf_acm_run(const mpf_acm_params* prm, int64_t n, int64_t n_int, int nl, const int32_t* sten,
                           const void* w, const int32_t* sn, const void* wn, void* v, void* p, double* vmax,
                           int n_steps, void* ws, size_t ws_bytes, void* stream) {
  using namespace mpf;
  if (!prm || !sten || !w || !v || !p || !vmax || n < 1 || n_int < 0 || n_int > n || nl < 2 || n_steps < 0 ||
      prm->n_p < 1 || !(prm->dt > 0.0) || !(prm->rho > 0.0))
    return MPF_ERR_ARG;
  if (n > n_int && (!sn || !wn)) return MPF_ERR_ARG;
  if (prm->precision != MPF_F64 && prm->precision != MPF_F32) return MPF_ERR_ARG;
  if (!ws || ws_bytes < mpf_acm_workspace(n, prm->precision)) return MPF_ERR_WORKSPACE;
  if (n_steps == 0) return MPF_OK;
  hipStream_t st = as_stream(stream);
  if (prm->precision == MPF_F64)
    return run<double>(prm, n, n_int, nl, sten, (const double*)w, sn, (const double*)wn, (double*)v, (double*)p,
                       vmax, n_steps, ws, st);
  return run<float>(prm, n, n_int, nl, sten, (const float*)w, sn, (const float*)wn, (float*)v, (float*)p, vmax,
                    n_steps, ws, st);
}
