// Permeability and drag reductions (Eqs. k_definition, stress_tensor_force,
// integration_force) and the library's host-side helpers.
//
// Sums are deterministic: every block reduces its items with a fixed-shape
// tree into one partial, and one block then adds the partials in a fixed
// order, so a rerun gives the same bits.  All accumulation is FP64 whatever
// the precision of the fields.
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
  if (precision != MPF_F64 && precision != MPF_F32) return MPF_ERR_ARG;
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
  if (precision != MPF_F64 && precision != MPF_F32 && precision != MPF_MIXED) return MPF_ERR_ARG;
  if (!ws || ws_bytes < mpf_reduce_workspace(ns)) return MPF_ERR_WORKSPACE;
  hipStream_t st = as_stream(stream);
  double* part = reinterpret_cast<double*>(ws);
  const unsigned g = grid_for(ns, kRBlock);
  if (precision != MPF_F32)
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
  if (precision != MPF_F64 && precision != MPF_F32 && precision != MPF_MIXED) return MPF_ERR_ARG;
  if (!ws || ws_bytes < mpf_reduce_workspace(n > nb ? n : nb)) return MPF_ERR_WORKSPACE;
  hipStream_t st = as_stream(stream);
  double* part = reinterpret_cast<double*>(ws);
  const int64_t nmax = n > nb ? n : nb;
  const int64_t cap = (nmax + kRBlock - 1) / kRBlock;
  double* pmean = part + 3 * cap;
  // node mean of p
  const unsigned gn = grid_for(n, kRBlock);
  if (precision != MPF_F32)
    hipLaunchKernelGGL(sum_partial<double>, dim3(gn), dim3(kRBlock), 0, st, n, (const double*)p, part);
  else
    hipLaunchKernelGGL(sum_partial<float>, dim3(gn), dim3(kRBlock), 0, st, n, (const float*)p, part);
  hipLaunchKernelGGL(finish_sum, dim3(1), dim3(256), 0, st, (const double*)part, (int64_t)gn, 1, 1.0 / (double)n,
                     pmean);
  // tractions
  const unsigned gb = grid_for(nb, kRBlock);
  if (precision != MPF_F32)
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
  if (precision != MPF_F64 && precision != MPF_F32 && precision != MPF_MIXED) return MPF_ERR_ARG;
  if (!ws || ws_bytes < mpf_reduce_workspace(n > nb ? n : nb)) return MPF_ERR_WORKSPACE;
  if (nb == 0) return MPF_OK;
  hipStream_t st = as_stream(stream);
  double* part = reinterpret_cast<double*>(ws);
  const int64_t nmax = n > nb ? n : nb;
  const int64_t cap = (nmax + kRBlock - 1) / kRBlock;
  double* pmean = part + 3 * cap;
  const unsigned gn = grid_for(n, kRBlock);
  if (precision != MPF_F32)
    hipLaunchKernelGGL(sum_partial<double>, dim3(gn), dim3(kRBlock), 0, st, n, (const double*)p, part);
  else
    hipLaunchKernelGGL(sum_partial<float>, dim3(gn), dim3(kRBlock), 0, st, n, (const float*)p, part);
  hipLaunchKernelGGL(finish_sum, dim3(1), dim3(256), 0, st, (const double*)part, (int64_t)gn, 1, 1.0 / (double)n,
                     pmean);
  const unsigned gb = grid_for(nb, kRBlock);
  if (precision != MPF_F32)
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
    case MPF_ERR_WORKSPACE: return "workspace missing or too small";
    default: return "unknown error code";
  }
}

extern "C" int mpf_version(void) { return 100; }

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
