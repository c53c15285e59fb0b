// Shared device/host helpers of libmpf (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

#include "mpf.h"

namespace mpf {

constexpr int kWave = 64;

#define MPF_HIP(expr)                                     \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return MPF_ERR_HIP;             \
  } while (0)

#define MPF_LAUNCH_CHECK() MPF_HIP(hipGetLastError())

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// End of a *_run given a flags word: wait for the stream, read the word and
// report MPF_ERR_DIVERGED when a kernel has set any bit.  No flags, no wait.
inline int check_flags(const uint32_t* flags, hipStream_t st) {
  if (!flags) return MPF_OK;
  uint32_t h = 0;
  MPF_HIP(hipMemcpyAsync(&h, flags, sizeof(h), hipMemcpyDeviceToHost, st));
  MPF_HIP(hipStreamSynchronize(st));
  return h ? MPF_ERR_DIVERGED : MPF_OK;
}

// Precisions whose state (fields, populations) is stored in FP32.
inline bool state_is_f32(int precision) { return precision == MPF_F32 || precision == MPF_F32_KAHAN; }
inline bool precision_ok(int precision) {
  return precision == MPF_F64 || precision == MPF_F32 || precision == MPF_MIXED || precision == MPF_F32_KAHAN;
}

inline unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (unsigned)(g < 1 ? 1 : g);
}

// Minimum-image displacement in the unit periodic cell.
__device__ __forceinline__ double min_image(double d) { return d - rint(d); }

// Broadcast a double from a wave-uniform lane.
__device__ __forceinline__ double bcast(double x, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// ---------------------------------------------------------------- lattices
// Velocity sets in the pairing of the paper's D3Q15 table: k = 0 rest, odd k
// a listed vector, even k its opposite.
template <int Q>
struct Lattice;

template <>
struct Lattice<19> {
  static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr double w0 = 1.0 / 3.0, w1 = 1.0 / 18.0, w2 = 1.0 / 36.0;
};

template <>
struct Lattice<15> {
  static constexpr int ex[15] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
  static constexpr int ey[15] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1};
  static constexpr int ez[15] = {0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr double w0 = 2.0 / 9.0, w1 = 1.0 / 9.0, w2 = 1.0 / 72.0;
};

template <int Q>
__host__ __device__ constexpr double lat_w(int k) {
  return (Lattice<Q>::ex[k] * Lattice<Q>::ex[k] + Lattice<Q>::ey[k] * Lattice<Q>::ey[k] +
          Lattice<Q>::ez[k] * Lattice<Q>::ez[k]) == 0
             ? Lattice<Q>::w0
             : ((Lattice<Q>::ex[k] * Lattice<Q>::ex[k] + Lattice<Q>::ey[k] * Lattice<Q>::ey[k] +
                 Lattice<Q>::ez[k] * Lattice<Q>::ez[k]) == 1
                    ? Lattice<Q>::w1
                    : Lattice<Q>::w2);
}

// opposite of k in this pairing
__host__ __device__ constexpr int lat_opp(int k) { return k == 0 ? 0 : ((k & 1) ? k + 1 : k - 1); }

// ---------------------------------------------------------------- reductions
// Fixed-shape block sum (deterministic for a given block size).  Every thread
// of the block must call it; the result is valid in thread 0.
template <int BLOCK>
__device__ __forceinline__ double block_sum(double v, double* lds) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if (t < s) lds[t] += lds[t + s];
    __syncthreads();
  }
  double r = lds[0];
  __syncthreads();
  return r;
}

// Sum n partials in a fixed order with one block of 256 threads, scale the
// result and store it.
__global__ void finish_sum(const double* __restrict__ part, int64_t n, int stride, double scale,
                           double* __restrict__ out);

}  // namespace mpf
