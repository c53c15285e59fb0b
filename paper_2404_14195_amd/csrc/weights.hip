// Batched RBF-FD weight solves (Sec. 2.1, Eqs. operatorApprox, rbfScaling,
// augmentedSystem) on gfx950.
//
// One wave64 owns one stencil row.  Lane j holds row j of the augmented
// matrix M = [A P; P^T 0] (size N = NL + 10 <= 60) in registers; the first NL
// lanes also own the output weights w_j.  Gaussian elimination with partial
// pivoting keeps rows in place: at column c the pivot is the unused lane with
// the largest |M[.][c]| (wave butterfly, ties to the lowest lane), the pivot
// row is broadcast with readlane and every still-active lane subtracts its
// multiple, keeping the multiplier in column c.  The right-hand sides are then
// processed in chunks of RB with forward and backward substitution over the
// stored factors, so the O(N^3) factorisation is done once per row whatever
// the number of operators.  Everything is FP64 on the vector ALU: a 40 x 40
// pivoted LU is not a dense contraction that MFMA tiles would serve.
#include "common.hpp"

namespace mpf {
namespace {

constexpr int kMaxOps = 32;
constexpr int RB = 4;

struct OpsArg {
  int n;
  int kind[kMaxOps];
  double vec[kMaxOps][3];
};

__device__ __forceinline__ double mono(int l, double x, double y, double z) {
  switch (l) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * x;
    case 5: return x * y;
    case 6: return x * z;
    case 7: return y * y;
    case 8: return y * z;
    default: return z * z;
  }
}

__device__ __forceinline__ double cube_dist(double ax, double ay, double az, double bx, double by, double bz) {
  double dx = ax - bx, dy = ay - by, dz = az - bz;
  double r = sqrt(dx * dx + dy * dy + dz * dz);
  return r * r * r;
}

// Right-hand-side entry of row j (lane) for operator o.
template <int NL>
__device__ __forceinline__ double rhs_entry(int kind, const double* vec, const double* rv, int j, double xi0,
                                            double xi1, double xi2, double rho, double delta) {
  const double id = 1.0 / delta;
  if (kind == MPF_OP_SHIFT || kind == MPF_OP_SHIFT_ROW) {
    const double* s = kind == MPF_OP_SHIFT ? vec : rv;
    double s0 = s[0] * id, s1 = s[1] * id, s2 = s[2] * id;
    if (j < NL) return cube_dist(s0, s1, s2, xi0, xi1, xi2);
    return mono(j - NL, s0, s1, s2);
  }
  if (kind == MPF_OP_LAP) {
    if (j < NL) return 12.0 * rho * id * id;
    int l = j - NL;
    return (l == 4 || l == 7 || l == 9) ? 2.0 * id * id : 0.0;
  }
  // first-derivative family: e . grad with e a unit axis, vec, or rowvec
  double e0, e1, e2;
  if (kind <= MPF_OP_DZ) {
    e0 = kind == MPF_OP_DX; e1 = kind == MPF_OP_DY; e2 = kind == MPF_OP_DZ;
  } else {
    const double* e = kind == MPF_OP_DIR ? vec : rv;
    e0 = e[0]; e1 = e[1]; e2 = e[2];
  }
  if (j < NL) return -3.0 * id * rho * (e0 * xi0 + e1 * xi1 + e2 * xi2);
  int l = j - NL;
  return l == 1 ? e0 * id : (l == 2 ? e1 * id : (l == 3 ? e2 * id : 0.0));
}

template <int NL>
__global__ __launch_bounds__(256) void weights_kernel(const double* __restrict__ pos, int64_t n_nodes,
                                                      const int32_t* __restrict__ sten, int64_t m, OpsArg ops,
                                                      const double* __restrict__ rowvec, double* __restrict__ w64,
                                                      float* __restrict__ w32, int32_t* __restrict__ info) {
  constexpr int N = NL + 10;
  static_assert(N <= kWave, "system does not fit one wave");
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
  if (row >= m) return;  // whole wave exits together

  // --- scaled local coordinates xi_j = minimg(x_j - x_c) / delta, with
  // delta the distance from the centre to stencil column 1
  double xi0, xi1, xi2, delta;
  {
    const int sj = sten[(int64_t)(lane < NL ? lane : 0) * m + row];
    const int sc = sten[row];
    double d0 = min_image(pos[sj] - pos[sc]);
    double d1 = min_image(pos[n_nodes + sj] - pos[n_nodes + sc]);
    double d2 = min_image(pos[2 * n_nodes + sj] - pos[2 * n_nodes + sc]);
    const double q0 = bcast(d0, 1), q1 = bcast(d1, 1), q2 = bcast(d2, 1);
    delta = sqrt(q0 * q0 + q1 * q1 + q2 * q2);
    xi0 = d0 / delta; xi1 = d1 / delta; xi2 = d2 / delta;
    if (lane >= NL) xi0 = xi1 = xi2 = 0.0;
  }
  const double rho = sqrt(xi0 * xi0 + xi1 * xi1 + xi2 * xi2);

  // --- assemble row `lane` of M
  double a[N];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    double x0 = bcast(xi0, k), x1 = bcast(xi1, k), x2 = bcast(xi2, k);
    a[k] = lane < NL ? cube_dist(xi0, xi1, xi2, x0, x1, x2) : (lane < N ? mono(lane - NL, x0, x1, x2) : 0.0);
  }
#pragma unroll
  for (int l = 0; l < 10; ++l) a[NL + l] = lane < NL ? mono(l, xi0, xi1, xi2) : 0.0;

  // --- LU with partial pivoting, rows in place
  int pcol = (lane < N) ? 1 << 20 : -1;  // column at which this lane became pivot
  int bad = 0;
#pragma unroll
  for (int c = 0; c < N; ++c) {
    double cand = (pcol > c) ? fabs(a[c]) : -1.0;
    int cl = lane;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      double ov = __shfl_xor(cand, off);
      int ol = __shfl_xor(cl, off);
      if (ov > cand || (ov == cand && ol < cl)) { cand = ov; cl = ol; }
    }
    const int p = __builtin_amdgcn_readfirstlane(cl);
    const double best = bcast(cand, 0);
    if (!(best > 0.0)) { bad = c + 1; break; }
    const double pv = bcast(a[c], p);
    const bool act = pcol > c && lane != p;
    if (lane == p) pcol = c;
    const double l = act ? a[c] / pv : 0.0;
    if (act) a[c] = l;
#pragma unroll
    for (int k = c + 1; k < N; ++k) {
      double pk = bcast(a[k], p);
      if (act) a[k] = fma(-l, pk, a[k]);
    }
  }

  double rvv[3] = {0.0, 0.0, 0.0};
  if (rowvec) { rvv[0] = rowvec[row]; rvv[1] = rowvec[m + row]; rvv[2] = rowvec[2 * m + row]; }

  for (int o0 = 0; o0 < ops.n; o0 += RB) {
    double b[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      int o = o0 + r;
      b[r] = (o < ops.n && lane < N) ? rhs_entry<NL>(ops.kind[o], ops.vec[o], rvv, lane, xi0, xi1, xi2, rho, delta)
                                     : 0.0;
    }
    double x[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) x[r] = 0.0;
    if (!bad) {
      // forward substitution with the stored multipliers (pivot order)
#pragma unroll
      for (int c = 0; c < N; ++c) {
        const int p = __builtin_amdgcn_readfirstlane(__builtin_ctzll(__ballot(pcol == c)));
        const bool act = pcol > c;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          double y = bcast(b[r], p);
          if (act) b[r] = fma(-a[c], y, b[r]);
        }
      }
      // back substitution; lane c keeps unknown c
#pragma unroll
      for (int c = N - 1; c >= 0; --c) {
        const int p = __builtin_amdgcn_readfirstlane(__builtin_ctzll(__ballot(pcol == c)));
        const bool act = pcol < c;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          double xc = bcast(b[r] / a[c], p);
          if (lane == c) x[r] = xc;
          if (act) b[r] = fma(-a[c], xc, b[r]);
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < RB; ++r) x[r] = __builtin_nan("");
    }
    // store w[o][j][row]; FP32 copy with the self weight fixing the row sum
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      int o = o0 + r;
      if (o >= ops.n) break;
      if (w64 && lane < NL) w64[((int64_t)o * NL + lane) * m + row] = x[r];
      if (w32) {
        float xf = (float)x[r];
        double part = (lane >= 1 && lane < NL) ? (double)xf : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
        const int kd = ops.kind[o];
        const double target = (kd == MPF_OP_SHIFT || kd == MPF_OP_SHIFT_ROW) ? 1.0 : 0.0;
        if (lane == 0) xf = (float)(target - part);
        if (lane < NL) w32[((int64_t)o * NL + lane) * m + row] = xf;
      }
    }
  }
  if (lane == 0) info[row] = bad;
}

template <int NL>
int launch_weights(const double* pos, int64_t n_nodes, const int32_t* sten, int64_t m, const OpsArg& ops,
                   const double* rowvec, double* w64, float* w32, int32_t* info, hipStream_t st) {
  const int block = 256;
  const int per = block / kWave;
  hipLaunchKernelGGL(weights_kernel<NL>, dim3(grid_for(m, per)), dim3(block), 0, st, pos, n_nodes, sten, m, ops,
                     rowvec, w64, w32, info);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

}  // namespace
}  // namespace mpf

extern "C" int mpf_rbffd_weights(const double* pos, int64_t n_nodes, const int32_t* sten, int64_t m, int nl,
                                 int n_ops, const mpf_op* ops, const double* rowvec, double* w64, float* w32,
                                 int32_t* info, void* stream) {
  using namespace mpf;
  if (!pos || !sten || !ops || !info || n_nodes < 2 || m < 0 || n_ops < 1 || n_ops > kMaxOps) return MPF_ERR_ARG;
  if (!w64 && !w32) return MPF_ERR_ARG;
  OpsArg a{};
  a.n = n_ops;
  for (int o = 0; o < n_ops; ++o) {
    int k = ops[o].kind;
    if (k < MPF_OP_DX || k > MPF_OP_SHIFT_ROW) return MPF_ERR_ARG;
    if ((k == MPF_OP_DN || k == MPF_OP_SHIFT_ROW) && !rowvec) return MPF_ERR_ARG;
    a.kind[o] = k;
    for (int t = 0; t < 3; ++t) a.vec[o][t] = ops[o].vec[t];
  }
  if (m == 0) return MPF_OK;
  hipStream_t st = as_stream(stream);
  switch (nl) {
    case 20: return launch_weights<20>(pos, n_nodes, sten, m, a, rowvec, w64, w32, info, st);
    case 25: return launch_weights<25>(pos, n_nodes, sten, m, a, rowvec, w64, w32, info, st);
    case 27: return launch_weights<27>(pos, n_nodes, sten, m, a, rowvec, w64, w32, info, st);
    case 30: return launch_weights<30>(pos, n_nodes, sten, m, a, rowvec, w64, w32, info, st);
    case 35: return launch_weights<35>(pos, n_nodes, sten, m, a, rowvec, w64, w32, info, st);
    case 40: return launch_weights<40>(pos, n_nodes, sten, m, a, rowvec, w64, w32, info, st);
    case 45: return launch_weights<45>(pos, n_nodes, sten, m, a, rowvec, w64, w32, info, st);
    case 50: return launch_weights<50>(pos, n_nodes, sten, m, a, rowvec, w64, w32, info, st);
    default: return MPF_ERR_UNSUPPORTED;
  }
}
