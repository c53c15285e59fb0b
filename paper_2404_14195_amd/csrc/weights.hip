// Batched RBF-FD weight solves (Sec. 2.1, Eqs. operatorApprox, rbfScaling,
// augmentedSystem) on gfx950.
//
// One wave64 owns one stencil row at a time.  Lane j holds row j of the
// augmented matrix M = [A P; P^T 0] (size N = NL + 10 <= 60) in registers;
// the first NL lanes also own the output weights w_j.  Gaussian elimination
// with partial pivoting keeps rows in place: at column c the pivot is the
// unused lane with the largest |M[.][c]| (wave butterfly, ties to the lowest
// lane), the pivot row is broadcast with readlane and every still-active lane
// subtracts its multiple, keeping the multiplier in column c.  Right-hand
// sides then go through forward and backward substitution over the stored
// factors in chunks of RB, so the O(N^3) factorisation is done once per row
// whatever the number of operators.  With at most RB operators the
// right-hand sides instead ride along as extra columns of a Gauss-Jordan
// elimination (every row, not only those below the pivot, is reduced; in
// this row-per-lane layout that costs no extra instructions) and each pivot
// lane ends holding its unknown, with no substitution sweeps.  Everything
// runs on the vector ALU: a
// pivoted 40 x 40 LU per row is not a dense contraction MFMA tiles would
// serve.
//
// Launch: one grid over the concatenated rows of up to kMaxGeoms node clouds
// (a row-to-cloud table in the workspace), each wave solving `rows_per_wave`
// consecutive rows, so clouds of any sizes share one launch.  The block shape
// (waves per block, rows per wave) comes from the autotuner.
//
// Precision: FP64 direct, or FP32 factors with FP64-residual iterative
// refinement (x += LU32^-1 (b - M x) with M and the residual in FP64, up to
// kIrSweeps sweeps).  A sweep ends the refinement when |dx| <= 1e-15 |x|, or
// when |dx| <= 1e-9 |x| has stopped shrinking (by 4x per sweep): the FP64
// residual then limits x to about cond(M) eps64, as for a direct FP64 solve.
// Any other row is re-solved in FP64 and flagged with info < 0.
#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "common.hpp"

namespace mpf {
namespace {

constexpr int kMaxOps = 32;
constexpr int kMaxGeoms = 16;
constexpr int RB = 4;
// refinement sweeps after the FP32 solve: with kappa ~ 1e4 each sweep gains
// about log10(1 / (kappa eps32)) = 3.4 digits, so five reach 1e-15
constexpr int kIrSweeps = 5;

struct OpsArg {
  int n;
  int kind[kMaxOps];
  double vec[kMaxOps][3];
};

struct GeomArg {
  const double* pos;
  int64_t n_nodes;
  const int32_t* sten;
  int64_t m;
  const double* rowvec;
  double* w64;
  float* w32;
  int32_t* info;
  int64_t row0;  // first global row of this cloud
};

struct BatchArg {
  int n_geoms;
  int64_t total;
  GeomArg g[kMaxGeoms];
};

// workspace layout: 256 bytes reserved, then the geometry table
constexpr size_t kTableOffset = 256;
constexpr size_t kWorkspaceBytes = kTableOffset + sizeof(GeomArg) * kMaxGeoms;

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

// The monomial p_l of a lane-dependent l without branches: p_l = f1 f2 with
// each factor one of 1, x, y, z, picked by 0/1 coefficients, so the value is
// the same as mono(l, ...) bit for bit (one coefficient is 1, the rest 0).
struct MonoPick {
  double c1[4], c2[4];  // coefficients of (1, x, y, z) in f1 and f2
  __device__ __forceinline__ explicit MonoPick(int l) {
    const int i1 = l < 4 ? l : (l < 7 ? 1 : (l < 9 ? 2 : 3));
    const int i2 = l < 4 ? 0 : (l == 4 ? 1 : (l == 5 ? 2 : (l == 6 ? 3 : (l == 7 ? 2 : 3))));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      c1[q] = q == i1 ? 1.0 : 0.0;
      c2[q] = q == i2 ? 1.0 : 0.0;
    }
  }
  __device__ __forceinline__ double operator()(double x, double y, double z) const {
    const double f1 = fma(c1[1], x, fma(c1[2], y, fma(c1[3], z, c1[0])));
    const double f2 = fma(c2[1], x, fma(c2[2], y, fma(c2[3], z, c2[0])));
    return f1 * f2;
  }
};

__device__ __forceinline__ double cube_dist(double ax, double ay, double az, double bx, double by, double bz) {
  double dx = ax - bx, dy = ay - by, dz = az - bz;
  double r = sqrt(dx * dx + dy * dy + dz * dz);
  return r * r * r;
}

// Right-hand-side entry of row j (lane) for one operator.
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
  if (kind == MPF_OP_LAP) {  // lap r^3 = 3 (3 + 3 - 2) r = 12 r; lap of x^2, y^2, z^2 = 2
    if (j < NL) return 12.0 * rho * id * id;
    int l = j - NL;
    return (l == 4 || l == 7 || l == 9) ? 2.0 * id * id : 0.0;
  }
  // first-derivative family: e . grad with e a unit axis, vec, or rowvec;
  // the Taylor row adds the value at the centre (|xi_j|^3 and p_l(0))
  double e0, e1, e2;
  if (kind <= MPF_OP_DZ) {
    e0 = kind == MPF_OP_DX; e1 = kind == MPF_OP_DY; e2 = kind == MPF_OP_DZ;
  } else {
    const double* e = (kind == MPF_OP_DIR || kind == MPF_OP_TAYLOR) ? vec : rv;
    e0 = e[0]; e1 = e[1]; e2 = e[2];
  }
  const bool value = kind == MPF_OP_TAYLOR;
  if (j < NL) {
    const double d = -3.0 * id * rho * (e0 * xi0 + e1 * xi1 + e2 * xi2);
    return value ? rho * rho * rho + d : d;
  }
  int l = j - NL;
  return l == 0 ? (value ? 1.0 : 0.0) : (l == 1 ? e0 * id : (l == 2 ? e1 * id : (l == 3 ? e2 * id : 0.0)));
}

// Wave-wide maximum of an unsigned key: butterflies inside each row of 16
// lanes on DPP (quad permutes, half-row and row mirrors; register-to-register,
// no LDS crossbar), then the four row maxima through readlane.
__device__ __forceinline__ unsigned wave_max_u32(unsigned x) {
  x = max(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
  x = max(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
  x = max(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x141, 0xF, 0xF, false));  // row_half_mirror
  x = max(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x140, 0xF, 0xF, false));  // row_mirror
  const unsigned r0 = __builtin_amdgcn_readlane(x, 0), r1 = __builtin_amdgcn_readlane(x, 16);
  const unsigned r2 = __builtin_amdgcn_readlane(x, 32), r3 = __builtin_amdgcn_readlane(x, 48);
  return max(max(r0, r1), max(r2, r3));
}

// Pivot of column c: the lowest lane whose key equals the wave maximum, or -1
// if every key is zero.  Keys order candidates by magnitude: the high word of
// a non-negative double (exponent and 20 leading significand bits), so the
// pivot is within 2^-20 of the largest |a| (partial pivoting needs no more).
__device__ __forceinline__ int pivot_lane(unsigned key) {
  const unsigned mx = wave_max_u32(key);
  if (mx == 0u) return -1;
  return __builtin_amdgcn_readfirstlane(__builtin_ctzll(__ballot(key == mx)));
}

__device__ __forceinline__ float bcastf(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}

// Scaled local coordinates of stencil column `lane` (zero beyond NL):
// xi_j = minimg(x_j - x_c) / delta, delta the distance from the centre to
// stencil column 1 (Eq. rbfScaling).
template <int NL>
__device__ __forceinline__ void local_coords(const double* __restrict__ pos, int64_t n_nodes,
                                             const int32_t* __restrict__ sten, int64_t m, int64_t row, int lane,
                                             double& xi0, double& xi1, double& xi2, double& delta) {
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

// Row `lane` of M = [A P; P^T 0] (Eq. augmentedSystem; zero beyond N).
template <int NL>
__device__ __forceinline__ void assemble_row(int lane, double xi0, double xi1, double xi2, double (&a)[NL + 10]) {
  constexpr int N = NL + 10;
  const MonoPick pick(lane >= NL && lane < N ? lane - NL : 0);
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    double x0 = bcast(xi0, k), x1 = bcast(xi1, k), x2 = bcast(xi2, k);
    a[k] = lane < NL ? cube_dist(xi0, xi1, xi2, x0, x1, x2) : (lane < N ? pick(x0, x1, x2) : 0.0);
  }
#pragma unroll
  for (int l = 0; l < 10; ++l) a[NL + l] = lane < NL ? mono(l, xi0, xi1, xi2) : 0.0;
}

// Store weight j (the stencil column this lane solved for; none if j >= NL)
// of operator o: FP64 as solved, FP32 with the centre weight set so that the
// FP32 row sums to the operator's value on constants (1 for shifts and the
// Taylor row, 0 for derivatives), the sum taken in FP64 over the wave.
template <int NL>
__device__ __forceinline__ void store_weights(const OpsArg& ops, int o, int j, double x, double* __restrict__ w64,
                                              float* __restrict__ w32, int64_t m, int64_t row) {
  if (w64 && j < NL) w64[((int64_t)o * NL + j) * m + row] = x;
  if (w32) {
    float xf = (float)x;
    double part = (j >= 1 && j < NL) ? (double)xf : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    const int kd = ops.kind[o];
    const double target = (kd == MPF_OP_SHIFT || kd == MPF_OP_SHIFT_ROW || kd == MPF_OP_TAYLOR) ? 1.0 : 0.0;
    if (j == 0) xf = (float)(target - part);
    if (j < NL) w32[((int64_t)o * NL + j) * m + row] = xf;
  }
}

// 1/d from the hardware's approximate reciprocal and two Newton steps
// r <- r + r (1 - d r): within an ulp or so of the rounded quotient, for the
// normal, moderate pivots of these scaled systems.
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// Up to RB operators: Gauss-Jordan elimination of the augmented matrix
// [M | b_1 .. b_RB] with partial pivoting, rows in place.  Each pivot row is
// broadcast once and every other row (above and below) subtracts its
// multiple, right-hand sides included, so after the last column the pivot
// row of column c holds M'_cc x_c = b'_c and no substitution sweeps follow.
// The pivot choice is the LU's (same keys, same order), so the two agree to
// rounding.
template <int NL>
__device__ __forceinline__ void solve_row_gj(const double* __restrict__ pos, int64_t n_nodes,
                                             const int32_t* __restrict__ sten, int64_t m, int64_t row,
                                             const OpsArg& ops, const double* __restrict__ rowvec,
                                             double* __restrict__ w64, float* __restrict__ w32,
                                             int32_t* __restrict__ info, int lane) {
  constexpr int N = NL + 10;
  static_assert(N <= kWave, "system does not fit one wave");
  double xi0, xi1, xi2, delta;
  local_coords<NL>(pos, n_nodes, sten, m, row, lane, xi0, xi1, xi2, delta);
  const double rho = sqrt(xi0 * xi0 + xi1 * xi1 + xi2 * xi2);
  double a[N];
  assemble_row<NL>(lane, xi0, xi1, xi2, a);
  double rvv[3] = {0.0, 0.0, 0.0};
  if (rowvec) { rvv[0] = rowvec[row]; rvv[1] = rowvec[m + row]; rvv[2] = rowvec[2 * m + row]; }
  double b[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r)
    b[r] = (r < ops.n && lane < N) ? rhs_entry<NL>(ops.kind[r], ops.vec[r], rvv, lane, xi0, xi1, xi2, rho, delta)
                                   : 0.0;

  int pcol = (lane < N) ? 1 << 20 : -1;  // column at which this lane became pivot
  int bad = 0;
  double dinv = 0.0;
#pragma unroll
  for (int c = 0; c < N; ++c) {
    const unsigned key = (pcol > c) ? (unsigned)__double2hiint(fabs(a[c])) : 0u;
    const int p = pivot_lane(key);
    if (p < 0) { bad = c + 1; break; }
    const double piv = bcast(a[c], p);
    if (!(fabs(piv) > 0.0)) { bad = c + 1; break; }
    const double inv = recip(piv);
    if (lane == p) { pcol = c; dinv = inv; }
    // every row but the pivot's; a zero multiplier leaves a row as it is
    const double l = lane != p ? a[c] * inv : 0.0;
#pragma unroll
    for (int k = c + 1; k < N; ++k) a[k] = fma(-l, bcast(a[k], p), a[k]);
#pragma unroll
    for (int r = 0; r < RB; ++r) b[r] = fma(-l, bcast(b[r], p), b[r]);
  }
  const int j = (!bad && lane < N) ? pcol : kWave;  // the unknown this lane holds
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    if (r >= ops.n) break;
    store_weights<NL>(ops, r, bad ? lane : j, bad ? __builtin_nan("") : b[r] * dinv, w64, w32, m, row);
  }
  if (lane == 0) info[row] = bad;
}

template <int NL>
__device__ __forceinline__ void solve_row_fp64(const double* __restrict__ pos, int64_t n_nodes,
                                               const int32_t* __restrict__ sten, int64_t m, int64_t row,
                                               const OpsArg& ops, const double* __restrict__ rowvec,
                                               double* __restrict__ w64, float* __restrict__ w32,
                                               int32_t* __restrict__ info, int lane) {
  constexpr int N = NL + 10;
  static_assert(N <= kWave, "system does not fit one wave");

  double xi0, xi1, xi2, delta;
  local_coords<NL>(pos, n_nodes, sten, m, row, lane, xi0, xi1, xi2, delta);
  const double rho = sqrt(xi0 * xi0 + xi1 * xi1 + xi2 * xi2);
  double a[N];
  assemble_row<NL>(lane, xi0, xi1, xi2, a);

  // --- LU with partial pivoting, rows in place
  int pcol = (lane < N) ? 1 << 20 : -1;  // column at which this lane became pivot
  int bad = 0;
  double dinv = 0.0;  // 1 / pivot, kept by the lane that holds the pivot row
#pragma unroll
  for (int c = 0; c < N; ++c) {
    const unsigned key = (pcol > c) ? (unsigned)__double2hiint(fabs(a[c])) : 0u;
    const int p = pivot_lane(key);
    if (p < 0 || !(fabs(bcast(a[c], p)) > 0.0)) { bad = c + 1; break; }
    const double inv = 1.0 / bcast(a[c], p);
    const bool act = pcol > c && lane != p;
    if (lane == p) { pcol = c; dinv = inv; }
    // rows that are not eliminated here get a zero multiplier: fma(-0, u, a) = a
    const double l = act ? a[c] * inv : 0.0;
    if (act) a[c] = l;
#pragma unroll
    for (int k = c + 1; k < N; ++k) a[k] = fma(-l, bcast(a[k], p), a[k]);
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
        const double mc = pcol > c ? a[c] : 0.0;
#pragma unroll
        for (int r = 0; r < RB; ++r) b[r] = fma(-mc, bcast(b[r], p), b[r]);
      }
      // back substitution; lane c keeps unknown c
#pragma unroll
      for (int c = N - 1; c >= 0; --c) {
        const int p = __builtin_amdgcn_readfirstlane(__builtin_ctzll(__ballot(pcol == c)));
        const double uc = pcol < c ? a[c] : 0.0;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const double xc = bcast(b[r] * dinv, p);
          if (lane == c) x[r] = xc;
          b[r] = fma(-uc, xc, b[r]);
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < RB; ++r) x[r] = __builtin_nan("");
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      if (o0 + r >= ops.n) break;
      store_weights<NL>(ops, o0 + r, lane, x[r], w64, w32, m, row);
    }
  }
  if (lane == 0) info[row] = bad;
}


// FP32 factors with FP64-residual refinement for one stencil row (same lane
// layout as the FP64 solve).  Returns false if some chunk of right-hand sides
// has not settled after kIrSweeps sweeps (or the FP32 factorisation met a zero
// pivot); the caller then re-solves the row in FP64.
template <int NL>
__device__ __forceinline__ bool solve_row_ir(const double* __restrict__ pos, int64_t n_nodes,
                                             const int32_t* __restrict__ sten, int64_t m, int64_t row,
                                             const OpsArg& ops, const double* __restrict__ rowvec,
                                             double* __restrict__ w64, float* __restrict__ w32,
                                             int32_t* __restrict__ info, int lane) {
  constexpr int N = NL + 10;
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
  float a[N];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    double x0 = bcast(xi0, k), x1 = bcast(xi1, k), x2 = bcast(xi2, k);
    a[k] = (float)(lane < NL ? cube_dist(xi0, xi1, xi2, x0, x1, x2) : (lane < N ? mono(lane - NL, x0, x1, x2) : 0.0));
  }
#pragma unroll
  for (int l = 0; l < 10; ++l) a[NL + l] = (float)(lane < NL ? mono(l, xi0, xi1, xi2) : 0.0);
  int pcol = (lane < N) ? 1 << 20 : -1;
  float dinv = 0.0f;
#pragma unroll
  for (int c = 0; c < N; ++c) {
    const unsigned key = (pcol > c) ? __float_as_uint(fabsf(a[c])) : 0u;  // exact order for floats
    const int p = pivot_lane(key);
    if (p < 0) return false;
    const float inv = 1.0f / bcastf(a[c], p);
    const bool act = pcol > c && lane != p;
    if (lane == p) { pcol = c; dinv = inv; }
    const float l = act ? a[c] * inv : 0.0f;
    if (act) a[c] = l;
#pragma unroll
    for (int k = c + 1; k < N; ++k) a[k] = fmaf(-l, bcastf(a[k], p), a[k]);
  }
  double rvv[3] = {0.0, 0.0, 0.0};
  if (rowvec) { rvv[0] = rowvec[row]; rvv[1] = rowvec[m + row]; rvv[2] = rowvec[2 * m + row]; }
  for (int o0 = 0; o0 < ops.n; o0 += RB) {
    double b[RB], x[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      int o = o0 + r;
      b[r] = (o < ops.n && lane < N) ? rhs_entry<NL>(ops.kind[o], ops.vec[o], rvv, lane, xi0, xi1, xi2, rho, delta)
                                     : 0.0;
      x[r] = 0.0;
    }
    bool ok = false;
    double dprev = 0.0;
    // sweep 0 solves M x = b; later sweeps solve M d = b - M x (FP64 residual)
    for (int sweep = 0; sweep < 1 + kIrSweeps && !ok; ++sweep) {
      float rf[RB];
      if (sweep == 0) {
#pragma unroll
        for (int r = 0; r < RB; ++r) rf[r] = (float)b[r];
      } else {
        double s[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) s[r] = b[r];
#pragma unroll
        for (int k = 0; k < N; ++k) {
          double mk;
          if (k < NL) {
            double x0 = bcast(xi0, k), x1 = bcast(xi1, k), x2 = bcast(xi2, k);
            mk = lane < NL ? cube_dist(xi0, xi1, xi2, x0, x1, x2) : (lane < N ? mono(lane - NL, x0, x1, x2) : 0.0);
          } else {
            mk = lane < NL ? mono(k - NL, xi0, xi1, xi2) : 0.0;
          }
#pragma unroll
          for (int r = 0; r < RB; ++r) s[r] = fma(-mk, bcast(x[r], k), s[r]);
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) rf[r] = (float)(lane < N ? s[r] : 0.0);
      }
      // forward and back substitution with the FP32 factors
#pragma unroll
      for (int c = 0; c < N; ++c) {
        const int p = __builtin_amdgcn_readfirstlane(__builtin_ctzll(__ballot(pcol == c)));
        const float mc = pcol > c ? a[c] : 0.0f;
#pragma unroll
        for (int r = 0; r < RB; ++r) rf[r] = fmaf(-mc, bcastf(rf[r], p), rf[r]);
      }
      float d[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) d[r] = 0.0f;
#pragma unroll
      for (int c = N - 1; c >= 0; --c) {
        const int p = __builtin_amdgcn_readfirstlane(__builtin_ctzll(__ballot(pcol == c)));
        const float uc = pcol < c ? a[c] : 0.0f;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const float xc = bcastf(rf[r] * dinv, p);
          if (lane == c) d[r] = xc;
          rf[r] = fmaf(-uc, xc, rf[r]);
        }
      }
      double dmax = 0.0, xmax = 0.0;
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        x[r] += (double)d[r];
        if (lane < N && o0 + r < ops.n) {
          dmax = fmax(dmax, fabs((double)d[r]));
          xmax = fmax(xmax, fabs(x[r]));
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        dmax = fmax(dmax, __shfl_xor(dmax, off));
        xmax = fmax(xmax, __shfl_xor(xmax, off));
      }
      // converged: the correction is at FP64 resolution, or it has stopped
      // shrinking at the floor set by the FP64 residual (about cond(M) eps64,
      // the accuracy of a direct FP64 solve as well) while already small
      ok = sweep > 0 && (dmax <= 1e-15 * xmax || (sweep > 1 && dmax > 0.25 * dprev && dmax <= 1e-9 * xmax));
      dprev = dmax;
    }
    if (!ok) return false;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int o = o0 + r;
      if (o >= ops.n) break;
      if (w64 && lane < NL) w64[((int64_t)o * NL + lane) * m + row] = x[r];
      if (w32) {
        float xf = (float)x[r];
        double part = (lane >= 1 && lane < NL) ? (double)xf : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
        const int kd = ops.kind[o];
        const double target = (kd == MPF_OP_SHIFT || kd == MPF_OP_SHIFT_ROW || kd == MPF_OP_TAYLOR) ? 1.0 : 0.0;
        if (lane == 0) xf = (float)(target - part);
        if (lane < NL) w32[((int64_t)o * NL + lane) * m + row] = xf;
      }
    }
  }
  if (lane == 0) info[row] = 0;
  return true;
}

// How a launch solves its rows: LU with substitution sweeps (any number of
// operators), Gauss-Jordan (at most RB operators), or FP32 factors with
// FP64-residual refinement (LU in FP64 for the rows it cannot settle).
enum Path { kPathLU = 0, kPathGJ = 1, kPathIR = 2 };

template <int NL, int PATH>
__global__ __launch_bounds__(512) void weights_batched(const GeomArg* __restrict__ table, int n_geoms, int64_t total,
                                                       OpsArg ops, int rows_per_wave) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int64_t base = wave * rows_per_wave;
  const int64_t end = base + rows_per_wave < total ? base + rows_per_wave : total;
  for (int64_t r = base; r < end; ++r) {
    int g = 0;
    while (g + 1 < n_geoms && r >= table[g + 1].row0) ++g;
    const GeomArg G = table[g];
    const int64_t row = r - G.row0;
    if constexpr (PATH == kPathGJ) {
      solve_row_gj<NL>(G.pos, G.n_nodes, G.sten, G.m, row, ops, G.rowvec, G.w64, G.w32, G.info, lane);
    } else {
      bool done = false;
      if (PATH == kPathIR)
        done = solve_row_ir<NL>(G.pos, G.n_nodes, G.sten, G.m, row, ops, G.rowvec, G.w64, G.w32, G.info, lane);
      if (!done) {
        solve_row_fp64<NL>(G.pos, G.n_nodes, G.sten, G.m, row, ops, G.rowvec, G.w64, G.w32, G.info, lane);
        if (PATH == kPathIR && lane == 0 && G.info[row] == 0) G.info[row] = -1;
      }
    }
  }
}

struct Tune {
  int waves, rows;  // waves per block, consecutive rows per wave
};

template <int NL, int PATH>
int launch(const BatchArg& B, const OpsArg& ops, const Tune& t, const void* ws, hipStream_t st) {
  const int64_t rows_per_block = (int64_t)t.waves * t.rows;
  const int64_t blocks = (B.total + rows_per_block - 1) / rows_per_block;
  const GeomArg* table = reinterpret_cast<const GeomArg*>(reinterpret_cast<const char*>(ws) + kTableOffset);
  hipLaunchKernelGGL((weights_batched<NL, PATH>), dim3((unsigned)blocks), dim3(t.waves * kWave), 0, st, table,
                     B.n_geoms, B.total, ops, t.rows);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

template <int PATH>
int dispatch_nl(int nl, const BatchArg& B, const OpsArg& ops, const Tune& t, const void* ws, hipStream_t st) {
  switch (nl) {
    case 20: return launch<20, PATH>(B, ops, t, ws, st);
    case 25: return launch<25, PATH>(B, ops, t, ws, st);
    case 27: return launch<27, PATH>(B, ops, t, ws, st);
    case 30: return launch<30, PATH>(B, ops, t, ws, st);
    case 35: return launch<35, PATH>(B, ops, t, ws, st);
    case 40: return launch<40, PATH>(B, ops, t, ws, st);
    case 45: return launch<45, PATH>(B, ops, t, ws, st);
    case 50: return launch<50, PATH>(B, ops, t, ws, st);
    default: return MPF_ERR_UNSUPPORTED;
  }
}

int dispatch(int solve, int nl, const BatchArg& B, const OpsArg& ops, const Tune& t, const void* ws,
             hipStream_t st) {
  if (solve != MPF_SOLVE_FP64) return dispatch_nl<kPathIR>(nl, B, ops, t, ws, st);
  return ops.n <= RB ? dispatch_nl<kPathGJ>(nl, B, ops, t, ws, st) : dispatch_nl<kPathLU>(nl, B, ops, t, ws, st);
}
bool nl_supported(int nl) {
  return nl == 20 || nl == 25 || nl == 27 || nl == 30 || nl == 35 || nl == 40 || nl == 45 || nl == 50;
}

int make_ops(int n_ops, const mpf_op* ops, bool have_rowvec, OpsArg& a) {
  if (!ops || n_ops < 1 || n_ops > kMaxOps) return MPF_ERR_ARG;
  a = OpsArg{};
  a.n = n_ops;
  for (int o = 0; o < n_ops; ++o) {
    int k = ops[o].kind;
    if (k < MPF_OP_DX || k > MPF_OP_TAYLOR) return MPF_ERR_ARG;
    if ((k == MPF_OP_DN || k == MPF_OP_SHIFT_ROW) && !have_rowvec) return MPF_ERR_ARG;
    a.kind[o] = k;
    for (int t = 0; t < 3; ++t) a.vec[o][t] = ops[o].vec[t];
  }
  return MPF_OK;
}

int make_batch(int n_geoms, const mpf_wgeom* geoms, bool needs_rowvec, BatchArg& B) {
  if (n_geoms < 1 || n_geoms > kMaxGeoms || !geoms) return MPF_ERR_ARG;
  B = BatchArg{};
  B.n_geoms = n_geoms;
  int64_t row = 0;
  for (int g = 0; g < n_geoms; ++g) {
    const mpf_wgeom& s = geoms[g];
    if (!s.pos || !s.sten || !s.info || s.n_nodes < 2 || s.m < 0 || (!s.w64 && !s.w32)) return MPF_ERR_ARG;
    if (needs_rowvec && !s.rowvec) return MPF_ERR_ARG;
    B.g[g] = GeomArg{s.pos, s.n_nodes, s.sten, s.m, s.rowvec, s.w64, s.w32, s.info, row};
    row += s.m;
  }
  B.total = row;
  return MPF_OK;
}

bool ops_need_rowvec(int n_ops, const mpf_op* ops) {
  for (int o = 0; o < n_ops; ++o)
    if (ops[o].kind == MPF_OP_DN || ops[o].kind == MPF_OP_SHIFT_ROW) return true;
  return false;
}

const Tune kDefaultTune{4, 1};

}  // namespace
}  // namespace mpf

// The library context: its device and the autotune cache, (nl, n_ops,
// solve) -> tile shape.
struct mpf_ctx {
  int device = 0;
  std::mutex mu;
  std::map<std::tuple<int, int, int>, mpf::Tune> tune;
};

using namespace mpf;

extern "C" int mpf_create(mpf_ctx** out, int hip_device) {
  if (!out) return MPF_ERR_ARG;
  *out = nullptr;
  int count = 0;
  MPF_HIP(hipGetDeviceCount(&count));
  if (hip_device < 0 || hip_device >= count) return MPF_ERR_ARG;
  MPF_HIP(hipSetDevice(hip_device));
  mpf_ctx* c = new (std::nothrow) mpf_ctx;
  if (!c) return MPF_ERR_HIP;
  c->device = hip_device;
  *out = c;
  return MPF_OK;
}

extern "C" int mpf_destroy(mpf_ctx* ctx) {
  delete ctx;
  return MPF_OK;
}

extern "C" size_t mpf_weights_workspace(void) { return kWorkspaceBytes; }


namespace {
// The table lives in the caller's stack frame (pageable memory), and an
// asynchronous copy from pageable memory may read its source after the call
// has returned; wait for the copy so the frame outlives it.
int upload_table(const BatchArg& B, void* ws, hipStream_t st) {
  MPF_HIP(hipMemcpyAsync(reinterpret_cast<char*>(ws) + kTableOffset, B.g, sizeof(GeomArg) * B.n_geoms,
                         hipMemcpyHostToDevice, st));
  MPF_HIP(hipStreamSynchronize(st));
  return MPF_OK;
}
}  // namespace

extern "C" int mpf_rbffd_weights_batched(mpf_ctx* ctx, int n_geoms, const mpf_wgeom* geoms, int nl, int n_ops,
                                         const mpf_op* ops, int solve, const mpf_wtune* tune, void* ws,
                                         size_t ws_bytes, void* stream) {
  if (solve != MPF_SOLVE_FP64 && solve != MPF_SOLVE_FP32_IR) return MPF_ERR_ARG;
  if (!ops || n_ops < 1 || n_ops > kMaxOps) return MPF_ERR_ARG;
  const bool rv = ops_need_rowvec(n_ops, ops);
  OpsArg a;
  int rc = make_ops(n_ops, ops, true, a);
  if (rc) return rc;
  BatchArg B;
  rc = make_batch(n_geoms, geoms, rv, B);
  if (rc) return rc;
  if (!nl_supported(nl)) return MPF_ERR_UNSUPPORTED;
  if (!ws || ws_bytes < mpf_weights_workspace()) return MPF_ERR_WORKSPACE;
  if (B.total == 0) return MPF_OK;
  Tune t = kDefaultTune;
  if (tune) {
    if (tune->waves_per_block < 1 || tune->waves_per_block > 8 || tune->rows_per_wave < 1 || tune->rows_per_wave > 64)
      return MPF_ERR_ARG;
    t = Tune{tune->waves_per_block, tune->rows_per_wave};
  } else if (ctx) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->tune.find(std::make_tuple(nl, n_ops, solve));
    if (it != ctx->tune.end()) t = it->second;
  }
  hipStream_t st = as_stream(stream);
  rc = upload_table(B, ws, st);
  if (rc) return rc;
  return dispatch(solve, nl, B, a, t, ws, st);
}

extern "C" int mpf_weights_autotune(mpf_ctx* ctx, int nl, int n_ops, const mpf_op* ops, int solve,
                                    const mpf_wgeom* sample, int64_t sample_rows, mpf_wtune* out, void* ws,
                                    size_t ws_bytes) {
  if (!ctx || !sample || !out || sample_rows < 1) return MPF_ERR_ARG;
  if (solve != MPF_SOLVE_FP64 && solve != MPF_SOLVE_FP32_IR) return MPF_ERR_ARG;
  if (!nl_supported(nl)) return MPF_ERR_UNSUPPORTED;
  if (!ws || ws_bytes < mpf_weights_workspace()) return MPF_ERR_WORKSPACE;
  OpsArg a;
  int rc = make_ops(n_ops, ops, sample->rowvec != nullptr, a);
  if (rc) return rc;
  mpf_wgeom g = *sample;
  g.m = std::min<int64_t>(g.m, sample_rows);
  BatchArg B;
  rc = make_batch(1, &g, ops_need_rowvec(n_ops, ops), B);
  if (rc) return rc;
  MPF_HIP(hipSetDevice(ctx->device));
  hipStream_t st = nullptr;
  MPF_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  rc = upload_table(B, ws, st);
  if (rc) return rc;
  hipEvent_t e0, e1;
  MPF_HIP(hipEventCreate(&e0));
  MPF_HIP(hipEventCreate(&e1));
  Tune best = kDefaultTune;
  float best_ms = 1e30f;
  const int waves[] = {1, 2, 4, 8};
  const int rows[] = {1, 2, 4, 8};
  int err = MPF_OK;
  for (int w : waves) {
    for (int rr : rows) {
      Tune t{w, rr};
      rc = dispatch(solve, nl, B, a, t, ws, st);
      if (rc) { err = rc; break; }
      (void)hipEventRecord(e0, st);
      rc = dispatch(solve, nl, B, a, t, ws, st);
      (void)hipEventRecord(e1, st);
      if (rc) { err = rc; break; }
      if (hipEventSynchronize(e1) != hipSuccess) { err = MPF_ERR_HIP; break; }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best_ms) { best_ms = ms; best = t; }
    }
    if (err) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(st);
  if (err) return err;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->tune[std::make_tuple(nl, n_ops, solve)] = best;
  }
  out->waves_per_block = best.waves;
  out->rows_per_wave = best.rows;
  return MPF_OK;
}

extern "C" int mpf_rbffd_weights(const double* pos, int64_t n_nodes, const int32_t* sten, int64_t m, int nl,
                                 int n_ops, const mpf_op* ops, const double* rowvec, double* w64, float* w32,
                                 int32_t* info, void* ws, size_t ws_bytes, void* stream) {
  if (!pos || !sten || !ops || !info || n_nodes < 2 || m < 0 || n_ops < 1 || n_ops > kMaxOps) return MPF_ERR_ARG;
  if (!w64 && !w32) return MPF_ERR_ARG;
  if (ops_need_rowvec(n_ops, ops) && !rowvec) return MPF_ERR_ARG;
  for (int o = 0; o < n_ops; ++o)
    if (ops[o].kind < MPF_OP_DX || ops[o].kind > MPF_OP_TAYLOR) return MPF_ERR_ARG;
  if (!nl_supported(nl)) return MPF_ERR_UNSUPPORTED;
  if (m == 0) return MPF_OK;
  mpf_wgeom g{pos, n_nodes, sten, m, rowvec, w64, w32, info};
  return mpf_rbffd_weights_batched(nullptr, 1, &g, nl, n_ops, ops, MPF_SOLVE_FP64, nullptr, ws, ws_bytes, stream);
}
