/*
 * CPU reference ("oracle") for the meshless pore-flow solvers of
 * Strzelczyk, Rot, Kosec, Matyka, "Cross-validation of meshless Navier-Stokes
 * solvers in porous media flows" (arXiv 2404.14195).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, scalar FP64
 * restatement of the paper's method.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load or call it; the product
 * library never does, and it shares no source with the HIP kernels.
 *
 * Every function follows the paper's steps in the paper's order:
 *   - Stencils: Sec. 2.1, the N_L nearest nodes of each node, by brute force.
 *   - RBF-FD weights: Sec. 2.1, Eqs. operatorApprox, rbfScaling,
 *     augmentedSystem (PHS r^3, monomials up to degree 2, local scaling by the
 *     distance to the nearest neighbour), solved by Gaussian elimination with
 *     partial pivoting.
 *   - ACM Navier-Stokes step: Sec. 2.3, Eqs. MNS_intermediate, MNS_pressure,
 *     MNS_velocity, MNS_C, and the MNS algorithm of Appendix A.
 *   - MLBM step: Sec. 2.2, Eqs. LBM_streaming, LBM_collision, feq, macro_var,
 *     force_lbm, interpolated_bounceback_mlbm, and the MLBM algorithm of
 *     Appendix A (collide everywhere, then stream by interpolation).
 *   - Permeability: Eq. k_definition (plane averages of v_x).
 *   - Hydrodynamic force: Eqs. stress_tensor_force, integration_force.
 *
 * Layouts are the natural row-major ones: positions [N][3], stencils [m][nl],
 * weights [m][n_ops][nl], velocities [N][3], populations [N][q].
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -std=c11 -shared -fPIC mpf_oracle.c
 *        -o libmpf_oracle.so -lm
 *
 * Threads: one by default.  mpfo_set_threads() lets the MLBM node loops run
 * on several host threads (an OpenMP parallel loop over nodes; every node's
 * arithmetic is the same in the same order, so results are identical for any
 * thread count).  It exists only to time the oracle on all host cores.
 */
#define _DEFAULT_SOURCE /* M_PI */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Host threads of the MLBM node loops (1 unless set); returns the count in
 * effect. */
static int g_threads = 1;
int mpfo_set_threads(int n) {
  g_threads = n < 1 ? 1 : n;
  return g_threads;
}

/* ------------------------------------------------------------------ geometry */

/* Minimum-image displacement in the unit periodic cell. */
static double mi(double d) { return d - nearbyint(d); }

/* Porosity of the simple-cubic cell of side 1 with a sphere of radius r
 * centred in it (Sec. 2.4).  For r > 1/2 the six caps beyond the faces are
 * removed; the images' caps that enter the cell lie inside the central sphere.
 * Valid for r < sqrt(2)/2. */
double mpfo_porosity(double r) {
  double vs = 4.0 / 3.0 * M_PI * r * r * r;
  if (r > 0.5) {
    double hc = r - 0.5;
    vs -= 6.0 * M_PI * hc * hc * (3.0 * r - hc) / 3.0;
  }
  return 1.0 - vs;
}

/* Area of the grain surface inside the cell (the A of Delta A = A / N_b). */
double mpfo_area(double r) {
  double a = 4.0 * M_PI * r * r;
  if (r > 0.5) a -= 6.0 * 2.0 * M_PI * r * (r - 0.5);
  return a;
}

/* ------------------------------------------------------------------ stencils */

/* Squared minimum-image distance from q to p: each coordinate difference
 * t = p_a - q_a is reduced by t - nearbyint(t), and the squares are summed
 * x, y, z, every operation rounded on its own (x86-64 SSE2 doubles, no
 * contraction).  Fixing the operations fixes ties to the last bit. */
static double dist2(const double* p, const double* q) {
  double t0 = mi(p[0] - q[0]), t1 = mi(p[1] - q[1]), t2 = mi(p[2] - q[2]);
  double s = t0 * t0;
  s = s + t1 * t1;
  return s + t2 * t2;
}

/* The k nearest of the n points pts [n][3] to each query qry [m][3] in the
 * unit periodic cell, nearest first: the stencil of Sec. 2.1 ("the N_L
 * nearest nodes").  Order: squared distance (dist2), then point index.  Brute
 * force over every point, keeping a sorted list by insertion.  Output
 * idx [m][k].  Returns -1 unless 1 <= k <= n. */
int mpfo_knn(const double* pts, int64_t n, const double* qry, int64_t m, int k, int32_t* idx) {
  if (k < 1 || (int64_t)k > n) return -1;
  double* bd = (double*)malloc(sizeof(double) * k);
  int32_t* bi = (int32_t*)malloc(sizeof(int32_t) * k);
  for (int64_t j = 0; j < m; ++j) {
    int cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
      double d = dist2(pts + 3 * i, qry + 3 * j);
      int32_t ii = (int32_t)i;
      if (cnt == k && !(d < bd[k - 1] || (d == bd[k - 1] && ii < bi[k - 1]))) continue;
      int p = cnt < k ? cnt : k - 1;
      while (p > 0 && (bd[p - 1] > d || (bd[p - 1] == d && bi[p - 1] > ii))) {
        bd[p] = bd[p - 1];
        bi[p] = bi[p - 1];
        --p;
      }
      bd[p] = d;
      bi[p] = ii;
      if (cnt < k) ++cnt;
    }
    for (int c = 0; c < k; ++c) idx[j * k + c] = bi[c];
  }
  free(bd);
  free(bi);
  return 0;
}

/* ------------------------------------------------------------------ weights */

enum { OP_DX = 0, OP_DY = 1, OP_DZ = 2, OP_LAP = 3, OP_DIR = 4, OP_SHIFT = 5, OP_DN = 6, OP_SHIFT_ROW = 7, OP_TAYLOR = 8 };

#define NP 10 /* monomials 1, x, y, z, x^2, xy, xz, y^2, yz, z^2 (m = 2, D = 3) */

static void monomials(const double* x, double* p) {
  p[0] = 1.0;
  p[1] = x[0]; p[2] = x[1]; p[3] = x[2];
  p[4] = x[0] * x[0]; p[5] = x[0] * x[1]; p[6] = x[0] * x[2];
  p[7] = x[1] * x[1]; p[8] = x[1] * x[2]; p[9] = x[2] * x[2];
}

/* Right-hand side [b; c] of the augmented system for the first derivative
 * along unit axis a, at the centre (xi = 0), in scaled coordinates:
 *   b_j = d/dx_a |xi(x) - xi_j|^3 at x_i = -(3/delta) |xi_j| xi_j,a
 *   c_l = d/dx_a p_l(xi(x)) at x_i   = 1/delta for the linear monomial x_a. */
static void rhs_axis(int a, int nl, const double* xi, const double* rho, double delta, double scale,
                     double* rhs) {
  for (int j = 0; j < nl; ++j) rhs[j] += scale * (-3.0 / delta) * rho[j] * xi[3 * j + a];
  rhs[nl + 1 + a] += scale / delta;
}

/* Solve M X = B for n x n M and k right-hand sides by Gaussian elimination
 * with partial (row) pivoting.  M is row-major and destroyed; B is [n][k]
 * row-major and overwritten by X.  Returns 0, or 1 + the column of a zero
 * pivot. */
static int solve_gepp(int n, int k, double* M, double* B) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    double best = fabs(M[c * n + c]);
    for (int r = c + 1; r < n; ++r) {
      double v = fabs(M[r * n + c]);
      if (v > best) { best = v; piv = r; }
    }
    if (best == 0.0) return 1 + c;
    if (piv != c) {
      for (int j = 0; j < n; ++j) { double t = M[c * n + j]; M[c * n + j] = M[piv * n + j]; M[piv * n + j] = t; }
      for (int j = 0; j < k; ++j) { double t = B[c * k + j]; B[c * k + j] = B[piv * k + j]; B[piv * k + j] = t; }
    }
    for (int r = c + 1; r < n; ++r) {
      double l = M[r * n + c] / M[c * n + c];
      if (l == 0.0) continue;
      for (int j = c + 1; j < n; ++j) M[r * n + j] -= l * M[c * n + j];
      for (int j = 0; j < k; ++j) B[r * k + j] -= l * B[c * k + j];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    for (int j = 0; j < k; ++j) {
      double s = B[c * k + j];
      for (int t = c + 1; t < n; ++t) s -= M[c * n + t] * B[t * k + j];
      B[c * k + j] = s / M[c * n + c];
    }
  }
  return 0;
}

/* RBF-FD weights (Eq. operatorApprox) for m stencil rows.
 *
 * Row i has stencil nodes S_i(0..nl-1) = sten[i*nl + j]; S_i(0) is the centre
 * x_i.  The local scale delta_i is the distance from x_i to S_i(1) (its
 * nearest neighbour when the stencil is the nl nearest nodes), Eq. rbfScaling.
 * Operators (kind[o], vec[o*3..]):
 *   OP_DX/DY/DZ  d/dx_a          OP_LAP     Laplacian
 *   OP_DIR       vec . grad      OP_DN      rowvec_i . grad (row normal)
 *   OP_SHIFT     value at x_i + vec         OP_SHIFT_ROW value at x_i + rowvec_i
 *   OP_TAYLOR    value at x_i plus vec . grad (the first-order Taylor
 *                estimate of the value at x_i + vec)
 * Output w[(i*n_ops + o)*nl + j]; info[i] = 0 or 1 + zero-pivot column. */
int mpfo_weights(const double* pos, int64_t n_nodes, const int32_t* sten, int64_t m, int nl, int n_ops,
                 const int32_t* kind, const double* vec, const double* rowvec, double* w, int32_t* info) {
  if (nl < NP + 1 || n_ops < 1) return -1;
  const int n = nl + NP;
  double* M = (double*)malloc(sizeof(double) * n * n);
  double* B = (double*)malloc(sizeof(double) * n * n_ops);
  double* xi = (double*)malloc(sizeof(double) * 3 * nl);
  double* rho = (double*)malloc(sizeof(double) * nl);
  int bad = 0;
  for (int64_t i = 0; i < m; ++i) {
    const int32_t* S = sten + i * nl;
    for (int j = 0; j < nl; ++j)
      if (S[j] < 0 || S[j] >= n_nodes) bad = 1;
    if (bad) break;
    const double* xc = pos + 3 * (int64_t)S[0];
    double d1[3];
    for (int a = 0; a < 3; ++a) d1[a] = mi(pos[3 * (int64_t)S[1] + a] - xc[a]);
    double delta = sqrt(d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2]);
    for (int j = 0; j < nl; ++j) {
      double s2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        double d = mi(pos[3 * (int64_t)S[j] + a] - xc[a]) / delta;
        xi[3 * j + a] = d;
        s2 += d * d;
      }
      rho[j] = sqrt(s2);
    }
    /* M = [A P; P^T 0], A_jk = |xi_j - xi_k|^3, P_jl = p_l(xi_j) */
    for (int j = 0; j < nl; ++j) {
      for (int k = 0; k < nl; ++k) {
        double dx = xi[3 * j] - xi[3 * k], dy = xi[3 * j + 1] - xi[3 * k + 1], dz = xi[3 * j + 2] - xi[3 * k + 2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        M[j * n + k] = r * r * r;
      }
      double p[NP];
      monomials(xi + 3 * j, p);
      for (int l = 0; l < NP; ++l) { M[j * n + nl + l] = p[l]; M[(nl + l) * n + j] = p[l]; }
    }
    for (int l = 0; l < NP; ++l)
      for (int t = 0; t < NP; ++t) M[(nl + l) * n + nl + t] = 0.0;
    /* right-hand sides, one column per operator */
    double* col = (double*)calloc(n, sizeof(double));
    for (int o = 0; o < n_ops; ++o) {
      memset(col, 0, sizeof(double) * n);
      const double* v = vec + 3 * o;
      const double* rv = rowvec ? rowvec + 3 * i : NULL;
      switch (kind[o]) {
        case OP_DX: case OP_DY: case OP_DZ:
          rhs_axis(kind[o] - OP_DX, nl, xi, rho, delta, 1.0, col);
          break;
        case OP_LAP: /* lap r^3 = 3*(3+3-2) r = 12 r; lap of x^2, y^2, z^2 = 2 */
          for (int j = 0; j < nl; ++j) col[j] = 12.0 * rho[j] / (delta * delta);
          col[nl + 4] = col[nl + 7] = col[nl + 9] = 2.0 / (delta * delta);
          break;
        case OP_DIR:
          for (int a = 0; a < 3; ++a) rhs_axis(a, nl, xi, rho, delta, v[a], col);
          break;
        case OP_DN:
          if (!rv) { bad = 2; break; }
          for (int a = 0; a < 3; ++a) rhs_axis(a, nl, xi, rho, delta, rv[a], col);
          break;
        case OP_TAYLOR: /* value at the centre (xi = 0) plus the directional derivative */
          for (int j = 0; j < nl; ++j) col[j] = rho[j] * rho[j] * rho[j];
          col[nl] = 1.0;
          for (int a = 0; a < 3; ++a) rhs_axis(a, nl, xi, rho, delta, v[a], col);
          break;
        case OP_SHIFT: case OP_SHIFT_ROW: {
          const double* s = kind[o] == OP_SHIFT ? v : rv;
          if (!s) { bad = 2; break; }
          double sg[3] = {s[0] / delta, s[1] / delta, s[2] / delta};
          for (int j = 0; j < nl; ++j) {
            double dx = sg[0] - xi[3 * j], dy = sg[1] - xi[3 * j + 1], dz = sg[2] - xi[3 * j + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            col[j] = r * r * r;
          }
          monomials(sg, col + nl);
          break;
        }
        default:
          bad = 3;
      }
      for (int j = 0; j < n; ++j) B[j * n_ops + o] = col[j];
    }
    free(col);
    if (bad) break;
    info[i] = solve_gepp(n, n_ops, M, B);
    for (int o = 0; o < n_ops; ++o)
      for (int j = 0; j < nl; ++j) w[(i * n_ops + o) * nl + j] = B[j * n_ops + o];
  }
  free(M); free(B); free(xi); free(rho);
  return bad ? -bad : 0;
}

/* ------------------------------------------------------------------ ACM */

/* Artificial-compressibility Navier-Stokes, explicit Euler (Sec. 2.3).
 *
 * Nodes [0, n_int) are interior, [n_int, n) boundary.  w holds, for every
 * node, the weights of d/dx, d/dy, d/dz and the Laplacian: w[(i*4+o)*nl+j].
 * wn[(b*nl)+j] are the normal-derivative weights of boundary node n_int+b on
 * the stencil sn[b*nl + j] (column 0 is the node itself).  v [n][3] (zero on the boundary) and p [n] are updated in
 * place; *C carries the artificial sound speed between calls.
 *
 * One step: intermediate velocity v' (pressure term omitted) on interior
 * nodes, v = 0 on the boundary; then n_p coupling iterations, each one
 *   p_i <- p_i - dt C^2 rho (div v)_i      (interior; v is v' at the first)
 *   boundary p from dp/dn = 0, solved for the node's own value with the
 *     neighbours' current values (Jacobi over boundary nodes)
 *   v_i <- v'_i - (dt/rho) (grad p)_i       (interior)
 *   C = beta * max(max_i |v_i|, |v_ref|).
 * edac = 1 takes the entropically damped form of the pressure equation that
 * Sec. 2.3 names as the remedy for the pressure oscillations of Sec. 3.6,
 * dp/dt + v . grad p = -rho C^2 div v + nu lap p, as the pressure update:
 *   p_i <- p_i + dt (-C^2 rho (div v)_i - v_i . (grad p)_i + nu (lap p)_i)
 * with every term from the pressure before the update (Jacobi). */
int mpfo_acm_run(int64_t n, int64_t n_int, int nl, const int32_t* sten, const double* w, const int32_t* sn,
                 const double* wn,
                 double nu, double rho, double dt, double beta, double v_ref, const double* g, int n_p,
                 double* v, double* p, double* C, int n_steps, int edac) {
  const int64_t nb = n - n_int;
  double* vp = (double*)malloc(sizeof(double) * 3 * n);
  double* pb = (double*)malloc(sizeof(double) * (nb > 0 ? nb : 1));
  double* pold = (double*)malloc(sizeof(double) * n);
  for (int step = 0; step < n_steps; ++step) {
    /* intermediate velocity, Eq. MNS_intermediate */
    for (int64_t i = 0; i < n_int; ++i) {
      const int32_t* S = sten + i * nl;
      const double* wx = w + (i * 4 + 0) * nl;
      const double* wy = w + (i * 4 + 1) * nl;
      const double* wz = w + (i * 4 + 2) * nl;
      const double* wl = w + (i * 4 + 3) * nl;
      for (int a = 0; a < 3; ++a) {
        double gx = 0.0, gy = 0.0, gz = 0.0, lap = 0.0;
        for (int j = 0; j < nl; ++j) {
          double u = v[3 * (int64_t)S[j] + a];
          gx += wx[j] * u; gy += wy[j] * u; gz += wz[j] * u; lap += wl[j] * u;
        }
        double adv = v[3 * i + 0] * gx + v[3 * i + 1] * gy + v[3 * i + 2] * gz;
        vp[3 * i + a] = v[3 * i + a] + dt * (nu * lap - adv + g[a]);
      }
    }
    for (int64_t i = n_int; i < n; ++i) vp[3 * i] = vp[3 * i + 1] = vp[3 * i + 2] = 0.0;
    memcpy(v, vp, sizeof(double) * 3 * n);
    /* pressure-velocity coupling */
    for (int it = 0; it < n_p; ++it) {
      double c2 = (*C) * (*C);
      memcpy(pold, p, sizeof(double) * n);
      for (int64_t i = 0; i < n_int; ++i) { /* Eq. MNS_pressure */
        const int32_t* S = sten + i * nl;
        const double* wx = w + (i * 4 + 0) * nl;
        const double* wy = w + (i * 4 + 1) * nl;
        const double* wz = w + (i * 4 + 2) * nl;
        const double* wl = w + (i * 4 + 3) * nl;
        double div = 0.0;
        for (int j = 0; j < nl; ++j) {
          const double* u = v + 3 * (int64_t)S[j];
          div += wx[j] * u[0] + wy[j] * u[1] + wz[j] * u[2];
        }
        if (!edac) {
          p[i] -= dt * c2 * rho * div;
          continue;
        }
        double gp[3] = {0.0, 0.0, 0.0}, lp = 0.0;
        for (int j = 0; j < nl; ++j) {
          double q = pold[S[j]];
          gp[0] += wx[j] * q; gp[1] += wy[j] * q; gp[2] += wz[j] * q; lp += wl[j] * q;
        }
        double adv = v[3 * i] * gp[0] + v[3 * i + 1] * gp[1] + v[3 * i + 2] * gp[2];
        p[i] = pold[i] + dt * (-c2 * rho * div - adv + nu * lp);
      }
      for (int64_t b = 0; b < nb; ++b) { /* dp/dn = 0 on the grain */
        const int32_t* S = sn + b * nl;
        const double* wb = wn + b * nl;
        double s = 0.0;
        for (int j = 1; j < nl; ++j) s += wb[j] * p[S[j]];
        pb[b] = -s / wb[0];
      }
      for (int64_t b = 0; b < nb; ++b) p[n_int + b] = pb[b];
      double vmax = 0.0;
      for (int64_t i = 0; i < n_int; ++i) { /* Eq. MNS_velocity */
        const int32_t* S = sten + i * nl;
        double gp[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 3; ++a) {
          const double* wa = w + (i * 4 + a) * nl;
          for (int j = 0; j < nl; ++j) gp[a] += wa[j] * p[S[j]];
        }
        for (int a = 0; a < 3; ++a) v[3 * i + a] = vp[3 * i + a] - dt / rho * gp[a];
        double m = sqrt(v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2]);
        if (m > vmax) vmax = m;
      }
      *C = beta * (vmax > v_ref ? vmax : v_ref); /* Eq. MNS_C */
    }
  }
  free(vp); free(pb); free(pold);
  return 0;
}

/* ------------------------------------------------------------------ MLBM */

/* Velocity sets.  D3Q15 is the paper's (Sec. 2.2): rest, the three axes at odd
 * k = 1, 3, 5, the diagonals (1,1,1), (1,1,-1), (1,-1,1), (1,-1,-1) at odd
 * k = 7..13, and e_k = -e_{k-1} for even k; weights 2/9, 1/9, 1/72.
 * D3Q19 follows the same pairing: rest; odd k = 1, 3, 5 the axes x, y, z;
 * odd k = 7..17 the edge vectors (1,1,0), (1,-1,0), (1,0,1), (1,0,-1),
 * (0,1,1), (0,1,-1); even k the opposite of k-1; weights 1/3, 1/18, 1/36. */
static const int Q15_POS[7][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};
static const int Q19_POS[9][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, -1, 0},
                                  {1, 0, 1}, {1, 0, -1}, {0, 1, 1}, {0, 1, -1}};

/* Fill e [q][3] (as doubles), weights [q], opposite [q]; returns 0 or -1. */
int mpfo_lattice(int q, double* e, double* wk, int32_t* opp) {
  int npos;
  const int(*pos)[3];
  if (q == 15) { npos = 7; pos = Q15_POS; }
  else if (q == 19) { npos = 9; pos = Q19_POS; }
  else return -1;
  e[0] = e[1] = e[2] = 0.0;
  opp[0] = 0;
  for (int t = 0; t < npos; ++t) {
    int k = 2 * t + 1;
    for (int a = 0; a < 3; ++a) { e[3 * k + a] = pos[t][a]; e[3 * (k + 1) + a] = -pos[t][a]; }
    opp[k] = k + 1;
    opp[k + 1] = k;
  }
  for (int k = 0; k < q; ++k) {
    double n2 = e[3 * k] * e[3 * k] + e[3 * k + 1] * e[3 * k + 1] + e[3 * k + 2] * e[3 * k + 2];
    if (q == 15) wk[k] = n2 == 0.0 ? 2.0 / 9.0 : (n2 == 1.0 ? 1.0 / 9.0 : 1.0 / 72.0);
    else wk[k] = n2 == 0.0 ? 1.0 / 3.0 : (n2 == 1.0 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
  return 0;
}

/* Second-order equilibrium, Eq. feq, with c_s^2 = 1/3. */
static void equilibrium(int q, const double* e, const double* wk, double rho, const double* u, double* feq) {
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int k = 0; k < q; ++k) {
    double eu = e[3 * k] * u[0] + e[3 * k + 1] * u[1] + e[3 * k + 2] * u[2];
    feq[k] = rho * wk[k] * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
  }
}

/* Density and velocity, Eq. macro_var. */
static void moments(int q, const double* e, const double* f, double* rho, double* u) {
  double r = 0.0, m[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < q; ++k) {
    r += f[k];
    for (int a = 0; a < 3; ++a) m[a] += f[k] * e[3 * k + a];
  }
  *rho = r;
  for (int a = 0; a < 3; ++a) u[a] = m[a] / r;
}

void mpfo_lbm_equilibrium(int q, int64_t n, double rho, const double* u, double* f) {
  double e[3 * 19], wk[19];
  int32_t opp[19];
  mpfo_lattice(q, e, wk, opp);
  for (int64_t i = 0; i < n; ++i) equilibrium(q, e, wk, rho, u, f + i * q);
}

void mpfo_lbm_moments(int q, int64_t n, const double* f, double* rho, double* u) {
  double e[3 * 19], wk[19];
  int32_t opp[19];
  mpfo_lattice(q, e, wk, opp);
  for (int64_t i = 0; i < n; ++i) moments(q, e, f + i * q, rho + i, u + 3 * i);
}

/* TRT collision with forcing, Eqs. LBM_collision, feq, force_lbm, applied to
 * one node's populations f[q] -> fpost[q]. */
static void collide(int q, const double* e, const double* wk, const int32_t* opp, double tau_p, double tau_m,
                    const double* g_lb, const double* f, double* fpost) {
  double rho, u[3], feq[19], F[3];
  moments(q, e, f, &rho, u);
  equilibrium(q, e, wk, rho, u, feq);
  for (int a = 0; a < 3; ++a) F[a] = rho * g_lb[a];
  for (int k = 0; k < q; ++k) {
    int kb = opp[k];
    double fp = 0.5 * (f[k] + f[kb]), fm = 0.5 * (f[k] - f[kb]);
    double ep = 0.5 * (feq[k] + feq[kb]), em = 0.5 * (feq[k] - feq[kb]);
    double Fk = wk[k] * 3.0 * (e[3 * k] * F[0] + e[3 * k + 1] * F[1] + e[3 * k + 2] * F[2]);
    fpost[k] = f[k] - (fp - ep) / tau_p - (fm - em) / tau_m + Fk;
  }
}

/* Which populations of boundary node b are unknown after streaming, as a bit
 * mask (bit k for population k; the rest population is never unknown).
 *   rule 0 (Sec. 2.2, Eq. interpolated_bounceback_mlbm): the local normal
 *     decides, e_k . n_b > 0 with n_b [nb][3] pointing into the fluid: the
 *     departure point x_b - dx e_k is on the solid side of the tangent plane.
 *   rule 1 (Sec. 3.3, the touching limit): the departure point itself is
 *     tested, unknown when it lies inside the solid.  The solid is the union
 *     of the balls of radius r centred at (1/2, 1/2, 1/2) + Z^3; for a point of
 *     the unit cell moved by less than 1/2 the nearest centres are the 27
 *     images with offsets in {-1, 0, 1}^3, and all of them are tested.
 * pos_b [nb][3] boundary positions in the unit cell. */
int mpfo_lbm_unknown(int q, int64_t nb, const double* pos_b, const double* nrm, int rule, double dx, double r,
                     uint32_t* unknown) {
  double e[3 * 19], wk[19];
  int32_t opp[19];
  if (mpfo_lattice(q, e, wk, opp) || rule < 0 || rule > 1) return -1;
  if (rule == 1 && !(dx > 0.0 && dx < 0.5)) return -1;
  for (int64_t b = 0; b < nb; ++b) {
    uint32_t mask = 0;
    for (int k = 1; k < q; ++k) {
      int out = 0;
      if (rule == 0) {
        const double* nv = nrm + 3 * b;
        out = e[3 * k] * nv[0] + e[3 * k + 1] * nv[1] + e[3 * k + 2] * nv[2] > 0.0;
      } else {
        double p[3];
        for (int a = 0; a < 3; ++a) p[a] = pos_b[3 * b + a] - dx * e[3 * k + a];
        for (int i = -1; i <= 1 && !out; ++i)
          for (int j = -1; j <= 1 && !out; ++j)
            for (int l = -1; l <= 1 && !out; ++l) {
              double d0 = p[0] - (0.5 + i), d1 = p[1] - (0.5 + j), d2 = p[2] - (0.5 + l);
              out = d0 * d0 + d1 * d1 + d2 * d2 < r * r;
            }
      }
      if (out) mask |= 1u << k;
    }
    unknown[b] = mask;
  }
  return 0;
}

/* Meshless LBM (Sec. 2.2, MLBM algorithm of Appendix A), n_steps steps.
 *
 * f [n][q] holds the populations at the start of a step.  W[(i*q + k)*nl + j]
 * are, for each moving population k >= 1, the weights that interpolate a
 * field at the departure point of node i for that population (row k = 0 is
 * not read: the rest population does not move).  Boundary nodes are
 * [n_int, n); bit k of unknown[b] marks population k of boundary node
 * n_int + b as unknown (mpfo_lbm_unknown gives the two rules).
 * Per step: collide on every node; stream each moving population by
 * interpolating its post-collision field at the departure point (Eq.
 * LBM_streaming with Eq. operatorApprox, L = 1); at boundary nodes an unknown
 * population takes the streamed value of its opposite (Eq.
 * interpolated_bounceback_mlbm).  When both members of a pair are unknown
 * (the solid rule allows it) each takes the other's streamed value. */
int mpfo_lbm_run(int q, int64_t n, int64_t n_int, int nl, const int32_t* sten, const double* W,
                 const uint32_t* unknown, double tau_p, double tau_m, const double* g_lb, double* f, int n_steps) {
  double e[3 * 19], wk[19];
  int32_t opp[19];
  if (mpfo_lattice(q, e, wk, opp)) return -1;
  double* fpost = (double*)malloc(sizeof(double) * q * n);
  for (int step = 0; step < n_steps; ++step) {
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (int64_t i = 0; i < n; ++i) collide(q, e, wk, opp, tau_p, tau_m, g_lb, f + i * q, fpost + i * q);
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      const int32_t* S = sten + i * nl;
      f[i * q] = fpost[i * q];
      for (int k = 1; k < q; ++k) {
        const double* Wk = W + (i * q + k) * nl;
        double s = 0.0;
        for (int j = 0; j < nl; ++j) s += Wk[j] * fpost[(int64_t)S[j] * q + k];
        f[i * q + k] = s;
      }
    }
    for (int64_t i = n_int; i < n; ++i) {
      const uint32_t mask = unknown[i - n_int];
      double streamed[19];
      for (int k = 0; k < q; ++k) streamed[k] = f[i * q + k];
      for (int k = 1; k < q; ++k)
        if (mask >> k & 1u) f[i * q + k] = streamed[opp[k]];
    }
  }
  free(fpost);
  return 0;
}

/* ------------------------------------------------------------------ reductions */

/* Mean x-velocity over the cross-sections, Eq. k_definition: the integral
 * over each plane is the mean over its M x M midpoint samples, the planes are
 * averaged, so q = (sum over fluid samples of v_x) / n_all with n_all = all
 * samples of all planes.  Sample s interpolates v_x from its stencil
 * s_idx[s][.] with weights s_w[s][.]; solid samples contribute zero. */
double mpfo_flux(int64_t ns, int nl, const int32_t* s_idx, const double* s_w, const double* vx, int64_t n_all) {
  double acc = 0.0;
  for (int64_t s = 0; s < ns; ++s) {
    double v = 0.0;
    for (int j = 0; j < nl; ++j) v += s_w[s * nl + j] * vx[s_idx[s * nl + j]];
    acc += v;
  }
  return acc / (double)n_all;
}

/* Hydrodynamic force on the grain, Eqs. stress_tensor_force and
 * integration_force.  For boundary node b: velocity gradient from its
 * derivative weights wg[(b*3 + a)*nl + j] (a = x, y, z) over stencil
 * sb[b*nl + j]; pressure relative to the node mean of p over all n nodes;
 * sigma = -p' I + rho nu (grad v + grad v^T); F = dA * sum_b sigma n_b. */
/* Traction t = sigma n at every boundary node (Eq. stress_tensor_force), the
 * surface map of Sec. 3.1: t_b = -(p_b - <p>) n_b + rho nu (grad v + grad v^T) n_b,
 * written t [nb][3]; the centred pressure p_b - <p> goes to pc [nb] (if not
 * NULL).  <p> is the mean of p over all n nodes. */
void mpfo_traction(int64_t nb, int nl, const int32_t* sb, const double* wg, const double* nrm, int64_t n,
                   const double* v, const double* p, double rho, double nu, double* t, double* pc) {
  double pm = 0.0;
  for (int64_t i = 0; i < n; ++i) pm += p[i];
  pm /= (double)n;
  for (int64_t b = 0; b < nb; ++b) {
    const int32_t* S = sb + b * nl;
    double G[3][3]; /* G[i][j] = d v_i / d x_j */
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double* wj = wg + (b * 3 + j) * nl;
        double s = 0.0;
        for (int q = 0; q < nl; ++q) s += wj[q] * v[3 * (int64_t)S[q] + i];
        G[i][j] = s;
      }
    double pp = p[S[0]] - pm;
    const double* nv = nrm + 3 * b;
    for (int i = 0; i < 3; ++i) {
      double ti = -pp * nv[i];
      for (int j = 0; j < 3; ++j) ti += rho * nu * (G[i][j] + G[j][i]) * nv[j];
      t[3 * b + i] = ti;
    }
    if (pc) pc[b] = pp;
  }
}

/* Hydrodynamic force, Eq. integration_force: F = dA sum_b t_b. */
void mpfo_drag(int64_t nb, int nl, const int32_t* sb, const double* wg, const double* nrm, int64_t n,
               const double* v, const double* p, double rho, double nu, double dA, double* F) {
  double* t = (double*)malloc(sizeof(double) * 3 * (nb > 0 ? nb : 1));
  mpfo_traction(nb, nl, sb, wg, nrm, n, v, p, rho, nu, t, NULL);
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t b = 0; b < nb; ++b)
    for (int i = 0; i < 3; ++i) acc[i] += t[3 * b + i];
  for (int i = 0; i < 3; ++i) F[i] = dA * acc[i];
  free(t);
}

/* ------------------------------------------------------------------ stop control */

/* Residual monitors of the stop control (the quantities a run reads at its
 * checks besides k, Eq. stopCrit): over the interior nodes i < n_int,
 *   out[0] = max_i |v_i - vprev_i| (0 when vprev is NULL),
 *   out[1] = max_i |v_i|,
 *   out[2] = sqrt(mean_i (div v)_i^2), (div v)_i = sum_j w^x_ij v_x(S_ij)
 *            + w^y_ij v_y(S_ij) + w^z_ij v_z(S_ij)  (the divergence of Eq.
 *            MNS_pressure).
 * w [n][n_ops >= 3][nl] with d/dx, d/dy, d/dz first; v, vprev [n][3]. */
void mpfo_residual(int64_t n_int, int nl, const int32_t* sten, const double* w, int n_ops, const double* v,
                   const double* vprev, double* out) {
  double dmax = 0.0, vmax = 0.0, s2 = 0.0;
  for (int64_t i = 0; i < n_int; ++i) {
    const double* vi = v + 3 * i;
    double m = sqrt(vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]);
    if (m > vmax) vmax = m;
    if (vprev) {
      const double* pi = vprev + 3 * i;
      double e0 = vi[0] - pi[0], e1 = vi[1] - pi[1], e2 = vi[2] - pi[2];
      double d = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
      if (d > dmax) dmax = d;
    }
    double div = 0.0;
    for (int j = 0; j < nl; ++j) {
      const double* u = v + 3 * (int64_t)sten[i * nl + j];
      for (int a = 0; a < 3; ++a) div += w[(i * n_ops + a) * nl + j] * u[a];
    }
    s2 += div * div;
  }
  out[0] = dmax;
  out[1] = vmax;
  out[2] = n_int > 0 ? sqrt(s2 / (double)n_int) : 0.0;
}

/* ------------------------------------------------------------------ cross-validation */

/* Pointwise relative difference of two velocity fields on the same nodes,
 * Eq. pointwise_error of Sec. 3.6: delta_i = |v_a,i - v_b,i| / |v_b,i| with
 * the Euclidean norm (a = MLBM, b = MNS in the paper), and dv_i = |v_a,i -
 * v_b,i|.  Where |v_b,i| = 0 the quotient is +inf if dv_i > 0 and 0 if the two
 * velocities are both zero (the no-slip grain).  v_a, v_b [n][3]; delta, dv
 * [n]. */
void mpfo_pointwise(int64_t n, const double* va, const double* vb, double* delta, double* dv) {
  for (int64_t i = 0; i < n; ++i) {
    double d0 = va[3 * i] - vb[3 * i], d1 = va[3 * i + 1] - vb[3 * i + 1], d2 = va[3 * i + 2] - vb[3 * i + 2];
    double num = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    double den = sqrt(vb[3 * i] * vb[3 * i] + vb[3 * i + 1] * vb[3 * i + 1] + vb[3 * i + 2] * vb[3 * i + 2]);
    dv[i] = num;
    delta[i] = den > 0.0 ? num / den : (num > 0.0 ? INFINITY : 0.0);
  }
}
