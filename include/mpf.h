/*
 * mpf.h -- C ABI of libmpf, the MI355X (gfx950) library for the hot path of the
 * meshless pore-flow solvers of Strzelczyk, Rot, Kosec and Matyka,
 * "Cross-validation of meshless Navier-Stokes solvers in porous media flows"
 * (arXiv 2404.14195).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Arrays named "dev" are device pointers (memory of the current HIP device);
 *   arrays named "host" are host pointers.  The caller owns all memory: the
 *   library never allocates or frees caller buffers.  Scratch memory is passed
 *   in as a caller-owned workspace whose size the matching *_workspace call
 *   reports.
 * - Every call is asynchronous on the caller's stream (a hipStream_t passed as
 *   void*; NULL is the default stream).  Scalar results are written to device
 *   memory.  Host-side argument checks happen before any launch.
 * - Return value: MPF_OK (0) or a negative MPF_ERR_* code; mpf_strerror()
 *   names it.  No C++ exception crosses the ABI.
 * - Layouts are structure-of-arrays with the node index fastest:
 *     positions        pos[3][n]          double
 *     stencils         sten[nl][m]        int32, column 0 = the row's centre
 *     weights          w[n_ops][nl][m]    double or float
 *     velocity         v[3][n]            double or float (precision flag)
 *     populations      f[n][qp]           double or float, node-major records
 *                                         of qp = 20 (D3Q19) or 16 (D3Q15)
 *                                         values; entries k >= q are zero.
 *                                         Stored shifted by the lattice
 *                                         weight: f~_k = f_k - w_k
 * - Nodes [0, n_int) are interior; nodes [n_int, n) lie on the grain surface,
 *   with unit normals nrm[3][nb] (nb = n - n_int) pointing from the solid into
 *   the fluid.
 * - Velocity sets (both follow the pairing of the paper's D3Q15 table, Sec.
 *   2.2: k = 0 rest, odd k a listed vector, even k = the opposite of k - 1):
 *     D3Q15 odd k = 1..13: (1,0,0) (0,1,0) (0,0,1) (1,1,1) (1,1,-1) (1,-1,1)
 *                          (1,-1,-1); weights 2/9, 1/9, 1/72
 *     D3Q19 odd k = 1..17: (1,0,0) (0,1,0) (0,0,1) (1,1,0) (1,-1,0) (1,0,1)
 *                          (1,0,-1) (0,1,1) (0,1,-1); weights 1/3, 1/18, 1/36
 */
#ifndef MPF_H
#define MPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPF_OK 0
#define MPF_ERR_ARG (-1)         /* invalid argument (host check, nothing launched) */
#define MPF_ERR_HIP (-2)         /* a HIP runtime call failed */
#define MPF_ERR_UNSUPPORTED (-3) /* valid but not built: e.g. a stencil size without a kernel */
#define MPF_ERR_DIVERGED (-4)    /* a *_run given a flags word found it set at the end of the call */
#define MPF_ERR_WORKSPACE (-5)   /* workspace missing or too small */

/* Precision of stencil weights and state.
 *   MPF_F64        weights and state FP64
 *   MPF_F32        weights and state FP32 (reductions stay FP64)
 *   MPF_MIXED      weights FP32, state and all step arithmetic FP64.  An
 *                  explicit iteration whose slowest mode decays over tau steps
 *                  and whose state is rounded every step stops within about
 *                  tau ulp of its fixed point (the updates fall below half an
 *                  ulp), so an FP32 state stalls at ~1e-3 relative on the
 *                  cells here (tau ~ 2e4 steps).
 *   MPF_F32_KAHAN  weights and state FP32 plus an FP32 compensation term per
 *                  state value (caller-owned, argument comp): the state is
 *                  hi + lo with hi the FP32 rounding of the value, neighbours
 *                  gather hi only, and each node's update is formed in FP64
 *                  from its own hi + lo and split back, so updates below half
 *                  an ulp of hi accumulate in lo instead of being lost.  The
 *                  gathered bytes stay those of MPF_F32. */
#define MPF_F64 0
#define MPF_F32 1
#define MPF_MIXED 2
#define MPF_F32_KAHAN 3

/* Flags word (device uint32) that the *_run calls OR bits into when given
 * one; the caller clears it.  At the end of such a call the library waits for
 * the stream, reads the word and returns MPF_ERR_DIVERGED if any bit is set
 * (pass NULL to keep a call fully asynchronous, e.g. under graph capture).
 *   bit 0  a non-finite state value (NaN or inf) was produced
 *   bit 1  a stability limit was exceeded: for the ACM the Courant number
 *          of the pressure waves, C dt / h_min > 1 (only when the params give
 *          h_min > 0); for the MLBM a lattice speed |u| >= c_s = 1/sqrt(3),
 *          where the second-order equilibrium of Eq. feq loses its meaning */
#define MPF_FLAG_NONFINITE 1u
#define MPF_FLAG_LIMIT 2u

/* Library context: the HIP device it was created for and the weight solve's
 * autotune cache (tile shape per stencil size, operator count and solve).
 * Field memory is never owned by it.  One context per host thread, or calls
 * on it externally synchronised.  mpf_create makes `hip_device` current on
 * the calling thread. */
typedef struct mpf_ctx mpf_ctx;
int mpf_create(mpf_ctx** out, int hip_device);
int mpf_destroy(mpf_ctx* ctx);

/* Static description of an error code; never NULL. */
const char* mpf_strerror(int code);

/* Library version, major*10000 + minor*100 + patch. */
int mpf_version(void);

/* ------------------------------------------------------------- geometry
 * Porosity and grain-surface area of the periodic simple-cubic cell of side
 * 1 holding one sphere of radius r at its centre (Sec. 2.4; A enters
 * Delta A = A / N_b of Eq. integration_force).  For r > 1/2 the six caps that
 * leave the cell are removed.  Host-only; valid for 0 <= r < sqrt(2)/2,
 * otherwise MPF_ERR_ARG. */
int mpf_sc_cell(double r, double* porosity_host, double* area_host);

/* ------------------------------------------------------------- stencils
 * The stencil of a node is its N_L nearest nodes (Sec. 2.1), here in the unit
 * periodic cell.  Order: squared minimum-image distance in FP64, formed
 * operation by operation (t = p_a - q_a reduced by t - rint(t), then
 * x^2 + y^2, + z^2, each rounded), ties by point index; nearest first.
 * Points must be distinct.
 *
 * mpf_knn: the k nearest of n_pts points to each of n_qry queries.
 *   pts    dev [3][ld_pts] double (coordinate a of point i at a * ld_pts + i)
 *   qry    dev [3][ld_qry] double
 *   idx    dev [k][ld_idx] int32 out (column c of query j at c * ld_idx + j)
 *   ws     dev workspace of mpf_knn_workspace(n_pts) bytes (the cell grid)
 *   1 <= k <= 64, k <= n_pts <= 2^31 - 1; MPF_ERR_ARG otherwise.
 * mpf_solver_stencils: the solvers' stencils [nl][n] of n nodes, interior
 *   first.  Interior nodes: their nl nearest nodes (the node itself first).
 *   Surface nodes [n_int, n): the node itself, then its nl - 1 nearest
 *   interior nodes (a surface node's nearest nodes are mostly other surface
 *   nodes, whose coordinates satisfy x^2 + y^2 + z^2 = r^2 and make the
 *   quadratic block of the weight system nearly singular).
 *   pos dev [3][n] double; sten dev [nl][n] int32 out; ws of
 *   mpf_knn_workspace(n) bytes; 2 <= nl <= 64, n_int >= nl - 1 when n > n_int. */
size_t mpf_knn_workspace(int64_t n_pts);
int mpf_knn(const double* pts, int64_t n_pts, int64_t ld_pts, const double* qry, int64_t n_qry, int64_t ld_qry,
            int k, int32_t* idx, int64_t ld_idx, void* ws, size_t ws_bytes, void* stream);
int mpf_solver_stencils(const double* pos, int64_t n, int64_t n_int, int nl, int32_t* sten, void* ws,
                        size_t ws_bytes, void* stream);

/* ------------------------------------------------------------- RBF-FD weights
 * Weights w of Eq. operatorApprox for m stencil rows, from the augmented
 * polyharmonic system of Eq. augmentedSystem: PHS r^3 plus the ten monomials
 * 1, x, y, z, x^2, xy, xz, y^2, yz, z^2, all in coordinates centred on the
 * row's centre c = sten[0][i] and scaled by delta_i = |x_{sten[1][i]} - x_c|
 * (Eq. rbfScaling; with nearest-first stencils the nearest-neighbour
 * distance).  Each system (size nl + 10) is solved in FP64 by Gaussian
 * elimination with partial pivoting; the Lagrange part is discarded.
 *
 * Operators (mpf_op.kind):                          right-hand side for
 *   MPF_OP_DX, _DY, _DZ   d/dx_a                    b_j = L |x - x_j|^3 at c,
 *   MPF_OP_LAP            Laplacian                 c_l = L p_l at c
 *   MPF_OP_DIR            vec . grad
 *   MPF_OP_SHIFT          value at c + vec          (L = 1 at a shifted point)
 *   MPF_OP_DN             rowvec_i . grad           (rowvec: dev [3][m])
 *   MPF_OP_SHIFT_ROW      value at c + rowvec_i
 *   MPF_OP_TAYLOR         value at c plus vec . grad: the first-order estimate
 *                         of the value at c + vec (the e . grad form of
 *                         streaming, Sec. 2.2, with vec = -dx e_k)
 *
 * pos      dev [3][n_nodes] double, in the unit periodic cell (displacements
 *          use the minimum image)
 * sten     dev [nl][m] int32, entries in [0, n_nodes) (not checked on device)
 * ops      host [n_ops], 1 <= n_ops <= 32
 * rowvec   dev [3][m] double, required iff an op is MPF_OP_DN/_SHIFT_ROW
 * w64      dev [n_ops][nl][m] double, or NULL
 * w32      dev [n_ops][nl][m] float, or NULL: the FP32 copy; its self weight
 *          (column 0) is replaced so that the row sums, computed in FP64, equal
 *          the exact ones (1 for the two shift kinds and the Taylor row,
 *          0 for derivatives)
 * info     dev [m] int32: 0; 1 + the column of a zero pivot (weights of that
 *          row are then NaN); -1 if FP32 refinement did not settle and the
 *          row was re-solved in FP64 (batched call with MPF_SOLVE_FP32_IR)
 * ws       workspace of mpf_weights_workspace() bytes (holds the row table)
 * nl must be one of 20, 25, 27, 30, 35, 40, 45, 50 (MPF_ERR_UNSUPPORTED
 * otherwise).  At least one of w64 / w32 must be given. */
#define MPF_OP_DX 0
#define MPF_OP_DY 1
#define MPF_OP_DZ 2
#define MPF_OP_LAP 3
#define MPF_OP_DIR 4
#define MPF_OP_SHIFT 5
#define MPF_OP_DN 6
#define MPF_OP_SHIFT_ROW 7
#define MPF_OP_TAYLOR 8

typedef struct {
  int32_t kind;
  int32_t reserved;
  double vec[3];
} mpf_op;

size_t mpf_weights_workspace(void);
int mpf_rbffd_weights(const double* pos, int64_t n_nodes, const int32_t* sten, int64_t m, int nl, int n_ops,
                      const mpf_op* ops, const double* rowvec, double* w64, float* w32, int32_t* info, void* ws,
                      size_t ws_bytes, void* stream);

/* Batched weights: every row of up to 16 node clouds (same nl and operators)
 * in one launch over their concatenated rows; each wave solves rows_per_wave
 * consecutive rows, so clouds of very different sizes share the chip.  Each
 * cloud is described by an mpf_wgeom with the same
 * meaning as the arguments of mpf_rbffd_weights (rowvec per cloud when an
 * operator needs it).
 * solve: MPF_SOLVE_FP64 (direct), or MPF_SOLVE_FP32_IR: FP32 factors with
 *        FP64-residual iterative refinement (at most five sweeps; stop at
 *        |dx| <= 1e-15 |x|, or once |dx| <= 1e-9 |x| no longer shrinks 4x per
 *        sweep, the FP64-residual floor; otherwise the row is re-solved in
 *        FP64, info -1).
 * ctx:   the context whose autotune cache supplies the tile shape when
 *        tune is NULL; may be NULL (then the default shape).
 * tune:  host pointer to the tile shape, or NULL for the shape that
 *        mpf_weights_autotune last stored in ctx for (nl, n_ops, solve), or a
 *        default (4 waves per block, 1 row per wave).
 * The geometry table is copied into ws on the stream, and the call waits for
 * that copy (one stream synchronisation) before it launches the solve. */
#define MPF_SOLVE_FP64 0
#define MPF_SOLVE_FP32_IR 1

typedef struct {
  const double* pos; /* dev [3][n_nodes] */
  int64_t n_nodes;
  const int32_t* sten; /* dev [nl][m] */
  int64_t m;
  const double* rowvec; /* dev [3][m] or NULL */
  double* w64;          /* dev [n_ops][nl][m] or NULL */
  float* w32;           /* dev [n_ops][nl][m] or NULL */
  int32_t* info;        /* dev [m] */
} mpf_wgeom;

typedef struct {
  int32_t waves_per_block; /* 1..8 */
  int32_t rows_per_wave;   /* 1..64 */
} mpf_wtune;

int mpf_rbffd_weights_batched(mpf_ctx* ctx, int n_geoms, const mpf_wgeom* geoms_host, int nl, int n_ops,
                              const mpf_op* ops, int solve, const mpf_wtune* tune, void* ws, size_t ws_bytes,
                              void* stream);

/* Autotuner: times every candidate tile shape (waves per block 1, 2, 4, 8 x
 * rows per wave 1, 2, 4, 8) on the first sample_rows rows of *sample (whose
 * outputs it overwrites), on a private stream of the context's device,
 * synchronously; stores the fastest in *out and in ctx's cache, which
 * mpf_rbffd_weights_batched reads when it gets tune = NULL.  ctx must not be
 * NULL. */
int mpf_weights_autotune(mpf_ctx* ctx, int nl, int n_ops, const mpf_op* ops, int solve, const mpf_wgeom* sample,
                         int64_t sample_rows, mpf_wtune* out, void* ws, size_t ws_bytes);

/* Tile plan of the LDS-staged stencil gather.  The MLBM step works on tiles
 * of 64 consecutive nodes, the ACM passes on tiles of 64, 128 or 256; a
 * tile's stencils (Sec. 2.1) name few distinct nodes (about 350 for 64 x 30
 * entries on the refined clouds here, 940 for 256 x 30).  The plan lists
 * each tile's distinct stencil nodes in ascending order (its halo) and every
 * stencil entry as its 16-bit position in that list, so a step copies the
 * halo's records into LDS with contiguous loads and gathers from LDS.  Built
 * once per stencil set and tile size:
 *   count dev int32 [G + 1], G = mpf_tile_count_sized(n, tile): halo sizes,
 *         and in count[G] the largest (also returned in *h_max_host)
 *   halo  dev int32 [G][h_cap]: the halo of tile t in halo[t][0, count[t])
 *   lidx  dev uint16 [nl][n]: sten[j][i] == halo[i / tile][lidx[j][i]]
 * sten dev [nl][n]; 1 <= nl <= 64; tile 64, 128 or 256;
 * 64 <= h_cap <= 64 tile.  The call waits for the stream (it reads back the
 * largest halo) and returns MPF_ERR_UNSUPPORTED if a tile's halo exceeds
 * h_cap (the plan is then incomplete and must not be used).
 * mpf_tile_plan and mpf_tile_count are the same with tile = 64. */
typedef struct {
  const int32_t* count;
  const int32_t* halo;
  const uint16_t* lidx;
  int32_t h_cap; /* row length of halo */
  int32_t h_max; /* the largest halo, as mpf_tile_plan returned it */
  int32_t tile;  /* nodes per tile (0 is read as 64) */
} mpf_tiles;
int64_t mpf_tile_count(int64_t n);
int64_t mpf_tile_count_sized(int64_t n, int tile);
int mpf_tile_plan(int64_t n, int nl, const int32_t* sten, int h_cap, int32_t* count, int32_t* halo, uint16_t* lidx,
                  int32_t* h_max_host, void* stream);
int mpf_tile_plan_sized(int64_t n, int nl, const int32_t* sten, int tile, int h_cap, int32_t* count, int32_t* halo,
                        uint16_t* lidx, int32_t* h_max_host, void* stream);

/* ------------------------------------------------------------- ACM step
 * Explicit artificial-compressibility Navier-Stokes steps (Sec. 2.3, Eqs.
 * MNS_intermediate, MNS_pressure, MNS_velocity, MNS_C; MNS algorithm of
 * Appendix A).  One step:
 *   v'_i = v_i + dt (nu Lap v_i - (v_i . grad) v_i + g)   interior i; v' = 0 on
 *                                                          the boundary
 *   n_p times:
 *     p_i -= dt C^2 rho (div v)_i                         interior (v = v' at
 *                                                          the first iteration)
 *     p_b  = -(sum_{j>=1} wn_bj p_{sn_b(j)}) / wn_b0      boundary, dp/dn = 0
 *     v_i  = v'_i - (dt / rho) (grad p)_i                 interior
 *     C    = beta max(max_i |v_i|, v_ref)
 * The Neumann stencil sn of boundary node b must hold b itself in column 0
 * and only interior nodes after it (then the boundary update reads no other
 * boundary value and runs in place).
 *
 * w     dev [4][nl][n]: d/dx, d/dy, d/dz, Laplacian weights of every node
 *       (rows of boundary nodes are not read)
 * sten  dev [nl][n]
 * sn    dev [nl][nb]; wn dev [nl][nb] normal-derivative weights on sn
 * tiles the tile plan of sten (mpf_tile_plan_sized) or NULL: with one or
 *       two lanes per node the interior passes then copy each tile's halo
 *       values into LDS and gather from there, when a block of 256 lanes
 *       holds whole tiles (tile x lanes <= 256) and its halos fit 64 KiB
 *       (64-node tiles: h_max <= 819 for FP32 at one lane and for an FP64
 *       state at two, 1638 for FP32 at two, 409 for an FP64 state at one;
 *       one 256-node tile at one lane or one 128-node tile at two: 3276 FP32,
 *       1638 FP64); otherwise, and for NULL, they gather through the caches.
 *       Results are the same bit for bit either way.
 * v     dev [3][n], p dev [n]: state, updated in place (v stays 0 on the
 *       boundary)
 * comp  dev float [4][n] for MPF_F32_KAHAN (NULL otherwise): the
 *       compensation terms of v (rows 0-2) and p (row 3), in/out; zero for a
 *       state given exactly in FP32 (e.g. rest).  The true state is v + comp,
 *       p + comp[3]; boundary entries stay zero.
 * vmax  dev double [1]: max_i |v_i| of the current state, in/out (0 for a
 *       state at rest); C is derived from it.  A non-finite |v_i| counts as
 *       +inf.
 * flags dev uint32 [1] or NULL: bit 0 when a velocity is not finite, bit 1
 *       when h_min > 0 and C dt / h_min > 1 at a pressure pass (see the
 *       flags word above; MPF_ERR_DIVERGED when set at the end of the call)
 * ws    workspace of mpf_acm_workspace() bytes (velocity and v' records
 *       [n][4], a second pressure [n], and for MPF_F32_KAHAN the
 *       compensation of v' [n][4])
 * precision: MPF_F64, MPF_F32 (weights and fields FP32, all arithmetic
 * except the max FP32), MPF_MIXED (weights w, wn FP32; fields v, p and the
 * workspace FP64; FP64 arithmetic) or MPF_F32_KAHAN (as MPF_F32, and each
 * interior node's v and p updates are added to hi + lo with an error-free
 * two-sum, so increments below half an ulp of the FP32 value are kept).
 * lanes: how many adjacent lanes share one node's stencil sum (1, 2, 4, 8 or
 * 16; 0 lets the library pick from n_int and the state's precision: 8 up to
 * 12000 interior nodes, 2 up to 50000, then 1, and 2 again above 500000 for
 * an FP64 state; 2 in place of 1 when a tile plan is given whose halos fit
 * LDS at two lanes but not at one).  Results agree to rounding (the order of
 * the partial sums differs).
 * edac: 0 for the method as written; 1 for the entropically damped pressure
 * equation, which Sec. 2.3 names as the remedy for the stagnant-region
 * pressure oscillations of Sec. 3.6.  Its pressure update is
 *     p_i += dt (-C^2 rho (div v)_i - v_i . (grad p)_i + nu (lap p)_i)
 * with the iteration's velocity (v' at the first) and every pressure term
 * from before the update; the other passes are unchanged.
 * On cells of at most 50,000 nodes a run of 32 or more steps enqueues its
 * steps as replays of a captured HIP graph of 16 steps (the same kernels in
 * the same order, so the same results bit for bit) and waits for the stream
 * before it returns. */
typedef struct {
  double nu, rho, dt, beta, v_ref;
  double g[3];
  int32_t n_p;
  int32_t precision;
  int32_t lanes;
  int32_t edac;
  double h_min; /* smallest node spacing, for the Courant check of flags bit 1; 0 = no check */
} mpf_acm_params;

/* The ACM time step of Sec. 2.3, dt = 0.1 h_min^2 / (2 nu).  Host-only. */
int mpf_acm_dt(double h_min, double nu, double* dt_host);
size_t mpf_acm_workspace(int64_t n, int precision);
int mpf_acm_run(const mpf_acm_params* prm, int64_t n, int64_t n_int, int nl, const int32_t* sten, const void* w,
                const int32_t* sn, const void* wn, const mpf_tiles* tiles, void* v, void* p, void* comp,
                double* vmax, uint32_t* flags, int n_steps, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------- MLBM step
 * Meshless lattice Boltzmann steps with TRT collision (Sec. 2.2, Eqs.
 * LBM_streaming, LBM_collision, feq, macro_var, force_lbm,
 * interpolated_bounceback_mlbm; MLBM algorithm of Appendix A).  The state f
 * holds the populations at step boundaries (after streaming and bounce-back),
 * shifted: f~_k = f_k - w_k.  One step:
 *   collide on every node: rho = 1 + sum f~, u = sum f~ e / rho, f^eq of Eq.
 *     feq, F_k = 3 w_k e_k . (rho g_lb), TRT relaxation with tau+ and tau-;
 *   stream: f_k(i) = sum_j W_k[j][i] f^post_k(sten[j][i]) for k >= 1 (W_k
 *     interpolates at the departure point of population k), f_0 = f^post_0;
 *   bounce-back at boundary node b (Eq. interpolated_bounceback_mlbm): where
 *     bit k of unknown[b] is set, f_k = f_{opp(k)}.
 * W       dev [q-1][nl][n] (population k uses slice k - 1): double for
 *         MPF_F64, float for MPF_F32, MPF_MIXED and MPF_F32_KAHAN
 * unknown dev [nb] uint32 bit masks from mpf_lbm_unknown (nb = n - n_int;
 *         may be NULL when nb = 0)
 * f     dev [n][qp] state, updated in place; f_tmp dev [n][qp] scratch:
 *       double for MPF_F64 and MPF_MIXED, float for MPF_F32 and
 *       MPF_F32_KAHAN
 * comp  dev float [n][qp] for MPF_F32_KAHAN (NULL otherwise), in/out: the
 *       compensation of f, so that the state is f + comp (zero for a state
 *       given exactly in FP32).  In that mode the stencil sums gather the FP32
 *       records f only, the node's own comp enters its rest population and
 *       its self column in FP64, and the collision and the split back into
 *       f and comp run in FP64.
 * flags dev uint32 [1] or NULL: bit 0 when a collided node has a non-finite
 *       density or velocity, bit 1 when |u|^2 >= 1/3 there (see the flags
 *       word above; MPF_ERR_DIVERGED when set at the end of the call)
 * tiles host pointer to the tile plan of sten with 64-node tiles
 *       (mpf_tile_plan), or NULL: the step then stages each tile's halo
 *       records in LDS and gathers from there when the largest halo's
 *       records fit 64 KiB (80 KiB for MPF_F64), and reads the neighbours'
 *       records through the caches otherwise (and without a plan).  Results
 *       are the same bit for bit either way.  A plan of another tile size is
 *       MPF_ERR_ARG.
 * q is 15 or 19.  A W larger than 512 MiB (twice the Infinity Cache) is read
 * with non-temporal loads so that it does not evict the gathered population
 * records; the results are the same bit for bit either way. */
typedef struct {
  int32_t q;
  int32_t precision;
  double tau_plus, tau_minus;
  double g_lb[3];
} mpf_lbm_params;

/* f~ = f^eq(rho, u) - w_k on every node. */
int mpf_lbm_init(const mpf_lbm_params* prm, int64_t n, double rho, const double* u_host, void* f, void* stream);
/* f~ = f^eq(rho_i, u_i) - w_k from fields in physical units, the inverse of
 * mpf_lbm_moments: u_i = v_i / vel_scale, rho_i = 1 + 3 p_i / vel_scale^2.
 * v dev [3][n] double, p dev [n] double (any gauge: only differences of p
 * drive the flow).  Starts a run from a predicted field (warm start). */
int mpf_lbm_init_fields(const mpf_lbm_params* prm, int64_t n, const double* v, const double* p, double vel_scale,
                        void* f, void* stream);
int mpf_lbm_run(const mpf_lbm_params* prm, int64_t n, int64_t n_int, int nl, const int32_t* sten, const void* W,
                const uint32_t* unknown, const mpf_tiles* tiles, void* f, void* f_tmp, void* comp, uint32_t* flags,
                int n_steps, void* stream);
/* Lattice units of Sec. 2.2 (Eqs. lbm_viscosity and conversion_factors) for
 * a cloud of smallest spacing h_min: dx = h_min / 2, nu_lb = (tau+ - 1/2) / 3,
 * dt = nu_lb dx^2 / nu, g_lb = g dt^2 / dx, vel_scale = dx / dt (physical
 * velocity per lattice velocity) and tau- = 1/2 + Lambda / (tau+ - 1/2) from
 * the magic parameter Lambda.  g_host [3]; host-only; MPF_ERR_ARG unless
 * h_min > 0, nu > 0, tau+ > 1/2 and Lambda > 0. */
typedef struct {
  double dx, dt, nu_lb, tau_minus, vel_scale;
  double g_lb[3];
} mpf_lbm_units;
int mpf_lbm_units_of(double h_min, double nu, double tau_plus, double magic, const double* g_host,
                     mpf_lbm_units* out_host);
/* Which populations of each boundary node n_int + b are unknown after
 * streaming, as bit masks unknown[b] (bit k for population k, bit 0 never set):
 *   MPF_UNKNOWN_NORMAL (Sec. 2.2): e_k . n_b > 0, with nrm dev [3][nb] double
 *     pointing from the solid into the fluid; pos, dx and r are not read.
 *   MPF_UNKNOWN_SOLID (Sec. 3.3, the rule of the touching limit): the
 *     departure point x_b - dx e_k lies inside the solid, the union of the
 *     balls of radius r > 0 centred at (1/2, 1/2, 1/2) + Z^3 (the simple-cubic
 *     cell, grains may overlap).  pos dev [3][n] double in the unit cell,
 *     0 < dx < 1/2; nrm is not read.
 * Written once per geometry; MPF_ERR_ARG for a bad rule, q or argument. */
#define MPF_UNKNOWN_NORMAL 0
#define MPF_UNKNOWN_SOLID 1
int mpf_lbm_unknown(int q, int64_t n, int64_t n_int, const double* pos, const double* nrm, int rule, double dx,
                    double r, uint32_t* unknown, void* stream);
/* Macroscopic fields in physical units (Eq. conversion_factors): v[3][n] =
 * vel_scale * u_lb, p[n] = vel_scale^2 (rho - 1) / 3 (not centred: the drag
 * reduction subtracts the node mean).  Outputs are double.  comp: the FP32
 * remainders of an MPF_F32_KAHAN state (added to f in FP64), or NULL; given
 * for another precision, MPF_ERR_ARG. */
int mpf_lbm_moments(const mpf_lbm_params* prm, int64_t n, const void* f, const void* comp, double vel_scale, double* v,
                    double* p, void* stream);

/* ------------------------------------------------------------- reductions
 * Mean x-velocity over the five cross-sections, Eq. k_definition, as the mean
 * over all n_all = 5 M^2 midpoint samples, solid samples counting zero.  The
 * ns fluid samples interpolate v_x with weights s_w over stencils s_idx.
 * s_idx dev [nl][ns]; s_w dev [nl][ns] double; vx dev [n] (float for MPF_F32,
 * double for MPF_F64 and MPF_MIXED: the type of the state);
 * q_out dev double[1].  The sum is a fixed-order FP64 tree, so results are
 * bitwise reproducible. */
size_t mpf_reduce_workspace(int64_t n_items);
/* x[i] *= c for i < n; x dev, double (MPF_F64) or float (MPF_F32 and
 * MPF_F32_KAHAN; a compensated field scales its comp with a second call).
 * Used to rescale a velocity field to a target flux (the warm start's flux
 * match). */
int mpf_scale(int64_t n, void* x, int precision, double c, void* stream);
int mpf_flux_planes(int64_t ns, int nl, const int32_t* s_idx, const double* s_w, const void* vx, int precision,
                    int64_t n_all, double* q_out, void* ws, size_t ws_bytes, void* stream);
/* The same reduction without a workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation): the block partials live in a static device array
 * of the library, 64 KiB per GPU, held until the process ends, so this call
 * allocates nothing.  ns may be at most mpf_flux_planes_noalloc_max() (2^21
 * samples), otherwise MPF_ERR_WORKSPACE.  Every call on one GPU shares that
 * array: calls that overlap on one GPU (two streams, two threads) race and
 * must be serialised by the caller.  Nothing in it needs clearing between
 * calls (every partial is written before it is read).  Arguments and result
 * as for mpf_flux_planes. */
int64_t mpf_flux_planes_noalloc_max(void);
int mpf_flux_planes_noalloc(int64_t ns, int nl, const int32_t* s_idx, const double* s_w, const void* vx,
                            int precision, int64_t n_all, double* q_out, void* stream);
/* Permeability from the plane flux, Eq. k_definition: k / d^2 = q nu / (|g| d^2).
 * K from the drag, Eq. K_definition: K = F_x / (6 pi r phi q mu).  g_host
 * [3]; host-only; MPF_ERR_ARG for a zero force, d, r, phi, q or mu. */
int mpf_permeability(double q, double nu, const double* g_host, double d, double* k_host);
int mpf_drag_coefficient(double Fx, double r, double phi, double q, double mu, double* K_host);

/* Pointwise relative difference of the two solvers' velocity fields on the
 * same nodes, Eq. pointwise_error of Sec. 3.6 (the cross-validation):
 *   delta[i] = |va_i - vb_i| / |vb_i|,  dv[i] = |va_i - vb_i|   (i < n)
 * with Euclidean norms in FP64 (va = MLBM, vb = MNS in the paper); where
 * |vb_i| = 0, delta is +inf if dv > 0 and 0 if both velocities are zero.
 * va, vb dev [3][n] of the state types of prec_a / prec_b (float for MPF_F32
 * and MPF_F32_KAHAN, else double); delta, dv dev double [n] or NULL.
 * Isocontour statistics: counts[l] = number of nodes i < n_count with
 * delta[i] > levels_host[l], for l < n_levels <= 16 (counts dev int64
 * [n_levels], overwritten; exact integer sums).  n_levels = 0 for none. */
int mpf_pointwise(int64_t n, const void* va, int prec_a, const void* vb, int prec_b, double* delta, double* dv,
                  int64_t n_count, int n_levels, const double* levels_host, int64_t* counts, void* stream);

/* Residual monitors of the stop control (every check; not in the step):
 *   out[0] = max_i |v_i - v_prev_i|   over interior nodes (0 if v_prev NULL)
 *   out[1] = max_i |v_i|              over interior nodes
 *   out[2] = sqrt(mean_i (div v)_i^2) over interior nodes, with
 *            (div v)_i = sum_j (wx_ij v_x + wy_ij v_y + wz_ij v_z)(sten_ij)
 * w dev [>= 3][nl][n] (d/dx, d/dy, d/dz first, as mpf_acm_run takes them):
 * double for MPF_F64, float otherwise; v, v_prev dev [3][n]: the state type
 * of precision (float for MPF_F32 and MPF_F32_KAHAN, else double).  A NaN
 * makes the maxima NaN.  out dev double [3]; ws: mpf_reduce_workspace(n)
 * bytes.  Fixed-order FP64 sums (bitwise reproducible). */
int mpf_residual(int64_t n, int64_t n_int, int nl, const int32_t* sten, const void* w, const void* v,
                 const void* v_prev, int precision, double* out, void* ws, size_t ws_bytes, void* stream);

/* Hydrodynamic force on the grains, Eqs. stress_tensor_force and
 * integration_force: F = dA sum_b (-(p_b - <p>) n_b + rho nu (grad v + grad
 * v^T) n_b), with <p> the mean of p over all n nodes and grad v at boundary
 * node b from derivative weights wg dev [3][nl][nb] over stencils sb dev
 * [nl][nb].  v dev [3][n], p dev [n] (precision); nrm dev [3][nb]; F_out dev
 * double[3].  Fixed-order FP64 sums.  Workspace: mpf_reduce_workspace(max(n,
 * nb)) bytes. */
int mpf_drag(int64_t n, const void* v, const void* p, int precision, int64_t nb, int nl, const int32_t* sb,
             const double* wg, const double* nrm, double rho, double nu, double dA, double* F_out, void* ws,
             size_t ws_bytes, void* stream);
/* The surface maps of Sec. 3.1: the traction t_b = sigma n_b of the force
 * above at every boundary node, t_out dev [3][nb] double, and the centred
 * pressure p_b - <p>, pc_out dev [nb] double (the tangential force is
 * t - (t . n) n).  Same arguments and workspace as mpf_drag. */
int mpf_traction(int64_t n, const void* v, const void* p, int precision, int64_t nb, int nl, const int32_t* sb,
                 const double* wg, const double* nrm, double rho, double nu, double* t_out, double* pc_out, void* ws,
                 size_t ws_bytes, void* stream);

/* ------------------------------------------------------------- learned warm start
 * An addition to the paper's method: a multilayer perceptron maps per-node
 * features of a cell to a predicted steady state (velocity and pressure),
 * which starts the explicit iteration of either solver instead of rest.  It
 * is trained on the solvers' own steady fields; the cold-started solver stays
 * the reference for its error.
 *
 * Shape (the only one built): in_dim 5, width 128, depth 4 linear layers,
 * out_dim 4, i.e. 5 -> 128 -> 128 -> 128 -> 4 with SiLU, z / (1 + e^-z),
 * after each hidden layer; any other desc gives MPF_ERR_UNSUPPORTED.
 * master   dev float [mpf_mlp_param_count()]: W_1, b_1, ..., W_4, b_4, with
 *          W_l [out][in] row-major (the FP32 master copy Adam updates)
 * packed   dev BF16 [mpf_mlp_packed_count()]: the weights as the products
 *          read them; refresh with mpf_mlp_pack after every update
 * x        dev float [rows][5]: features (mpf_mlp_features)
 * rows     dev int64 [B] or NULL: sample b of a batch is row rows[b] of x
 *          (and of t in mpf_mlp_mse); NULL means b itself
 * y        dev float [B][4]: outputs (v_x, v_y, v_z, p) / (U, P)
 * Products use BF16 operands with FP32 accumulation (MFMA); biases,
 * pre-activations and the derivative of SiLU are FP32.  All sums are in a
 * fixed order: repeated calls give identical bits.  Workspaces are device
 * memory of at least the stated size; they are not zeroed by the caller. */
typedef struct {
  int32_t in_dim, width, depth, out_dim;
} mpf_mlp_desc;

int64_t mpf_mlp_param_count(const mpf_mlp_desc* d);  /* 34308, or -1 */
int64_t mpf_mlp_packed_count(const mpf_mlp_desc* d); /* BF16 elements, or -1 */
/* Bytes for a batch of B samples; train != 0 adds what backward reads. 0 for
 * an unsupported desc or B outside [1, 2^26]. */
size_t mpf_mlp_workspace(const mpf_mlp_desc* d, int64_t B, int train);
int mpf_mlp_pack(const mpf_mlp_desc* d, const float* master, void* packed, void* stream);
/* y = net(x[rows]).  train != 0 keeps the activations in ws for
 * mpf_mlp_backward (ws sized with train = 1). */
int mpf_mlp_forward(const mpf_mlp_desc* d, const float* master, const void* packed, const float* x,
                    const int64_t* rows, float* y, int64_t B, int train, void* ws, size_t ws_bytes, void* stream);
/* grad (dev float, master layout) = d(sum dy . y)/d(params) for the batch of
 * the last mpf_mlp_forward with train = 1 on the same ws and B; dy dev float
 * [B][4].  grad is overwritten. */
int mpf_mlp_backward(const mpf_mlp_desc* d, const void* packed, const float* dy, float* grad, int64_t B, void* ws,
                     size_t ws_bytes, void* stream);
/* loss (dev double[1]) = mean over B x 4 entries of (y - t[rows])^2 (FP64
 * fixed-order sum); dy (dev float [B][4]) = 2 (y - t) / (4 B).  t dev float
 * [rows][4].  ws: mpf_reduce_workspace(4 B) bytes. */
int mpf_mlp_mse(int64_t B, const float* y, const float* t, const int64_t* rows, float* dy, double* loss, void* ws,
                size_t ws_bytes, void* stream);
/* One Adam step (t = step >= 1, bias-corrected): m = b1 m + (1 - b1) g,
 * v = b2 v + (1 - b2) g^2, p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 * p, g, m, v dev float [n]; m and v start at zero. */
int mpf_adam_step(int64_t n, float* p, const float* g, float* m, float* v, int step, float lr, float b1, float b2,
                  float eps, void* stream);
/* Features of the nodes of the simple-cubic cell with a grain of radius r at
 * (1/2, 1/2, 1/2) (Sec. 2.4): x[i] = (d_x, d_y, d_z, |d| - r, phi) with d the
 * minimum-image offset of pos_i from the grain centre.  pos dev [3][n]
 * double; x dev float [n][5]. */
int mpf_mlp_features(int64_t n, const double* pos, double r, double phi, float* x, void* stream);
/* Network outputs y dev float [n][4] -> solver state: v = U y_{0..2} on the
 * interior nodes [0, n_int) and 0 on the grain (no slip), p = P y_3 minus its
 * node mean (fixed-order FP64 mean).  v dev [3][n], p dev [n], of the state
 * type of precision (float for MPF_F32 and MPF_F32_KAHAN, whose comp the
 * caller zeroes, else double).  vmax dev double[1] or
 * NULL: receives max |v| (the input mpf_acm_run expects).  ws:
 * mpf_reduce_workspace(n) bytes. */
int mpf_mlp_to_state(int64_t n, int64_t n_int, const float* y, double U, double P, int precision, void* v, void* p,
                     double* vmax, void* ws, size_t ws_bytes, void* stream);
/* n_batches Adam steps on consecutive minibatches, all launched from one host
 * call: batch i uses rows[i B .. (i+1) B) of x and t, Adam step number
 * step0 + i + 1 and learning rate lr0 lr_ratio^i; each step is forward (train),
 * MSE, backward, Adam and pack, exactly as the separate calls do them.
 * loss_sum (dev double[1]) receives the sum of the n_batches losses.  m, v,
 * grad dev float [param_count]; rows dev int64 [n_batches B]; ws:
 * mpf_mlp_train_workspace(B) bytes. */
size_t mpf_mlp_train_workspace(const mpf_mlp_desc* d, int64_t B);
int mpf_mlp_train(const mpf_mlp_desc* d, float* master, void* packed, float* m, float* v, float* grad, const float* x,
                  const float* t, const int64_t* rows, int64_t n_batches, int64_t B, int step0, float lr0,
                  float lr_ratio, float b1, float b2, float eps, double* loss_sum, void* ws, size_t ws_bytes,
                  void* stream);
/* The same training step fused: one persistent kernel per step runs forward,
 * MSE, backward and the weight gradients of 64-row tiles with the
 * activations in LDS and the gradient sums in registers (one block of eight
 * waves per compute unit, at most 1024 blocks), then a fixed-order sum of the
 * blocks' partial gradients.  Same network, operand and accumulation precisions as
 * the separate calls; the derivative of SiLU is kept in FP16 between the
 * passes and the batch's rows are summed in another order, so results agree
 * with them to rounding, not bit for bit, and are bitwise reproducible for a
 * given device.
 * mpf_mlp_grad_fused: grad (dev float [param_count], overwritten) and loss
 *   (dev double [1] or NULL: the MSE) of one batch x[rows], t[rows] of B
 *   samples, without an optimiser step.
 * mpf_mlp_train_fused: as mpf_mlp_train (n_batches Adam steps, loss_sum the
 *   sum of their losses) with the fused step; the kernel that sums the
 *   partial gradients also applies the Adam step (the arithmetic of
 *   mpf_adam_step) and rewrites the packed BF16 copy (as mpf_mlp_pack), so a
 *   step is two launches.  grad holds the last step's gradient.
 * ws: mpf_mlp_fused_workspace(B) bytes (the blocks' partial gradients). */
size_t mpf_mlp_fused_workspace(const mpf_mlp_desc* d, int64_t B);
int mpf_mlp_grad_fused(const mpf_mlp_desc* d, const float* master, const void* packed, const float* x, const float* t,
                       const int64_t* rows, int64_t B, float* grad, double* loss, void* ws, size_t ws_bytes,
                       void* stream);
int mpf_mlp_train_fused(const mpf_mlp_desc* d, float* master, void* packed, float* m, float* v, float* grad,
                        const float* x, const float* t, const int64_t* rows, int64_t n_batches, int64_t B, int step0,
                        float lr0, float lr_ratio, float b1, float b2, float eps, double* loss_sum, void* ws,
                        size_t ws_bytes, void* stream);
/* rows[i] = pi(i) for i < count, pi a permutation of [0, n) fixed by seed
 * (a Feistel network with cycle walking, evaluated pointwise): the minibatch
 * order of an epoch without a host-side shuffle.  rows dev int64 [count];
 * count <= n. */
int mpf_shuffle_rows(int64_t n, int64_t count, uint64_t seed, int64_t* rows, void* stream);
/* The library's BF16 product on its own: C[m][n] = sum_k A[m][k] Bt[n][k]
 * with FP32 accumulation.  A dev BF16 [M][lda], Bt dev BF16 [N][ldb] (16-byte
 * aligned, lda and ldb multiples of 8), C dev float [M][ldc]; K a multiple of
 * 32, K <= lda, ldb; N <= ldc. */
int mpf_gemm_bf16(int64_t M, int N, int64_t K, const void* A, int64_t lda, const void* Bt, int64_t ldb, float* C,
                  int64_t ldc, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MPF_H */
