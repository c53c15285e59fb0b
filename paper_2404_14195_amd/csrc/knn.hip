// Periodic k nearest neighbours in the unit cell on gfx950: the stencils of
// Sec. 2.1 (each node's N_L nearest nodes, minimum image).
//
// The points are binned into a uniform grid of G^3 cells, G odd and chosen for
// about two points per cell: one pass writes each point's cell and counts the
// cells with atomics, a two-level scan turns the counts into cell starts, and
// a scatter pass copies the coordinates and indices cell by cell (the order
// inside a cell is whatever the atomics gave; the result does not depend on
// it).  Each query thread then visits the cells ring by ring around its own
// cell (Chebyshev rings; with G odd the rings up to (G - 1)/2 cover every cell
// exactly once), skipping a cell whose box is farther than the current k-th
// neighbour and stopping once every unvisited ring is.  The running k best
// sit in LDS as a list sorted by (squared distance, index), the total order
// that defines the stencil, so ties fall exactly as in a brute-force search.
#include "common.hpp"

namespace mpf {
namespace {

constexpr int kBlock = 256;
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kQueryBlock = 64;
constexpr int kMaxK = 64;
constexpr int kMaxSide = 255;
// slack subtracted from every box gap: far above the rounding of cell
// coordinates (about 1e-16), far below any node spacing
constexpr double kGapSlack = 1e-12;

int grid_side(int64_t n) {
  int G = (int)cbrt((double)n / 2.0);
  if (G > kMaxSide) G = kMaxSide;
  if (G % 2 == 0) G -= 1;
  return G < 1 ? 1 : G;
}

__device__ __forceinline__ double wrap01(double x) { return x - floor(x); }

__device__ __forceinline__ int cell_of(double w, int G) {
  int c = (int)(w * G);
  return c < 0 ? 0 : (c >= G ? G - 1 : c);
}

// Squared minimum-image distance, each operation rounded on its own: t = p - q,
// t - rint(t), then x^2 + y^2, + z^2.  hipcc fuses multiplies and adds by
// default; the pragma keeps these operations (written here, not in helper
// functions, so that it covers them) separate.
__device__ __forceinline__ double dist2(double px, double py, double pz, double qx, double qy, double qz) {
#pragma clang fp contract(off)
  double tx = px - qx, ty = py - qy, tz = pz - qz;
  tx = tx - rint(tx);
  ty = ty - rint(ty);
  tz = tz - rint(tz);
  double s = tx * tx;
  s = s + ty * ty;
  return s + tz * tz;
}

__global__ __launch_bounds__(kBlock) void bin_points(int64_t n, const double* __restrict__ pts, int64_t ld, int G,
                                                     int32_t* __restrict__ cell, int32_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int cx = cell_of(wrap01(pts[i]), G), cy = cell_of(wrap01(pts[ld + i]), G),
            cz = cell_of(wrap01(pts[2 * ld + i]), G);
  const int c = (cx * G + cy) * G + cz;
  cell[i] = c;
  atomicAdd(&count[c], 1);
}

__global__ __launch_bounds__(kBlock) void fill_i32(int64_t n, int32_t* __restrict__ x, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] = v;
}

// Exclusive scan of one tile of kScanTile counts; the tile total goes to sums.
__global__ __launch_bounds__(kScanThreads) void scan_tiles(int64_t n, const int32_t* __restrict__ count,
                                                           int32_t* __restrict__ start, int32_t* __restrict__ sums) {
  __shared__ int32_t part[kScanThreads];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)t * kScanItems;
  int32_t v[kScanItems];
  int32_t run = 0;
#pragma unroll
  for (int e = 0; e < kScanItems; ++e) {
    v[e] = base + e < n ? count[base + e] : 0;
    run += v[e];
  }
  part[t] = run;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread totals
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const int32_t add = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  int32_t acc = part[t] - run;
#pragma unroll
  for (int e = 0; e < kScanItems; ++e) {
    if (base + e < n) start[base + e] = acc;
    acc += v[e];
  }
  if (t == kScanThreads - 1) sums[blockIdx.x] = part[t];
}

// Exclusive scan of the tile totals by one block, chunk after chunk.
__global__ __launch_bounds__(kScanThreads) void scan_sums(int64_t n, int32_t* __restrict__ sums) {
  __shared__ int32_t part[kScanThreads];
  const int t = threadIdx.x;
  int32_t carry = 0;
  for (int64_t b0 = 0; b0 < n; b0 += kScanThreads) {
    const int64_t i = b0 + t;
    const int32_t x = i < n ? sums[i] : 0;
    part[t] = x;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
      const int32_t add = t >= off ? part[t - off] : 0;
      __syncthreads();
      part[t] += add;
      __syncthreads();
    }
    if (i < n) sums[i] = carry + part[t] - x;
    const int32_t total = part[kScanThreads - 1];
    __syncthreads();
    carry += total;
  }
}

__global__ __launch_bounds__(kBlock) void scan_add(int64_t n, int32_t* __restrict__ start,
                                                   const int32_t* __restrict__ sums, int32_t total) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) start[i] += sums[i / kScanTile];
  if (i == n) start[n] = total;
}

// Copy each point into its cell's range.  The counts are consumed as cursors.
__global__ __launch_bounds__(kBlock) void scatter_points(int64_t n, const double* __restrict__ pts, int64_t ld,
                                                         const int32_t* __restrict__ cell,
                                                         const int32_t* __restrict__ start,
                                                         int32_t* __restrict__ count, double* __restrict__ sx,
                                                         double* __restrict__ sy, double* __restrict__ sz,
                                                         int32_t* __restrict__ sidx) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int c = cell[i];
  const int32_t slot = start[c] + atomicSub(&count[c], 1) - 1;
  sx[slot] = pts[i];
  sy[slot] = pts[ld + i];
  sz[slot] = pts[2 * ld + i];
  sidx[slot] = (int32_t)i;
}

// Lower bound on the distance from the query to cell offset o along one axis,
// given the query's offset f inside its own cell of side c.
__device__ __forceinline__ double axis_gap(int o, double f, double c) {
  double g = o > 0 ? (o - 1) * c + (c - f) : (o < 0 ? (-o - 1) * c + f : 0.0);
  g -= kGapSlack;
  return g > 0.0 ? g : 0.0;
}

struct GridView {
  const double *sx, *sy, *sz;
  const int32_t *sidx, *start;
  int G;
};

// One thread per query.  The sorted k best live in dynamic LDS as [slot][thread].
__global__ __launch_bounds__(kQueryBlock) void knn_query(GridView gr, const double* __restrict__ qry, int64_t ldq,
                                                         int64_t m, int k, int32_t* __restrict__ idx,
                                                         int64_t ld_idx) {
  extern __shared__ double lds_d[];
  double* D = lds_d;
  int32_t* I = reinterpret_cast<int32_t*>(lds_d + (size_t)k * kQueryBlock);
  const int t = threadIdx.x;
  const int64_t j = (int64_t)blockIdx.x * kQueryBlock + t;
  if (j >= m) return;  // no block-wide synchronisation below
  const int G = gr.G;
  const double c = 1.0 / G;
  const double qx = qry[j], qy = qry[ldq + j], qz = qry[2 * ldq + j];
  const double wx = wrap01(qx), wy = wrap01(qy), wz = wrap01(qz);
  const int cx = cell_of(wx, G), cy = cell_of(wy, G), cz = cell_of(wz, G);
  const double fx = fmin(fmax(wx - cx * c, 0.0), c), fy = fmin(fmax(wy - cy * c, 0.0), c),
               fz = fmin(fmax(wz - cz * c, 0.0), c);
  const double near = fmin(fmin(fmin(fx, c - fx), fmin(fy, c - fy)), fmin(fz, c - fz));
  int cnt = 0;
  double kd = 0.0;  // k-th distance once cnt == k
  int32_t ki = 0;
  const int rmax = (G - 1) / 2;
  for (int R = 0; R <= rmax; ++R) {
    if (cnt == k && R >= 1) {
      const double g = (R - 1) * c + near - kGapSlack;
      if (g > 0.0 && g * g > kd) break;  // every unvisited point is farther than the k-th
    }
    for (int dx = -R; dx <= R; ++dx) {
      const int ox = cx + dx;
      const int gx = ox < 0 ? ox + G : (ox >= G ? ox - G : ox);
      const double bx = axis_gap(dx, fx, c);
      for (int dy = -R; dy <= R; ++dy) {
        const int oy = cy + dy;
        const int gy = oy < 0 ? oy + G : (oy >= G ? oy - G : oy);
        const double by = axis_gap(dy, fy, c);
        const bool side = dx == -R || dx == R || dy == -R || dy == R;
        const int step = side ? 1 : (R > 0 ? 2 * R : 1);
        for (int dz = -R; dz <= R; dz += step) {
          const double bz = axis_gap(dz, fz, c);
          if (cnt == k && bx * bx + by * by + bz * bz > kd) continue;
          const int oz = cz + dz;
          const int gz = oz < 0 ? oz + G : (oz >= G ? oz - G : oz);
          const int cell = (gx * G + gy) * G + gz;
          const int32_t s1 = gr.start[cell + 1];
          for (int32_t s = gr.start[cell]; s < s1; ++s) {
            const double d = dist2(gr.sx[s], gr.sy[s], gr.sz[s], qx, qy, qz);
            const int32_t id = gr.sidx[s];
            if (cnt == k && !(d < kd || (d == kd && id < ki))) continue;
            int p = cnt < k ? cnt : k - 1;
            while (p > 0) {
              const double dp = D[(p - 1) * kQueryBlock + t];
              const int32_t ip = I[(p - 1) * kQueryBlock + t];
              if (!(dp > d || (dp == d && ip > id))) break;
              D[p * kQueryBlock + t] = dp;
              I[p * kQueryBlock + t] = ip;
              --p;
            }
            D[p * kQueryBlock + t] = d;
            I[p * kQueryBlock + t] = id;
            if (cnt < k) ++cnt;
            if (cnt == k) {
              kd = D[(k - 1) * kQueryBlock + t];
              ki = I[(k - 1) * kQueryBlock + t];
            }
          }
        }
      }
    }
  }
  for (int col = 0; col < k; ++col) idx[col * ld_idx + j] = I[col * kQueryBlock + t];
}

__global__ __launch_bounds__(kBlock) void own_index(int64_t m, int32_t first, int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < m) out[i] = first + (int32_t)i;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Layout {
  size_t cell, count, start, sums, sx, sy, sz, sidx, total;
};

Layout layout(int64_t n, int G) {
  const int64_t cells = (int64_t)G * G * G;
  const int64_t tiles = (cells + kScanTile - 1) / kScanTile;
  Layout L;
  size_t o = 0;
  L.cell = o; o += align256(sizeof(int32_t) * n);
  L.count = o; o += align256(sizeof(int32_t) * cells);
  L.start = o; o += align256(sizeof(int32_t) * (cells + 1));
  L.sums = o; o += align256(sizeof(int32_t) * tiles);
  L.sx = o; o += align256(sizeof(double) * n);
  L.sy = o; o += align256(sizeof(double) * n);
  L.sz = o; o += align256(sizeof(double) * n);
  L.sidx = o; o += align256(sizeof(int32_t) * n);
  L.total = o;
  return L;
}

// Bin n points (rows of stride ld) into the grid held in ws.
int build_grid(const double* pts, int64_t n, int64_t ld, char* ws, GridView& gv, hipStream_t st) {
  const int G = grid_side(n);
  const Layout L = layout(n, G);
  const int64_t cells = (int64_t)G * G * G;
  const int64_t tiles = (cells + kScanTile - 1) / kScanTile;
  int32_t* cell = (int32_t*)(ws + L.cell);
  int32_t* count = (int32_t*)(ws + L.count);
  int32_t* start = (int32_t*)(ws + L.start);
  int32_t* sums = (int32_t*)(ws + L.sums);
  double* sx = (double*)(ws + L.sx);
  double* sy = (double*)(ws + L.sy);
  double* sz = (double*)(ws + L.sz);
  int32_t* sidx = (int32_t*)(ws + L.sidx);
  hipLaunchKernelGGL(fill_i32, dim3(grid_for(cells, kBlock)), dim3(kBlock), 0, st, cells, count, 0);
  hipLaunchKernelGGL(bin_points, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, st, n, pts, ld, G, cell, count);
  hipLaunchKernelGGL(scan_tiles, dim3((unsigned)tiles), dim3(kScanThreads), 0, st, cells, (const int32_t*)count,
                     start, sums);
  hipLaunchKernelGGL(scan_sums, dim3(1), dim3(kScanThreads), 0, st, tiles, sums);
  hipLaunchKernelGGL(scan_add, dim3(grid_for(cells + 1, kBlock)), dim3(kBlock), 0, st, cells, start,
                     (const int32_t*)sums, (int32_t)n);
  hipLaunchKernelGGL(scatter_points, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, st, n, pts, ld,
                     (const int32_t*)cell, (const int32_t*)start, count, sx, sy, sz, sidx);
  MPF_LAUNCH_CHECK();
  gv = GridView{sx, sy, sz, sidx, start, G};
  return MPF_OK;
}

int query(const GridView& gv, const double* qry, int64_t ldq, int64_t m, int k, int32_t* idx, int64_t ld_idx,
          hipStream_t st) {
  if (m == 0) return MPF_OK;
  const size_t lds = (size_t)k * kQueryBlock * (sizeof(double) + sizeof(int32_t));
  hipLaunchKernelGGL(knn_query, dim3(grid_for(m, kQueryBlock)), dim3(kQueryBlock), lds, st, gv, qry, ldq, m, k,
                     idx, ld_idx);
  MPF_LAUNCH_CHECK();
  return MPF_OK;
}

}  // namespace
}  // namespace mpf

extern "C" size_t mpf_knn_workspace(int64_t n_pts) {
  using namespace mpf;
  if (n_pts < 1) n_pts = 1;
  return layout(n_pts, grid_side(n_pts)).total;
}

extern "C" int mpf_knn(const double* pts, int64_t n_pts, int64_t ld_pts, const double* qry, int64_t n_qry,
                       int64_t ld_qry, int k, int32_t* idx, int64_t ld_idx, void* ws, size_t ws_bytes,
                       void* stream) {
  using namespace mpf;
  if (!pts || n_pts < 1 || n_pts > INT32_MAX || ld_pts < n_pts || n_qry < 0 || k < 1 || k > kMaxK ||
      (int64_t)k > n_pts)
    return MPF_ERR_ARG;
  if (n_qry == 0) return MPF_OK;
  if (!qry || !idx || ld_qry < n_qry || ld_idx < n_qry || !ws) return MPF_ERR_ARG;
  if (ws_bytes < mpf_knn_workspace(n_pts)) return MPF_ERR_ARG;
  hipStream_t st = as_stream(stream);
  GridView gv;
  int rc = build_grid(pts, n_pts, ld_pts, (char*)ws, gv, st);
  if (rc != MPF_OK) return rc;
  return query(gv, qry, ld_qry, n_qry, k, idx, ld_idx, st);
}

extern "C" int mpf_solver_stencils(const double* pos, int64_t n, int64_t n_int, int nl, int32_t* sten, void* ws,
                                   size_t ws_bytes, void* stream) {
  using namespace mpf;
  if (!pos || !sten || !ws || n < 1 || n > INT32_MAX || n_int < 0 || n_int > n || nl < 2 || nl > kMaxK ||
      (int64_t)nl > n)
    return MPF_ERR_ARG;
  const int64_t nb = n - n_int;
  if (nb > 0 && n_int < nl - 1) return MPF_ERR_ARG;
  if (ws_bytes < mpf_knn_workspace(n)) return MPF_ERR_ARG;
  hipStream_t st = as_stream(stream);
  GridView gv;
  int rc;
  if (n_int > 0) {  // interior rows: the nl nearest of all nodes (the node itself first)
    rc = build_grid(pos, n, n, (char*)ws, gv, st);
    if (rc != MPF_OK) return rc;
    rc = query(gv, pos, n, n_int, nl, sten, n, st);
    if (rc != MPF_OK) return rc;
  }
  if (nb > 0) {  // surface rows: the node itself, then its nl - 1 nearest interior nodes
    rc = build_grid(pos, n_int, n, (char*)ws, gv, st);
    if (rc != MPF_OK) return rc;
    hipLaunchKernelGGL(own_index, dim3(grid_for(nb, kBlock)), dim3(kBlock), 0, st, nb, (int32_t)n_int,
                       sten + n_int);
    MPF_LAUNCH_CHECK();
    rc = query(gv, pos + n_int, n, nb, nl - 1, sten + n + n_int, n, st);
    if (rc != MPF_OK) return rc;
  }
  return MPF_OK;
}
