// Tile/halo planning for the LDS-staged stencil gather on gfx950.
//
// The MLBM step works on tiles of 64 consecutive (Morton-ordered) nodes.
// The stencils of a tile (Sec. 2.1: each node's N_L nearest nodes) overlap
// heavily: on the refined clouds here its 64 x 30 entries name about 350
// distinct nodes.  The plan lists, once per geometry, each tile's distinct
// stencil nodes in ascending order (its halo) and rewrites every stencil
// entry as a 16-bit position in that list.  A step then copies the halo's
// records into LDS with contiguous loads and reads the neighbours' records
// from LDS, instead of issuing one scattered record load per (node, column)
// through the caches; the stencil indices shrink from 4 to 2 bytes.
//
// One block per tile: the tile's entries are sorted in LDS (bitonic),
// duplicates dropped by a block scan, and each entry's position found by
// binary search in the sorted list.  Tiles of 128 or 256 nodes serve the ACM
// passes, whose blocks of 256 lanes then share one halo (at one or two lanes
// per node): 3.7 instead of 5.5 halo entries per node on these clouds.
#include <climits>

#include "common.hpp"

namespace mpf {
namespace {

constexpr int kTileNodes = 64;  // the default tile (the MLBM step's)
constexpr int kPlanBlock = 256;

// PMAX: entries of a tile at the largest stencil (tile nodes x 64), a power of two
template <int PMAX>
__global__ __launch_bounds__(kPlanBlock) void tile_plan_kernel(int64_t n, int nl, const int32_t* __restrict__ sten,
                                                               int ts, int h_cap, int32_t* __restrict__ count,
                                                               int32_t* __restrict__ halo,
                                                               uint16_t* __restrict__ lidx, int64_t G) {
  __shared__ int32_t key[PMAX];
  __shared__ int32_t uniq[PMAX];
  __shared__ int32_t part[kPlanBlock + 1];
  const int t = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t i0 = tile * ts;
  const int nt = (int)(n - i0 < ts ? n - i0 : ts);
  const int E = nt * nl;
  int P = 1;
  while (P < E) P <<= 1;
  // entry e = (column j, node i0 + i) with e = j nt + i: rows read contiguously
  for (int e = t; e < P; e += kPlanBlock)
    key[e] = e < E ? sten[(int64_t)(e / nt) * n + i0 + e % nt] : INT_MAX;
  // bitonic sort, ascending
  for (int k = 2; k <= P; k <<= 1)
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      __syncthreads();
      for (int e = t; e < P; e += kPlanBlock) {
        const int o = e ^ jj;
        if (o > e) {
          const int32_t a = key[e], b = key[o];
          if ((a > b) == ((e & k) == 0)) {
            key[e] = b;
            key[o] = a;
          }
        }
      }
    }
  __syncthreads();
  // first occurrences, numbered by an exclusive scan: thread t owns the
  // contiguous chunk [t c, (t + 1) c)
  const int c = (P + kPlanBlock - 1) / kPlanBlock;
  int local = 0;
  for (int e = t * c; e < (t + 1) * c && e < P; ++e)
    local += (e < E && (e == 0 || key[e] != key[e - 1])) ? 1 : 0;
  part[t + 1] = local;
  if (t == 0) part[0] = 0;
  __syncthreads();
  if (t == 0)
    for (int s = 1; s <= kPlanBlock; ++s) part[s] += part[s - 1];
  __syncthreads();
  int pos = part[t];
  for (int e = t * c; e < (t + 1) * c && e < P; ++e)
    if (e < E && (e == 0 || key[e] != key[e - 1])) uniq[pos++] = key[e];
  const int U = part[kPlanBlock];
  __syncthreads();
  for (int r = t; r < U && r < h_cap; r += kPlanBlock) halo[tile * h_cap + r] = uniq[r];
  // every entry's position in the list
  for (int e = t; e < E; e += kPlanBlock) {
    const int64_t at = (int64_t)(e / nt) * n + i0 + e % nt;
    const int32_t v = sten[at];
    int lo = 0, hi = U - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (uniq[mid] < v) lo = mid + 1;
      else hi = mid;
    }
    lidx[at] = (uint16_t)lo;
  }
  if (t == 0) {
    count[tile] = U;
    atomicMax(count + G, U);  // the largest halo, in the extra entry
  }
}

__global__ void zero_int(int32_t* x) { *x = 0; }

}  // namespace
}  // namespace mpf

extern "C" int64_t mpf_tile_count_sized(int64_t n, int tile) {
  return n > 0 && tile > 0 ? (n + tile - 1) / tile : 0;
}

extern "C" int64_t mpf_tile_count(int64_t n) { return mpf_tile_count_sized(n, mpf::kTileNodes); }

extern "C" int mpf_tile_plan_sized(int64_t n, int nl, const int32_t* sten, int tile, int h_cap, int32_t* count,
                                   int32_t* halo, uint16_t* lidx, int32_t* h_max_host, void* stream) {
  using namespace mpf;
  if (n < 1 || nl < 1 || nl > 64 || !sten || !count || !halo || !lidx || !h_max_host) return MPF_ERR_ARG;
  if (tile != 64 && tile != 128 && tile != 256) return MPF_ERR_ARG;
  if (h_cap < kTileNodes || h_cap > tile * 64) return MPF_ERR_ARG;
  if (n > INT32_MAX) return MPF_ERR_ARG;
  const int64_t G = mpf_tile_count_sized(n, tile);
  hipStream_t st = as_stream(stream);
  hipLaunchKernelGGL(zero_int, dim3(1), dim3(1), 0, st, count + G);
  if (tile == 64)
    hipLaunchKernelGGL(tile_plan_kernel<64 * 64>, dim3((unsigned)G), dim3(kPlanBlock), 0, st, n, nl, sten, tile,
                       h_cap, count, halo, lidx, G);
  else if (tile == 128)
    hipLaunchKernelGGL(tile_plan_kernel<128 * 64>, dim3((unsigned)G), dim3(kPlanBlock), 0, st, n, nl, sten, tile,
                       h_cap, count, halo, lidx, G);
  else
    hipLaunchKernelGGL(tile_plan_kernel<256 * 64>, dim3((unsigned)G), dim3(kPlanBlock), 0, st, n, nl, sten, tile,
                       h_cap, count, halo, lidx, G);
  MPF_LAUNCH_CHECK();
  int32_t hm = 0;
  MPF_HIP(hipMemcpyAsync(&hm, count + G, sizeof(hm), hipMemcpyDeviceToHost, st));
  MPF_HIP(hipStreamSynchronize(st));
  *h_max_host = hm;
  return hm > h_cap ? MPF_ERR_UNSUPPORTED : MPF_OK;
}

extern "C" int mpf_tile_plan(int64_t n, int nl, const int32_t* sten, int h_cap, int32_t* count, int32_t* halo,
                             uint16_t* lidx, int32_t* h_max_host, void* stream) {
  return mpf_tile_plan_sized(n, nl, sten, mpf::kTileNodes, h_cap, count, halo, lidx, h_max_host, stream);
}
