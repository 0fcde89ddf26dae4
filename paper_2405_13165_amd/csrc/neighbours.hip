// Neighbourhoods S_i of Eq. (Nbd) by a cell list over Morton-ordered cells.
//
// Pipeline (one stream, one host read-back of sizes):
//   bbox/validate -> cell keys + per-cell counts (atomics) -> scan -> scatter
//   into cell order -> positions gathered in cell order -> per-particle count
//   over the 27 surrounding cells -> scan -> fill -> per-row bitonic sort
//   -> grouping of particles by (model, neighbour-count band) for the
//   batched stencil kernels.
// Cells are cubes of edge max(h) (per model, or over all particles for the
// cross-model sets), so every member of S_i lies in the 27 cells around i.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kMaxRow = 2048;

// -------------------------------------------------------------- reductions
__device__ inline double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// per model: lo[3], hi[3], hmax  (7 doubles) -> 14 doubles + invalid count
constexpr int kBoxVals = 14;

__global__ void __launch_bounds__(kBlock) k_bbox(const double *__restrict__ x, const double *__restrict__ y,
                                                 const double *__restrict__ z, const double *__restrict__ h,
                                                 const int8_t *__restrict__ model, int64_t n,
                                                 double *__restrict__ part, int *__restrict__ bad_part) {
  double v[kBoxVals];
  for (int m = 0; m < 2; ++m) {
    for (int d = 0; d < 3; ++d) { v[m * 7 + d] = INFINITY; v[m * 7 + 3 + d] = -INFINITY; }
    v[m * 7 + 6] = 0.0;
  }
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double p[3] = {x[i], y[i], z[i]};
    double hi = h[i];
    int m = model[i];
    bool ok = (m == 0 || m == 1) && isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]) && isfinite(hi) && hi > 0.0;
    if (!ok) { ++bad; continue; }
    for (int mm = 0; mm < 2; ++mm) {
      if (mm != m) continue;
      for (int d = 0; d < 3; ++d) {
        v[mm * 7 + d] = fmin(v[mm * 7 + d], p[d]);
        v[mm * 7 + 3 + d] = fmax(v[mm * 7 + 3 + d], p[d]);
      }
      v[mm * 7 + 6] = fmax(v[mm * 7 + 6], hi);
    }
  }
  __shared__ double sh[kBlock / 64][kBoxVals];
  __shared__ int shb[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = 0; k < kBoxVals; ++k) {
    int kk = k % 7;
    double r = (kk < 3) ? wave_min(v[k]) : wave_max(v[k]);
    if (lane == 0) sh[wid][k] = r;
  }
  int bs = wave_sum_i(bad);
  if (lane == 0) shb[wid] = bs;
  __syncthreads();
  if (threadIdx.x < kBoxVals) {
    int k = threadIdx.x, kk = k % 7;
    double r = sh[0][k];
    for (int w = 1; w < kBlock / 64; ++w) r = (kk < 3) ? fmin(r, sh[w][k]) : fmax(r, sh[w][k]);
    part[(int64_t)blockIdx.x * kBoxVals + k] = r;
  }
  if (threadIdx.x == 0) {
    int b = 0;
    for (int w = 0; w < kBlock / 64; ++w) b += shb[w];
    bad_part[blockIdx.x] = b;
  }
}

__global__ void k_bbox_final(const double *__restrict__ part, const int *__restrict__ bad_part, int nblk,
                             double *__restrict__ out, int *__restrict__ bad_out) {
  int k = threadIdx.x;
  if (k < kBoxVals) {
    int kk = k % 7;
    double r = part[k];
    for (int b = 1; b < nblk; ++b) {
      double t = part[(int64_t)b * kBoxVals + k];
      r = (kk < 3) ? fmin(r, t) : fmax(r, t);
    }
    out[k] = r;
  }
  if (k == 0) {
    int s = 0;
    for (int b = 0; b < nblk; ++b) s += bad_part[b];
    *bad_out = s;
  }
}

// -------------------------------------------------------------- grid
struct Grid {
  double lo[2][3];
  double inv_edge[2];
  int dim[2][3];
  int bits[2][3];
  int64_t base[2];  // key offset of each model's cells
  int64_t nkeys;
  int per_model;    // 1: separate grids per model; 0: one grid for all
};

__device__ inline int cell_of(double v, double lo, double inv_edge, int dim) {
  double t = floor((v - lo) * inv_edge);
  int c = (t < 0.0) ? 0 : (t >= (double)dim ? dim - 1 : (int)t);
  return c;
}

// Morton interleave with possibly different bit counts per axis
__device__ inline int64_t morton(int cx, int cy, int cz, int bx, int by, int bz) {
  int64_t key = 0;
  int pos = 0;
  int mb = max(bx, max(by, bz));
  for (int b = 0; b < mb; ++b) {
    if (b < bx) key |= (int64_t)((cx >> b) & 1) << pos++;
    if (b < by) key |= (int64_t)((cy >> b) & 1) << pos++;
    if (b < bz) key |= (int64_t)((cz >> b) & 1) << pos++;
  }
  return key;
}

__device__ inline int grid_slot(const Grid &g, int m) { return g.per_model ? m : 0; }

__global__ void __launch_bounds__(kBlock) k_fill_i32(int32_t *a, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

__global__ void __launch_bounds__(kBlock) k_keys(const double *__restrict__ x, const double *__restrict__ y,
                                                 const double *__restrict__ z, const int8_t *__restrict__ model,
                                                 int64_t n, Grid g, int32_t *__restrict__ key,
                                                 int32_t *__restrict__ slot, int32_t *__restrict__ counts) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int s = grid_slot(g, model[i]);
  int cx = cell_of(x[i], g.lo[s][0], g.inv_edge[s], g.dim[s][0]);
  int cy = cell_of(y[i], g.lo[s][1], g.inv_edge[s], g.dim[s][1]);
  int cz = cell_of(z[i], g.lo[s][2], g.inv_edge[s], g.dim[s][2]);
  int32_t k = (int32_t)(g.base[s] + morton(cx, cy, cz, g.bits[s][0], g.bits[s][1], g.bits[s][2]));
  key[i] = k;
  slot[i] = atomicAdd(&counts[k], 1);
}

__global__ void __launch_bounds__(kBlock) k_scatter(const int32_t *__restrict__ key, const int32_t *__restrict__ slot,
                                                    const int32_t *__restrict__ cell_start, int64_t n,
                                                    int32_t *__restrict__ order) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  order[cell_start[key[i]] + slot[i]] = (int32_t)i;
}

// Order the particles of each cell by a finer Morton key (kSubBits more bits
// per axis), so that runs of the cell order stay spatially compact when a
// cell is much larger than a typical support (uneven h).  One wave per cell,
// bitonic sort in LDS; cells with more than kCellSort particles keep their
// order.  The neighbour sets do not depend on this order.
constexpr int kSubBits = 4;
constexpr int kCellSort = 2048;

__device__ inline uint64_t fine_key(double x, double y, double z, const Grid &g, int s) {
  const double f = (double)(1 << kSubBits);
  int c[3];
  const double v[3] = {x, y, z};
  for (int d = 0; d < 3; ++d) {
    const double t = floor((v[d] - g.lo[s][d]) * g.inv_edge[s] * f);
    const double hi = (double)g.dim[s][d] * f - 1.0;
    c[d] = (int)(t < 0.0 ? 0.0 : (t > hi ? hi : t));
  }
  uint64_t key = 0;
  int pos = 0;
  for (int b = 0; b < 21; ++b)
    for (int d = 0; d < 3; ++d) key |= (uint64_t)((c[d] >> b) & 1) << pos++;
  return key;
}

__global__ void __launch_bounds__(64) k_cell_sort(const int32_t *__restrict__ cell_start, int64_t ncells,
                                                  const double *__restrict__ x, const double *__restrict__ y,
                                                  const double *__restrict__ z, const int8_t *__restrict__ model,
                                                  Grid g, int32_t *__restrict__ order) {
  __shared__ uint64_t kk[kCellSort];
  __shared__ int32_t id[kCellSort];
  for (int64_t c = blockIdx.x; c < ncells; c += gridDim.x) {
    const int32_t b = cell_start[c], len = cell_start[c + 1] - b;
    if (len <= 1 || len > kCellSort) continue;
    int P = 1;
    while (P < len) P <<= 1;
    for (int t = threadIdx.x; t < P; t += 64) {
      if (t < len) {
        const int32_t i = order[b + t];
        kk[t] = fine_key(x[i], y[i], z[i], g, grid_slot(g, model[i]));
        id[t] = i;
      } else {
        kk[t] = ~0ull;
        id[t] = 0x7fffffff;
      }
    }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int t = threadIdx.x; t < P; t += 64) {
          const int u = t ^ j;
          if (u > t) {
            const uint64_t a = kk[t], e = kk[u];
            const int32_t ia = id[t], ie = id[u];
            // ties (same sub-cell) by particle index: the order is deterministic
            const bool gt = (a > e) || (a == e && ia > ie);
            if (gt == ((t & k) == 0)) { kk[t] = e; kk[u] = a; id[t] = ie; id[u] = ia; }
          }
        }
        __syncthreads();
      }
    }
    for (int t = threadIdx.x; t < len; t += 64) order[b + t] = id[t];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kBlock) k_gather_pos(const int32_t *__restrict__ order, const double *__restrict__ x,
                                                       const double *__restrict__ y, const double *__restrict__ z,
                                                       const double *__restrict__ h, int64_t n,
                                                       double4 *__restrict__ sp) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  int32_t i = order[s];
  sp[s] = make_double4(x[i], y[i], z[i], h[i]);
}

// Eq. (Nbd) predicate, evaluated as written without contraction so that the
// decision is reproducible across implementations.
__device__ inline bool in_support(double4 a, double4 b) {
#pragma clang fp contract(off)
  double dx = b.x - a.x;
  double dy = b.y - a.y;
  double dz = b.z - a.z;
  double d2 = (dx * dx + dy * dy) + dz * dz;
  double r = 0.5 * (a.w + b.w);
  return d2 <= r * r;
}

// MODE 0: count (cnt[i] = |S_i|, group histogram, max row); MODE 1: fill col.
// Particles i >= n_rows (ghost particles) appear in the rows of others but
// their own row holds only i.
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_search(const int32_t *__restrict__ order, const double4 *__restrict__ sp,
                                                   const int8_t *__restrict__ model, const int32_t *__restrict__ cell_start,
                                                   int64_t n, int64_t n_rows, Grid g, int32_t *__restrict__ cnt,
                                                   int32_t *__restrict__ hist, int32_t *__restrict__ maxrow,
                                                   const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col) {
  const int64_t sidx0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = sidx0 < n;
  if (MODE == 1 && !valid) return;
  // MODE 0 keeps the idle lanes of the last wave alive for the wave-wide
  // histogram below; they search on behalf of particle n-1 and count nothing
  const int64_t sidx = valid ? sidx0 : n - 1;
  const int32_t i = order[sidx];
  const double4 pi = sp[sidx];
  const int m = model[i];
  const int s = grid_slot(g, m);
  const int cx = cell_of(pi.x, g.lo[s][0], g.inv_edge[s], g.dim[s][0]);
  const int cy = cell_of(pi.y, g.lo[s][1], g.inv_edge[s], g.dim[s][1]);
  const int cz = cell_of(pi.z, g.lo[s][2], g.inv_edge[s], g.dim[s][2]);
  int c = 0;
  int64_t out = 0;
  if (MODE == 1) out = row_ptr[i];
  if (i >= n_rows) {
    if (MODE == 1) col[out] = i;
    c = 1;
  } else
  for (int dz = -1; dz <= 1; ++dz) {
    int zz = cz + dz;
    if (zz < 0 || zz >= g.dim[s][2]) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      int yy = cy + dy;
      if (yy < 0 || yy >= g.dim[s][1]) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        int xx = cx + dx;
        if (xx < 0 || xx >= g.dim[s][0]) continue;
        int64_t k = g.base[s] + morton(xx, yy, zz, g.bits[s][0], g.bits[s][1], g.bits[s][2]);
        int32_t b = cell_start[k], e = cell_start[k + 1];
        for (int32_t t = b; t < e; ++t) {
          if (in_support(pi, sp[t])) {
            if (MODE == 1) {
              if (c < kMaxRow) col[out + c] = order[t];
            }
            ++c;
          }
        }
      }
    }
  }
  if (MODE == 0) {
    if (valid) cnt[i] = c;
    int band = 0;
    while (band < GF_NBAND - 1 && c > kBandHi[band]) ++band;
    // one atomic per wave and bin: same-address atomics from every particle
    // serialise in L2 and used to dominate this kernel
    const int bin = valid ? m * GF_NBAND + band : -1;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int b = 0; b < 2 * GF_NBAND; ++b) {
      const unsigned long long mask = __ballot(bin == b);
      if (lane == 0 && mask) atomicAdd(&hist[b], __popcll(mask));
    }
    int cm = valid ? c : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cm = max(cm, __shfl_xor(cm, o, 64));
    if (lane == 0) atomicMax(maxrow, cm);
  }
}

// Sort each row ascending: one wave per row, bitonic network in LDS.
__global__ void __launch_bounds__(64) k_row_sort(const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col,
                                                 int64_t n) {
  __shared__ int32_t buf[kMaxRow];
  const int64_t i = blockIdx.x;
  if (i >= n) return;
  const int64_t b = row_ptr[i];
  const int len = (int)(row_ptr[i + 1] - b);
  if (len <= 1) return;
  int P = 1;
  while (P < len) P <<= 1;
  for (int t = threadIdx.x; t < P; t += 64) buf[t] = (t < len) ? col[b + t] : 0x7fffffff;
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < P; t += 64) {
        int u = t ^ j;
        if (u > t) {
          int32_t a = buf[t], c = buf[u];
          bool up = (t & k) == 0;
          if ((a > c) == up) { buf[t] = c; buf[u] = a; }
        }
      }
      __syncthreads();
    }
  }
  for (int t = threadIdx.x; t < len; t += 64) col[b + t] = buf[t];
}

// grouping: particles (in cell order) of group gsel, stable; the tiled
// bands 0..kTileBand share the group of band kTileBand
__global__ void __launch_bounds__(kBlock) k_group_flag(const int32_t *__restrict__ order, const int32_t *__restrict__ cnt,
                                                       const int8_t *__restrict__ model, int64_t n, int gsel,
                                                       int32_t *__restrict__ flag) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  int32_t i = order[s];
  int c = cnt[i];
  int band = 0;
  while (band < GF_NBAND - 1 && c > kBandHi[band]) ++band;
  if (band < kTileBand) band = kTileBand;  // the tiled bands form one Morton-ordered range
  flag[s] = (model[i] * GF_NBAND + band) == gsel ? 1 : 0;
}

__global__ void __launch_bounds__(kBlock) k_group_scatter(const int32_t *__restrict__ order,
                                                          const int32_t *__restrict__ flag,
                                                          const int32_t *__restrict__ pos, int64_t n,
                                                          int64_t base, int32_t *__restrict__ grouped) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  if (flag[s]) grouped[base + pos[s]] = order[s];
}

// ---------------------------------------------------------------- tiles
// Tiled row ranges (one per model), as passed to the tile kernels: tiles
// [tile_start[q], tile_start[q+1]) cover rows [row_start[q], row_start[q] +
// nrows[q]) of the grouped order; gsel[q] is the model.
struct TileGroups {
  int nq = 0;
  int gsel[2];
  int64_t tile_start[3];
  int64_t row_start[2];
  int64_t nrows[2];
};
constexpr int kTileEntries = kTileRows * kTileBandRow;  // entries one tile can hold
constexpr int kTileThreads = 512;

// orders the LDS traffic of the lanes of one wave
__device__ inline void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int tile_group(const TileGroups &tg, int64_t t) {
  int q = 0;
  while (q + 1 < tg.nq && t >= tg.tile_start[q + 1]) ++q;
  return q;
}

// number of neighbour entries of each tile
__global__ void __launch_bounds__(kBlock) k_tile_entries(TileGroups tg, const int64_t *__restrict__ row_ptr,
                                                         const int32_t *__restrict__ grouped,
                                                         int32_t *__restrict__ ent) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= tg.tile_start[tg.nq]) return;
  const int q = tile_group(tg, t);
  const int64_t r0 = (t - tg.tile_start[q]) * kTileRows;
  const int64_t r1 = min(r0 + kTileRows, tg.nrows[q]);
  int64_t e = 0;
  for (int64_t r = r0; r < r1; ++r) {
    const int32_t i = grouped[tg.row_start[q] + r];
    e += row_ptr[i + 1] - row_ptr[i];
  }
  ent[t] = (int32_t)e;
}

// One block per tile: sort the tile's (index, entry) pairs, number the
// distinct indices in ascending order, write slot[] for every entry and the
// distinct indices to uniq[ent_off[t] ...]; cnt[t] = number of distinct.
__global__ void __launch_bounds__(kTileThreads) k_tile_unique(TileGroups tg, const int64_t *__restrict__ row_ptr,
                                                              const int32_t *__restrict__ col,
                                                              const int32_t *__restrict__ grouped,
                                                              const int64_t *__restrict__ ent_off,
                                                              uint16_t *__restrict__ slot,
                                                              int32_t *__restrict__ uniq, int32_t *__restrict__ cnt,
                                                              int32_t *__restrict__ grp_max) {
  __shared__ uint64_t key[kTileEntries];
  __shared__ int64_t rbase[kTileRows];
  __shared__ int32_t rloc[kTileRows + 1];
  __shared__ int32_t csum[kTileThreads];
  const int64_t t = blockIdx.x;
  const int q = tile_group(tg, t);
  const int64_t r0 = (t - tg.tile_start[q]) * kTileRows;
  const int R = (int)min((int64_t)kTileRows, tg.nrows[q] - r0);
  const int tid = threadIdx.x;
  if (tid < 64) {
    int len = 0;
    if (tid < R) {
      const int32_t i = grouped[tg.row_start[q] + r0 + tid];
      rbase[tid] = row_ptr[i];
      len = (int)(row_ptr[i + 1] - row_ptr[i]);
    }
    int inc = len;  // inclusive wave scan
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(inc, o, 64);
      if (tid >= o) inc += v;
    }
    if (tid < kTileRows) rloc[tid + 1] = inc;
    if (tid == 0) rloc[0] = 0;
  }
  __syncthreads();
  const int E = rloc[R];
  int P = 1;
  while (P < E) P <<= 1;
  auto row_of = [&](int e) {  // row r with rloc[r] <= e < rloc[r+1]
    int lo = 0, hi = R - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rloc[mid] <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
  };
  for (int e = tid; e < P; e += kTileThreads) {
    if (e < E) {
      const int r = row_of(e);
      const int32_t j = col[rbase[r] + (e - rloc[r])];
      key[e] = ((uint64_t)(uint32_t)j << 12) | (uint64_t)e;
    } else {
      key[e] = ~0ull;
    }
  }
  __syncthreads();
  // Bitonic network.  Element e is handled by thread e mod kTileThreads, so a
  // stage of distance j < 64 pairs lanes of one wave; a block barrier is
  // only needed around stages of distance >= 64.
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int e = tid; e < P; e += kTileThreads) {
        const int u = e ^ j;
        if (u > e) {
          const uint64_t a = key[e], b = key[u];
          if ((a > b) == ((e & k) == 0)) { key[e] = b; key[u] = a; }
        }
      }
      const int jn = (j > 1) ? (j >> 1) : k;  // distance of the next stage
      if (j >= 64 || jn >= 64) __syncthreads();
      else wave_fence();
    }
  }
  __syncthreads();
  // each thread numbers a contiguous chunk of the sorted list
  const int chunk = (P + kTileThreads - 1) / kTileThreads;
  const int s0 = tid * chunk;
  int c = 0;
  for (int s = s0; s < min(s0 + chunk, E); ++s)
    c += (s == 0 || (key[s] >> 12) != (key[s - 1] >> 12)) ? 1 : 0;
  csum[tid] = c;
  __syncthreads();
  if (tid < 64) {  // exclusive scan of the chunk counts by one wave
    constexpr int kPer = kTileThreads / 64;
    int v[kPer], tot = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) { v[u] = csum[tid * kPer + u]; tot += v[u]; }
    int inc = tot;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int w = __shfl_up(inc, o, 64);
      if (tid >= o) inc += w;
    }
    int run = inc - tot;
#pragma unroll
    for (int u = 0; u < kPer; ++u) { csum[tid * kPer + u] = run; run += v[u]; }
    if (tid == 63) {
      cnt[t] = inc;
      atomicMax(&grp_max[q], inc);
    }
  }
  __syncthreads();
  int uid = csum[tid] - 1;
  const int64_t ubase = ent_off[t];
  for (int s = s0; s < min(s0 + chunk, E); ++s) {
    const uint64_t kv = key[s];
    const int32_t j = (int32_t)(kv >> 12);
    if (s == 0 || j != (int32_t)(key[s - 1] >> 12)) {
      ++uid;
      uniq[ubase + uid] = j;
    }
    const int e = (int)(kv & 0xfff);
    const int r = row_of(e);
    slot[rbase[r] + (e - rloc[r])] = (uint16_t)uid;
  }
}

// uniq (at the entry offsets) -> tile_u (at the list offsets)
__global__ void __launch_bounds__(kTileThreads) k_tile_compact(const int64_t *__restrict__ ent_off,
                                                               const int64_t *__restrict__ u_off,
                                                               const int32_t *__restrict__ uniq,
                                                               int32_t *__restrict__ tile_u) {
  const int64_t t = blockIdx.x;
  const int64_t a = ent_off[t], b = u_off[t], m = u_off[t + 1] - b;
  for (int64_t s = threadIdx.x; s < m; s += kTileThreads) tile_u[b + s] = uniq[a + s];
}

// reverse-edge map: rev[k] = position of (j, i) in row j for entry k = (i, j)
// (binary search in the sorted row j); a team of kRevTeam lanes per row i
constexpr int kRevTeam = 8;
__global__ void __launch_bounds__(kBlock) k_rev(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                                int64_t n, int32_t *__restrict__ rev) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = gt / kRevTeam;
  if (i >= n) return;
  for (int64_t k = row_ptr[i] + gt % kRevTeam; k < row_ptr[i + 1]; k += kRevTeam) {
    const int32_t j = col[k];
    int64_t lo = row_ptr[j], hi = row_ptr[j + 1];
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (col[mid] < i) lo = mid + 1; else hi = mid;
    }
    rev[k] = (lo < row_ptr[j + 1] && col[lo] == i) ? (int32_t)lo : -1;
  }
}

int ceil_log2(int v) {
  int b = 0;
  while ((1 << b) < v) ++b;
  return b;
}

void free_nbr(gf_nbr *nb) {
  if (!nb) return;
  (void)hipSetDevice(nb->device);
  if (nb->row_ptr) (void)hipFree(nb->row_ptr);
  if (nb->col) (void)hipFree(nb->col);
  if (nb->order) (void)hipFree(nb->order);
  if (nb->grouped) (void)hipFree(nb->grouped);
  if (nb->rev) (void)hipFree(nb->rev);
  if (nb->slot) (void)hipFree(nb->slot);
  if (nb->tile_u) (void)hipFree(nb->tile_u);
  if (nb->tile_off) (void)hipFree(nb->tile_off);
  delete nb;
}

}  // namespace

extern "C" void gf_nbr_free(gf_nbr *nbr) { free_nbr(nbr); }

extern "C" gf_status gf_nbr_info(const gf_nbr *nbr, int64_t *n, int64_t *nnz, int32_t *max_row) {
  if (!nbr) return GF_EINVAL;
  if (n) *n = nbr->n;
  if (nnz) *nnz = nbr->nnz;
  if (max_row) *max_row = nbr->max_row;
  return GF_OK;
}

extern "C" gf_status gf_nbr_export(gf_ctx *ctx, const gf_nbr *nbr, int64_t *row_ptr, int32_t *col) {
  if (!ctx || !nbr) return GF_EINVAL;
  GF_HIP(ctx, hipSetDevice(ctx->device));
  if (row_ptr)
    GF_HIP(ctx, hipMemcpyAsync(row_ptr, nbr->row_ptr, sizeof(int64_t) * (nbr->n + 1), hipMemcpyDeviceToDevice, ctx->stream));
  if (col && nbr->nnz)
    GF_HIP(ctx, hipMemcpyAsync(col, nbr->col, sizeof(int32_t) * nbr->nnz, hipMemcpyDeviceToDevice, ctx->stream));
  return GF_OK;
}

gf_status ensure_rev(gf_ctx *ctx, gf_nbr *nbr) {
  if (nbr->rev) return GF_OK;
  if (nbr->nnz > (int64_t)0x7fffffff)
    return set_error(ctx, GF_ECAPACITY, "the reverse-edge map holds 32-bit positions; %lld entries exceed it",
                     (long long)nbr->nnz);
  if (hipMalloc(&nbr->rev, sizeof(int32_t) * std::max<int64_t>(nbr->nnz, 1)) != hipSuccess) {
    nbr->rev = nullptr;
    return set_error(ctx, GF_ENOMEM, "reverse-edge map allocation failed");
  }
  hipLaunchKernelGGL(k_rev, dim3(grid_for(nbr->n * kRevTeam, kBlock)), dim3(kBlock), 0, ctx->stream, nbr->row_ptr, nbr->col,
                     nbr->n, nbr->rev);
  GF_LAUNCH_CHECK(ctx);
  return GF_OK;
}

namespace {

// Cut the tiled groups into tiles and build slot[], tile_u[], tile_off[].
gf_status build_tiles(gf_ctx *ctx, gf_nbr *nb) {
  hipStream_t sm = ctx->stream;
  TileGroups tg;
  int64_t nt = 0;
  for (int m = 0; m < 2; ++m) {
    nb->tile_start[m] = nt;
    const int64_t r0 = nb->group_start[m * GF_NBAND], r1 = nb->group_start[m * GF_NBAND + kTileBand + 1];
    if (r1 <= r0) continue;
    tg.gsel[tg.nq] = m;
    tg.tile_start[tg.nq] = nt;
    tg.row_start[tg.nq] = r0;
    tg.nrows[tg.nq] = r1 - r0;
    ++tg.nq;
    nt += (r1 - r0 + kTileRows - 1) / kTileRows;
  }
  nb->tile_start[2] = nt;
  tg.tile_start[tg.nq] = nt;
  nb->ntiles = nt;
  if (nt == 0) return GF_OK;
  if (nt >= 0x7fffffff) return set_error(ctx, GF_ECAPACITY, "too many neighbour tiles");
  if (hipMalloc(&nb->slot, sizeof(uint16_t) * std::max<int64_t>(nb->nnz, 1)) != hipSuccess ||
      hipMalloc(&nb->tile_off, sizeof(int64_t) * (nt + 1)) != hipSuccess)
    return set_error(ctx, GF_ENOMEM, "neighbour tile allocation failed");
  Arena ar;
  std::vector<size_t> sz = {sizeof(int32_t) * nt, sizeof(int64_t) * (nt + 1), sizeof(int64_t) * scan_tmp_elems(nt + 1),
                            sizeof(int32_t) * std::max<int64_t>(nb->nnz, 1), sizeof(int32_t) * nt, 64};
  gf_status st;
  if ((st = ensure_scratch(ctx, arena_bytes(sz), &ar))) return st;
  int32_t *ent = ar.take<int32_t>(nt);
  int64_t *ent_off = ar.take<int64_t>(nt + 1);
  int64_t *tmp64 = ar.take<int64_t>(scan_tmp_elems(nt + 1));
  int32_t *uniq = ar.take<int32_t>(std::max<int64_t>(nb->nnz, 1));
  int32_t *cnt = ar.take<int32_t>(nt);
  int32_t *grp_max = ar.take<int32_t>(16);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, sm, grp_max, (int64_t)16, 0);
  hipLaunchKernelGGL(k_tile_entries, dim3(grid_for(nt, kBlock)), dim3(kBlock), 0, sm, tg, nb->row_ptr, nb->grouped,
                     ent);
  GF_LAUNCH_CHECK(ctx);
  if ((st = scan_i32_to_i64(ctx, ent, ent_off, nt, tmp64))) return st;
  hipLaunchKernelGGL(k_tile_unique, dim3((unsigned)nt), dim3(kTileThreads), 0, sm, tg, nb->row_ptr, nb->col,
                     nb->grouped, ent_off, nb->slot, uniq, cnt, grp_max);
  GF_LAUNCH_CHECK(ctx);
  if ((st = scan_i32_to_i64(ctx, cnt, nb->tile_off, nt, tmp64))) return st;
  if ((st = ensure_host(ctx, 4096))) return st;
  char *hp = (char *)ctx->host_pinned;
  GF_HIP(ctx, hipMemcpyAsync(hp, grp_max, sizeof(int32_t) * 16, hipMemcpyDeviceToHost, sm));
  GF_HIP(ctx, hipMemcpyAsync(hp + 128, nb->tile_off + nt, sizeof(int64_t), hipMemcpyDeviceToHost, sm));
  GF_HIP(ctx, hipStreamSynchronize(sm));
  for (int q = 0; q < tg.nq; ++q) nb->tile_max[tg.gsel[q]] = ((int32_t *)hp)[q];  // per model
  const int64_t total = *(int64_t *)(hp + 128);
  if (hipMalloc(&nb->tile_u, sizeof(int32_t) * std::max<int64_t>(total, 1)) != hipSuccess)
    return set_error(ctx, GF_ENOMEM, "neighbour tile list allocation failed");
  hipLaunchKernelGGL(k_tile_compact, dim3((unsigned)nt), dim3(kTileThreads), 0, sm, ent_off, nb->tile_off, uniq,
                     nb->tile_u);
  GF_LAUNCH_CHECK(ctx);
  return GF_OK;
}

}  // namespace

extern "C" gf_status gf_build_neighbours(gf_ctx *ctx, const gf_particles *p, int cross_model, gf_nbr **out) {
  if (!ctx) return GF_EINVAL;
  if (!p) return set_error(ctx, GF_EINVAL, "particles are NULL");
  return gf_build_neighbours_rows(ctx, p, cross_model, p->n, out);
}

extern "C" gf_status gf_build_neighbours_rows(gf_ctx *ctx, const gf_particles *p, int cross_model, int64_t n_rows,
                                              gf_nbr **out) {
  if (!ctx) return GF_EINVAL;
  if (!out) return set_error(ctx, GF_EINVAL, "out is NULL");
  *out = nullptr;
  gf_status st = check_particles(ctx, p, false, false);
  if (st) return st;
  const int64_t n = p->n;
  if (n_rows < 0 || n_rows > n)
    return set_error(ctx, GF_EINVAL, "n_rows = %lld outside [0, %lld]", (long long)n_rows, (long long)n);
  hipStream_t sm = ctx->stream;

  // ---- bounding boxes and validation
  const int nblk = (int)std::min<int64_t>(1024, (n + kBlock - 1) / kBlock);
  Arena ar;
  std::vector<size_t> sz = {sizeof(double) * kBoxVals * nblk, sizeof(int) * nblk, sizeof(double) * kBoxVals, 64};
  if ((st = ensure_scratch(ctx, arena_bytes(sz), &ar))) return st;
  double *part = ar.take<double>(kBoxVals * nblk);
  int *bad_part = ar.take<int>(nblk);
  double *box = ar.take<double>(kBoxVals);
  int *bad = ar.take<int>(16);
  hipLaunchKernelGGL(k_bbox, dim3(nblk), dim3(kBlock), 0, sm, p->x, p->y, p->z, p->h, p->model, n, part, bad_part);
  GF_LAUNCH_CHECK(ctx);
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(64), 0, sm, part, bad_part, nblk, box, bad);
  GF_LAUNCH_CHECK(ctx);
  if ((st = ensure_host(ctx, 4096))) return st;
  double *hbox = (double *)ctx->host_pinned;
  GF_HIP(ctx, hipMemcpyAsync(hbox, box, sizeof(double) * kBoxVals, hipMemcpyDeviceToHost, sm));
  GF_HIP(ctx, hipMemcpyAsync((char *)ctx->host_pinned + 256, bad, sizeof(int), hipMemcpyDeviceToHost, sm));
  GF_HIP(ctx, hipStreamSynchronize(sm));
  int nbad = *(int *)((char *)ctx->host_pinned + 256);
  if (nbad > 0)
    return set_error(ctx, GF_EINVAL, "%d particles have non-finite coordinates, h <= 0 or a model outside {0,1}", nbad);
  double bx[kBoxVals];
  memcpy(bx, hbox, sizeof(bx));

  // ---- grids (edge slightly above max h so that rounding of the cell
  // coordinate never hides a neighbour two cells away)
  Grid g;
  memset(&g, 0, sizeof(g));
  g.per_model = cross_model ? 0 : 1;
  double lo[2][3], hi[2][3], hmax[2];
  for (int m = 0; m < 2; ++m) {
    for (int d = 0; d < 3; ++d) { lo[m][d] = bx[m * 7 + d]; hi[m][d] = bx[m * 7 + 3 + d]; }
    hmax[m] = bx[m * 7 + 6];
  }
  if (!g.per_model) {  // merge into slot 0
    for (int d = 0; d < 3; ++d) {
      lo[0][d] = std::min(lo[0][d], lo[1][d]);
      hi[0][d] = std::max(hi[0][d], hi[1][d]);
    }
    hmax[0] = std::max(hmax[0], hmax[1]);
  }
  const int nslots = g.per_model ? 2 : 1;
  const int64_t key_budget = std::max<int64_t>(8 * n, 1 << 16);
  int64_t base = 0;
  for (int s = 0; s < nslots; ++s) {
    bool empty = !(hmax[s] > 0.0);
    double edge = empty ? 1.0 : hmax[s] * (1.0 + 1e-9);
    for (int it = 0; it < 200; ++it) {
      int tb = 0;
      for (int d = 0; d < 3; ++d) {
        double span = empty ? 0.0 : hi[s][d] - lo[s][d];
        double dd = std::floor(span / edge) + 1.0;
        if (dd > 1e6) dd = 1e6;
        g.dim[s][d] = (int)dd;
        g.bits[s][d] = ceil_log2(g.dim[s][d]);
        tb += g.bits[s][d];
      }
      if (tb <= 30 && ((int64_t)1 << tb) <= key_budget) break;
      edge *= 1.5;
    }
    for (int d = 0; d < 3; ++d) g.lo[s][d] = empty ? 0.0 : lo[s][d];
    g.inv_edge[s] = 1.0 / edge;
    g.base[s] = base;
    base += (int64_t)1 << (g.bits[s][0] + g.bits[s][1] + g.bits[s][2]);
  }
  g.nkeys = base;
  if (g.nkeys >= (int64_t)0x7fffffff) return set_error(ctx, GF_ECAPACITY, "cell grid too large");

  // ---- sort particles into cells
  const int64_t K = g.nkeys;
  sz = {sizeof(int32_t) * n, sizeof(int32_t) * n, sizeof(int32_t) * (K + 1), sizeof(int32_t) * scan_tmp_elems(K + 1),
        sizeof(double4) * n, sizeof(int32_t) * n, sizeof(int64_t) * scan_tmp_elems(n + 1), sizeof(int32_t) * 16,
        sizeof(int32_t) * n, sizeof(int32_t) * (n + 1), sizeof(int32_t) * scan_tmp_elems(n + 1)};
  if ((st = ensure_scratch(ctx, arena_bytes(sz), &ar))) return st;
  int32_t *key = ar.take<int32_t>(n);
  int32_t *slot = ar.take<int32_t>(n);
  int32_t *cell_start = ar.take<int32_t>(K + 1);
  int32_t *tmp32 = ar.take<int32_t>(scan_tmp_elems(K + 1));
  double4 *sp = ar.take<double4>(n);
  int32_t *cnt = ar.take<int32_t>(n);
  int64_t *tmp64 = ar.take<int64_t>(scan_tmp_elems(n + 1));
  int32_t *small = ar.take<int32_t>(16);  // hist[8], maxrow
  int32_t *gflag = ar.take<int32_t>(n);
  int32_t *gpos = ar.take<int32_t>(n + 1);
  int32_t *tmpg = ar.take<int32_t>(scan_tmp_elems(n + 1));

  gf_nbr *nb = new gf_nbr();
  nb->device = ctx->device;
  nb->n = n;
  nb->cross = cross_model ? 1 : 0;
  auto fail = [&](gf_status s2) { free_nbr(nb); return s2; };
  if (hipMalloc(&nb->row_ptr, sizeof(int64_t) * (n + 1)) != hipSuccess ||
      hipMalloc(&nb->order, sizeof(int32_t) * n) != hipSuccess ||
      hipMalloc(&nb->grouped, sizeof(int32_t) * n) != hipSuccess) {
    return fail(set_error(ctx, GF_ENOMEM, "neighbour handle allocation failed"));
  }

  {
  ProfScope prof_cells(ctx, "nbr_cells");
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(K + 1, kBlock)), dim3(kBlock), 0, sm, cell_start, K + 1, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, sm, small, (int64_t)16, 0);
  hipLaunchKernelGGL(k_keys, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, sm, p->x, p->y, p->z, p->model, n, g, key,
                     slot, cell_start);
  if (hipGetLastError() != hipSuccess) return fail(set_error(ctx, GF_EHIP, "key kernel launch failed"));
  if ((st = scan_i32_to_i32(ctx, cell_start, cell_start, K, tmp32))) return fail(st);
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, sm, key, slot, cell_start, n, nb->order);
  hipLaunchKernelGGL(k_cell_sort, dim3((unsigned)std::min<int64_t>(K, 65536)), dim3(64), 0, sm, cell_start, K, p->x,
                     p->y, p->z, p->model, g, nb->order);
  hipLaunchKernelGGL(k_gather_pos, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, sm, nb->order, p->x, p->y, p->z, p->h,
                     n, sp);
  }
  {
  ProfScope prof_count(ctx, "nbr_count");
  hipLaunchKernelGGL(k_search<0>, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, sm, nb->order, sp, p->model,
                     cell_start, n, n_rows, g, cnt, small, small + 8, (const int64_t *)nullptr, (int32_t *)nullptr);
  }
  if (hipGetLastError() != hipSuccess) return fail(set_error(ctx, GF_EHIP, "count kernel launch failed"));
  if ((st = scan_i32_to_i64(ctx, cnt, nb->row_ptr, n, tmp64))) return fail(st);
  int32_t *hsmall = (int32_t *)ctx->host_pinned;
  if (hipMemcpyAsync(hsmall, small, sizeof(int32_t) * 16, hipMemcpyDeviceToHost, sm) != hipSuccess ||
      hipMemcpyAsync((char *)ctx->host_pinned + 128, nb->row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, sm) !=
          hipSuccess ||
      hipStreamSynchronize(sm) != hipSuccess)
    return fail(set_error(ctx, GF_EHIP, "read-back of neighbour counts failed"));
  int32_t hist[2 * GF_NBAND];
  memcpy(hist, hsmall, sizeof(hist));
  // rows of the tiled bands are grouped together (under band kTileBand) so
  // that tiles stay spatially compact whatever the neighbour count
  for (int m = 0; m < 2; ++m)
    for (int band = 0; band < kTileBand; ++band) {
      hist[m * GF_NBAND + kTileBand] += hist[m * GF_NBAND + band];
      hist[m * GF_NBAND + band] = 0;
    }
  nb->max_row = hsmall[8];
  nb->nnz = *(int64_t *)((char *)ctx->host_pinned + 128);
  if (nb->max_row > kMaxRow)
    return fail(set_error(ctx, GF_ECAPACITY, "a particle has %d neighbours; the limit is %d", nb->max_row, kMaxRow));
  if (nb->nnz >= (int64_t)1 << 40) return fail(set_error(ctx, GF_ECAPACITY, "too many neighbour pairs"));
  if (hipMalloc(&nb->col, sizeof(int32_t) * std::max<int64_t>(nb->nnz, 1)) != hipSuccess)
    return fail(set_error(ctx, GF_ENOMEM, "neighbour list allocation (%lld entries) failed", (long long)nb->nnz));
  {
  ProfScope prof_fill(ctx, "nbr_fill");
  hipLaunchKernelGGL(k_search<1>, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, sm, nb->order, sp, p->model,
                     cell_start, n, n_rows, g, (int32_t *)nullptr, (int32_t *)nullptr, (int32_t *)nullptr, nb->row_ptr,
                     nb->col);
  }
  {
  ProfScope prof_sort(ctx, "nbr_row_sort");
  hipLaunchKernelGGL(k_row_sort, dim3((unsigned)n), dim3(64), 0, sm, nb->row_ptr, nb->col, n);
  }
  if (hipGetLastError() != hipSuccess) return fail(set_error(ctx, GF_EHIP, "fill/sort kernel launch failed"));

  // ---- groups by (model, band), Morton order kept inside each group
  ProfScope prof_group(ctx, "nbr_group_tiles");
  int64_t off = 0;
  for (int gsel = 0; gsel < 2 * GF_NBAND; ++gsel) {
    nb->group_start[gsel] = off;
    if (hist[gsel] == 0) continue;
    hipLaunchKernelGGL(k_group_flag, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, sm, nb->order, cnt, p->model, n,
                       gsel, gflag);
    if ((st = scan_i32_to_i32(ctx, gflag, gpos, n, tmpg))) return fail(st);
    hipLaunchKernelGGL(k_group_scatter, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, sm, nb->order, gflag, gpos, n,
                       off, nb->grouped);
    off += hist[gsel];
  }
  nb->group_start[2 * GF_NBAND] = off;
  if (hipGetLastError() != hipSuccess) return fail(set_error(ctx, GF_EHIP, "grouping kernels failed"));
  if (off != n) return fail(set_error(ctx, GF_EHIP, "internal error: grouping covers %lld of %lld", (long long)off,
                                      (long long)n));
  if ((st = build_tiles(ctx, nb))) return fail(st);
  *out = nb;
  return GF_OK;
}
