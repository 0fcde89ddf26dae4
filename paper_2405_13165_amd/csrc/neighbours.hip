// Neighbourhoods S_i of Eq. (Nbd) by cell lists over Morton-ordered cells.
//
// Pipeline (one stream, one host read-back of sizes):
//   bbox/validate -> grid of each particle (model, support level) and its
//   cell key + per-cell counts (atomics) -> scan -> scatter into cell order
//   -> list of non-empty cells -> finer Morton order inside cells ->
//   positions gathered in cell order -> per-cell search, count pass -> scan
//   -> fill pass -> per-row sort -> (several support levels: a second cell
//   pass over each model's finest grid, a model-wide Morton order) ->
//   grouping of particles by (model, neighbour-count band) for the batched
//   stencil kernels -> neighbour tiles.
// Each model has grids for up to four support levels (caps hmax, hmax/2,
// ...); a cell of a grid is a cube of edge slightly above its cap, and a row
// cell searches, in every grid of the requested models, the cells within
// (h_row + cap)/2 of its particles.
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

// orders the LDS traffic of the lanes of one wave
__device__ inline void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// per model: lo[3], hi[3], hmax, hmin (8 doubles) -> 16 doubles + invalid count
constexpr int kBoxVals = 16;
// value k of the box is reduced with min (else max)
__host__ __device__ inline bool box_is_min(int k) { return (k % 8) < 3 || (k % 8) == 7; }

__global__ void __launch_bounds__(kBlock) k_bbox(const double *__restrict__ x, const double *__restrict__ y,
                                                 const double *__restrict__ z, const double *__restrict__ h,
                                                 const int8_t *__restrict__ model, int64_t n,
                                                 double *__restrict__ part, int *__restrict__ bad_part) {
  double v[kBoxVals];
  for (int m = 0; m < 2; ++m) {
    for (int d = 0; d < 3; ++d) { v[m * 8 + d] = INFINITY; v[m * 8 + 3 + d] = -INFINITY; }
    v[m * 8 + 6] = 0.0;
    v[m * 8 + 7] = INFINITY;
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
        v[mm * 8 + d] = fmin(v[mm * 8 + d], p[d]);
        v[mm * 8 + 3 + d] = fmax(v[mm * 8 + 3 + d], p[d]);
      }
      v[mm * 8 + 6] = fmax(v[mm * 8 + 6], hi);
      v[mm * 8 + 7] = fmin(v[mm * 8 + 7], hi);
    }
  }
  __shared__ double sh[kBlock / 64][kBoxVals];
  __shared__ int shb[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = 0; k < kBoxVals; ++k) {
    double r = box_is_min(k) ? wave_min(v[k]) : wave_max(v[k]);
    if (lane == 0) sh[wid][k] = r;
  }
  int bs = wave_sum_i(bad);
  if (lane == 0) shb[wid] = bs;
  __syncthreads();
  if (threadIdx.x < kBoxVals) {
    int k = threadIdx.x;
    double r = sh[0][k];
    for (int w = 1; w < kBlock / 64; ++w) r = box_is_min(k) ? fmin(r, sh[w][k]) : fmax(r, sh[w][k]);
    part[(int64_t)blockIdx.x * kBoxVals + k] = r;
  }
  if (threadIdx.x == 0) {
    int b = 0;
    for (int w = 0; w < kBlock / 64; ++w) b += shb[w];
    bad_part[blockIdx.x] = b;
  }
}

// one block of kBboxFin threads: thread b takes block partial b (nblk <= kBboxFin)
constexpr int kBboxFin = 1024;
__global__ void __launch_bounds__(kBboxFin) k_bbox_final(const double *__restrict__ part,
                                                         const int *__restrict__ bad_part, int nblk,
                                                         double *__restrict__ out, int *__restrict__ bad_out) {
  __shared__ double sh[kBboxFin / 64][kBoxVals];
  __shared__ int shb[kBboxFin / 64];
  const int b = threadIdx.x, lane = b & 63, wid = b >> 6;
  const bool has = b < nblk;
  for (int k = 0; k < kBoxVals; ++k) {
    const bool lo = box_is_min(k);
    const double t = has ? part[(int64_t)b * kBoxVals + k] : (lo ? INFINITY : -INFINITY);
    const double r = lo ? wave_min(t) : wave_max(t);
    if (lane == 0) sh[wid][k] = r;
  }
  const int bs = wave_sum_i(has ? bad_part[b] : 0);
  if (lane == 0) shb[wid] = bs;
  __syncthreads();
  if (b < kBoxVals) {
    const bool lo = box_is_min(b);
    double r = sh[0][b];
    for (int w = 1; w < kBboxFin / 64; ++w) r = lo ? fmin(r, sh[w][b]) : fmax(r, sh[w][b]);
    out[b] = r;
  }
  if (b == 0) {
    int sum = 0;
    for (int w = 0; w < kBboxFin / 64; ++w) sum += shb[w];
    *bad_out = sum;
  }
}

// -------------------------------------------------------------- grid
// One cell grid per (model, level): level l of model m holds the particles
// with hmax_m 2^-(l+1) < h <= hmax_m 2^-l (the last level takes the rest),
// so a cell's edge follows the supports of its own particles.  A row cell
// searches, in each target grid, the cells within (h_row + hcap_target)/2 of
// its particles: uneven supports and dense fine regions do not inflate the
// candidate sets of the others.
constexpr int kMaxLevels = 4;
constexpr int kMaxSlots = 2 * kMaxLevels;
struct Grid {
  int nslots;
  int slot0[3];              // slots of model m: [slot0[m], slot0[m + 1])
  double lo[kMaxSlots][3];
  double inv_edge[kMaxSlots];
  double hcap[kMaxSlots];    // every particle of the slot has h <= hcap (0: model absent)
  int dim[kMaxSlots][3];
  int bits[kMaxSlots][3];
  int64_t base[kMaxSlots];   // key offset of each slot's cells
  int64_t nkeys;
};

__host__ __device__ inline int slot_of(const Grid &g, int m, double h) {
  int s = g.slot0[m];
  while (s + 1 < g.slot0[m + 1] && h <= g.hcap[s + 1]) ++s;
  return s;
}

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


__global__ void __launch_bounds__(kBlock) k_fill_i32(int32_t *a, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// key[i]: cell of particle i; counts[k]: particles per cell
__global__ void __launch_bounds__(kBlock) k_keys(const double *__restrict__ x, const double *__restrict__ y,
                                                 const double *__restrict__ z, const double *__restrict__ h,
                                                 const int8_t *__restrict__ model, int64_t n, Grid g,
                                                 int32_t *__restrict__ key, int32_t *__restrict__ slot,
                                                 int32_t *__restrict__ counts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = slot_of(g, model[i], h[i]);
  int cx = cell_of(x[i], g.lo[s][0], g.inv_edge[s], g.dim[s][0]);
  int cy = cell_of(y[i], g.lo[s][1], g.inv_edge[s], g.dim[s][1]);
  int cz = cell_of(z[i], g.lo[s][2], g.inv_edge[s], g.dim[s][2]);
  int32_t k = (int32_t)(g.base[s] + morton(cx, cy, cz, g.bits[s][0], g.bits[s][1], g.bits[s][2]));
  key[i] = k;
  // Slot within the cell.  Neighbouring particles mostly share a cell, and
  // 64 atomics on one counter serialise, so the lanes of the wave with the
  // same cell share one atomic: the lowest of them reserves their count and
  // each takes base + its rank among them.  (The order within a cell is
  // re-sorted later; only the set of slots 0..count-1 matters.)
  const int lane = threadIdx.x & 63;
  unsigned long long todo = __ballot(1);
  int32_t mine = 0;
  while (todo) {
    const int leader = __builtin_ctzll(todo);
    const int32_t lk = __shfl(k, leader, 64);
    const unsigned long long same = __ballot(k == lk) & todo;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(&counts[lk], (int32_t)__popcll(same));
    base = __shfl(base, leader, 64);
    if ((same >> lane) & 1ull) mine = base + (int32_t)__popcll(same & ((1ull << lane) - 1ull));
    todo &= ~same;
  }
  slot[i] = mine;
}

// particles per grid from the scanned cell counts (the cells of a grid are
// one key range; cell_start[nkeys] = n)
__global__ void k_slot_count(const int32_t *__restrict__ cell_start, Grid g, int32_t *__restrict__ slot_count) {
  const int q = threadIdx.x;
  if (q < g.nslots) {
    const int64_t e = (q + 1 < g.nslots) ? g.base[q + 1] : g.nkeys;
    slot_count[q] = cell_start[e] - cell_start[g.base[q]];
  }
}

__global__ void __launch_bounds__(kBlock) k_scatter(const int32_t *__restrict__ key, const int32_t *__restrict__ slot,
                                                    const int32_t *__restrict__ cell_start, int64_t n,
                                                    int32_t *__restrict__ order) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  order[cell_start[key[i]] + slot[i]] = (int32_t)i;
}

// non-empty cells: head[s] = 1 where sorted position s starts a cell
__global__ void __launch_bounds__(kBlock) k_cell_heads(const int32_t *__restrict__ order,
                                                       const int32_t *__restrict__ key, int64_t n,
                                                       int32_t *__restrict__ head) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  head[s] = (s == 0 || key[order[s]] != key[order[s - 1]]) ? 1 : 0;
}

__global__ void __launch_bounds__(kBlock) k_cell_list(const int32_t *__restrict__ head,
                                                      const int32_t *__restrict__ pos, int64_t n,
                                                      int32_t *__restrict__ cells) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  if (head[s]) cells[pos[s]] = (int32_t)s;
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

// cells[c]: first sorted position of the c-th non-empty cell; *ncells and
// the end n close the list
// Cells of up to kCellSortReg particles, one wave per cell, in registers.
// Inside a cell the fine keys differ only in their kSubBits low bits per axis
// (the interleaved low 3 * kSubBits bits), so (those bits, particle index)
// packed in 64 bits orders the cell exactly as the full comparison does.
constexpr int kCellSortReg = 64;
constexpr int kCellSortWaves = 4;
__global__ void __launch_bounds__(64 * kCellSortWaves) k_cell_sort_reg(
    const int32_t *__restrict__ cells, const int32_t *__restrict__ ncells, int64_t n, const double *__restrict__ x,
    const double *__restrict__ y, const double *__restrict__ z, const double *__restrict__ h,
    const int8_t *__restrict__ model, Grid g, int32_t *__restrict__ order) {
  const int lane = threadIdx.x & 63;
  const int32_t nc = *ncells;
  const int64_t stride = (int64_t)gridDim.x * kCellSortWaves;
  for (int64_t c = (int64_t)blockIdx.x * kCellSortWaves + (threadIdx.x >> 6); c < nc; c += stride) {
    const int32_t b = cells[c], len = (c + 1 < nc ? cells[c + 1] : (int32_t)n) - b;
    if (len <= 1 || len > kCellSortReg) continue;
    uint64_t v = ~0ull;
    if (lane < len) {
      const int32_t i = order[b + lane];
      const uint64_t sub = fine_key(x[i], y[i], z[i], g, slot_of(g, model[i], h[i])) & ((1ull << (3 * kSubBits)) - 1);
      v = (sub << 32) | (uint32_t)i;
    }
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
        const uint64_t p = __shfl_xor(v, j, 64);
        const bool up = (lane & k) == 0, lower = (lane & j) == 0;
        v = (lower == up) ? (v < p ? v : p) : (v < p ? p : v);
      }
    }
    if (lane < len) order[b + lane] = (int32_t)(uint32_t)v;
  }
}

__global__ void __launch_bounds__(64) k_cell_sort(const int32_t *__restrict__ cells, const int32_t *__restrict__ ncells,
                                                  int64_t n, const double *__restrict__ x,
                                                  const double *__restrict__ y, const double *__restrict__ z,
                                                  const double *__restrict__ h, const int8_t *__restrict__ model,
                                                  Grid g, int32_t *__restrict__ order) {
  __shared__ uint64_t kk[kCellSort];
  __shared__ int32_t id[kCellSort];
  const int32_t nc = *ncells;
  for (int64_t c = blockIdx.x; c < nc; c += gridDim.x) {
    const int32_t b = cells[c], len = (c + 1 < nc ? cells[c + 1] : (int32_t)n) - b;
    if (len <= kCellSortReg || len > kCellSort) continue;  // small cells: k_cell_sort_reg
    int P = 1;
    while (P < len) P <<= 1;
    for (int t = threadIdx.x; t < P; t += 64) {
      if (t < len) {
        const int32_t i = order[b + t];
        kk[t] = fine_key(x[i], y[i], z[i], g, slot_of(g, model[i], h[i]));
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

// Neighbour search, one wave per non-empty cell (waves take the next cell from
// a queue counter: bulk and film cells differ in cost), its rows in groups of
// up to 64.  For each target grid (the row
// model's grids, or all grids for cross-model sets) the cells within
// R = (max h of the rows + hcap of the grid)/2 of the rows are taken 64 at a
// time; their particles, numbered through a prefix sum of the cell ranges,
// are tested 64 at a time (one per lane) against each row, and a ballot gives
// the row's hits.  MODE 0: count (cnt[i] = |S_i|, group histogram, max row);
// MODE 1: fill col (each row in candidate order; rows are sorted afterwards).
// Both passes visit candidates in the same order, so the fill ends exactly at
// the counted length.  With `stage`, the count pass also writes each row's
// first sw hits to stage[i * sw ...] (sw, the stage width, 512 or 256 hits
// by the memory it takes), which saves the fill pass when no row is longer;
// with `stage` the fill pass writes only the longer rows (and skips the groups
// of rows without one).  Particles i >= n_rows (ghost particles) appear in the
// rows of others but their own row holds only i.
constexpr int kSearchBlock = 256;
constexpr int kSearchWaves = kSearchBlock / 64;
// occupancy the search kernels are compiled for: five waves per SIMD leave
// them the registers they use unconstrained (88); asking for six squeezes
// them into 80 and runs them 15% slower
constexpr int kSearchWavesPerSimd = 5;
constexpr int kQueueGrab = 4;           // cells a wave takes from the queue at once
constexpr int kStageWidths[2] = {512, 256};  // hits per row the count pass may stage, widest first

// the value of v in lane r (r the same in every lane)
__device__ inline int64_t readlane64(int64_t v, int r) {
  return ((int64_t)__builtin_amdgcn_readlane((int)(v >> 32), r) << 32) |
         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, r);
}

// a value known to be the same in every lane, moved to scalar registers
__device__ inline double uniform_f64(double v) {
  const int64_t b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)b);
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

template <int MODE>
__global__ void __launch_bounds__(kSearchBlock) __attribute__((amdgpu_waves_per_eu(kSearchWavesPerSimd))) k_search(const int32_t *__restrict__ order,
                                                         const double4 *__restrict__ sp,
                                                         const int8_t *__restrict__ model,
                                                         const int32_t *__restrict__ cell_start,
                                                         const int32_t *__restrict__ cells,
                                                         const int32_t *__restrict__ ncells,
                                                         const int32_t *__restrict__ slot_count,
                                                         int32_t *__restrict__ queue, int64_t n,
                                                         int64_t n_rows, Grid g, int cross,
                                                         int32_t *__restrict__ cnt, int32_t *__restrict__ hist,
                                                         int32_t *__restrict__ maxrow,
                                                         const int64_t *__restrict__ row_ptr,
                                                         int32_t *__restrict__ col, int32_t *__restrict__ stage,
                                                         int sw) {
  __shared__ int32_t s_rb[kSearchWaves][64];    // first sorted position of each cell of the batch
  __shared__ int32_t s_pref[kSearchWaves][65];  // candidates before each cell of the batch
  __shared__ double4 s_row[kSearchWaves][64];   // positions of the current row group
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int32_t nc = *ncells;
  int hist_local = 0;  // lane b < 2*GF_NBAND: rows counted in bin b (MODE 0)
  int max_local = 0;
  int32_t grab = 0, left = 0;
  while (true) {
    if (left == 0) {  // kQueueGrab cells per queue access
      int32_t next = 0;
      if (lane == 0) next = atomicAdd(queue, kQueueGrab);
      grab = __builtin_amdgcn_readfirstlane(next);
      left = kQueueGrab;
    }
    const int32_t ci = grab + (kQueueGrab - left);
    --left;
    if (ci >= nc) break;
    const int32_t c0 = cells[ci];
    const int32_t c1 = (ci + 1 < nc) ? cells[ci + 1] : (int32_t)n;
    const int mrow = model[order[c0]];
    const int t0 = cross ? 0 : g.slot0[mrow], t1 = cross ? g.nslots : g.slot0[mrow + 1];
    for (int32_t rg = c0; rg < c1; rg += 64) {
      const int nr = min(64, c1 - rg);
      int32_t myi = -1;
      bool ghost = false;
      int64_t myoff = 0;
      int mylen = 0;  // MODE 1: the row's CSR length (bounds every write)
      double4 me = make_double4(0.0, 0.0, 0.0, 0.0);
      if (lane < nr) {
        myi = order[rg + lane];
        me = sp[rg + lane];
        s_row[w][lane] = me;
        ghost = myi >= n_rows;
        if (MODE == 1) {
          myoff = row_ptr[myi];
          mylen = (int)(row_ptr[myi + 1] - myoff);
          if (stage && mylen <= sw) mylen = 0;  // staged by the count pass: not written here
          if (ghost && mylen > 0) col[myoff] = myi;
        } else if (stage) {
          myoff = (int64_t)myi * sw;
          mylen = sw;
          if (ghost) stage[myoff] = myi;
        }
      }
      if (MODE == 1 && stage && __ballot(mylen > 0) == 0) continue;  // no row of the group to fill
      const bool act = lane < nr && !ghost;
      const double bx0 = uniform_f64(wave_min(act ? me.x : INFINITY));
      const double bx1 = uniform_f64(wave_max(act ? me.x : -INFINITY));
      const double by0 = uniform_f64(wave_min(act ? me.y : INFINITY));
      const double by1 = uniform_f64(wave_max(act ? me.y : -INFINITY));
      const double bz0 = uniform_f64(wave_min(act ? me.z : INFINITY));
      const double bz1 = uniform_f64(wave_max(act ? me.z : -INFINITY));
      const double hrow = uniform_f64(wave_max(act ? me.w : 0.0));
      const uint64_t ghosts = __ballot(ghost);
      wave_fence();
      int run = 0;  // lane r < nr: hits of row r so far
      for (int ts = t0; ts < t1; ++ts) {
        if (hrow <= 0.0 || slot_count[ts] == 0) continue;  // no searching row, or an empty grid
        // cells within R of the rows (1e-6 margin against rounding of the cell coordinates)
        const double R = 0.5 * (hrow + g.hcap[ts]) * (1.0 + 1e-6);
        const double b0[3] = {bx0, by0, bz0}, b1[3] = {bx1, by1, bz1};
        int a0[3], ext[3];
        bool none = false;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const double f0 = floor((b0[d] - R - g.lo[ts][d]) * g.inv_edge[ts]);
          const double f1 = floor((b1[d] + R - g.lo[ts][d]) * g.inv_edge[ts]);
          const double top = (double)(g.dim[ts][d] - 1);
          none = none || f1 < 0.0 || f0 > top;
          a0[d] = __builtin_amdgcn_readfirstlane((int)fmax(f0, 0.0));
          ext[d] = __builtin_amdgcn_readfirstlane((int)fmin(f1, top)) - a0[d] + 1;
        }
        if (none) continue;
        const int64_t nbox = (int64_t)ext[0] * ext[1] * ext[2];
        for (int64_t kb = 0; kb < nbox; kb += 64) {
          int len = 0, rb = 0;
          const int64_t kc = kb + lane;
          if (kc < nbox) {
            const int ix = (int)(kc % ext[0]), iy = (int)((kc / ext[0]) % ext[1]), iz = (int)(kc / ((int64_t)ext[0] * ext[1]));
            const int64_t key = g.base[ts] + morton(a0[0] + ix, a0[1] + iy, a0[2] + iz, g.bits[ts][0], g.bits[ts][1],
                                                    g.bits[ts][2]);
            rb = cell_start[key];
            len = cell_start[key + 1] - rb;
          }
          int inc = len;
#pragma unroll
          for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(inc, o, 64);
            if (lane >= o) inc += v;
          }
          s_rb[w][lane] = rb;
          s_pref[w][lane + 1] = inc;
          if (lane == 0) s_pref[w][0] = 0;
          wave_fence();
          const int C = __shfl(inc, 63, 64);
          // candidate c's sorted position (c < C): its cell is the largest k
          // with s_pref[k] <= c
          auto cand = [&](int c) {
            int k = 0;
#pragma unroll
            for (int step = 32; step > 0; step >>= 1)
              if (k + step < 64 && s_pref[w][k + step] <= c) k += step;
            return s_rb[w][k] + (c - s_pref[w][k]);
          };
          // the next batch's candidates are requested while this batch is tested
          double4 qn = make_double4(0.0, 0.0, 0.0, 0.0);
          int32_t qjn = 0;
          if (lane < C) {
            const int32_t t = cand(lane);
            qn = sp[t];
            if (MODE == 1 || stage) qjn = order[t];
          }
          for (int cb = 0; cb < C; cb += 64) {
            const int c = cb + lane;
            const bool cv = c < C;
            const double4 q = qn;
            const int32_t qj = qjn;
            if (c + 64 < C) {
              const int32_t t = cand(c + 64);
              qn = sp[t];
              if (MODE == 1 || stage) qjn = order[t];
            }
            // two rows per step: independent chains for the FP64 pipeline
            for (int r = 0; r < nr; r += 2) {
              const int r2 = min(r + 1, nr - 1);  // == r when r is the last row
              const double4 pa = s_row[w][r], pb = s_row[w][r2];
              const bool ha = cv && !((ghosts >> r) & 1) && in_support(pa, q);
              const bool hb = r2 != r && cv && !((ghosts >> r2) & 1) && in_support(pb, q);
              const uint64_t ma = __ballot(ha), mb = __ballot(hb);
              if (MODE == 1 || stage) {
                // each row's fill position and output offset, read from its lane (uniform)
                const int run_a = __builtin_amdgcn_readlane(run, r), run_b = __builtin_amdgcn_readlane(run, r2);
                const int64_t off_a = readlane64(myoff, r), off_b = readlane64(myoff, r2);
                const int bef_a = __builtin_amdgcn_mbcnt_hi((uint32_t)(ma >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ma, 0));
                const int bef_b = __builtin_amdgcn_mbcnt_hi((uint32_t)(mb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mb, 0));
                const int pos_a = run_a + bef_a, pos_b = run_b + bef_b;
                int32_t *out = MODE == 1 ? col : stage;
                if (ha && pos_a < __builtin_amdgcn_readlane(mylen, r)) out[off_a + pos_a] = qj;
                if (hb && pos_b < __builtin_amdgcn_readlane(mylen, r2)) out[off_b + pos_b] = qj;
              }
              if (lane == r) run += __popcll(ma);
              if (r2 != r && lane == r2) run += __popcll(mb);
            }
          }
          wave_fence();
        }
      }
      if (MODE == 0) {
        int bin = -1;
        if (lane < nr) {
          const int cc = ghost ? 1 : run;
          cnt[myi] = cc;
          int band = 0;
          while (band < GF_NBAND - 1 && cc > kBandHi[band]) ++band;
          bin = model[myi] * GF_NBAND + band;
          max_local = max(max_local, cc);
        }
        // per-wave histogram, all lanes active: lane b counts bin b
#pragma unroll
        for (int b = 0; b < 2 * GF_NBAND; ++b) {
          const int hb = __popcll(__ballot(bin == b));
          if (lane == b) hist_local += hb;
        }
      }
      wave_fence();
    }
  }
  if (MODE == 0) {
    if (lane < 2 * GF_NBAND && hist_local) atomicAdd(&hist[lane], hist_local);
    int cm = max_local;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cm = max(cm, __shfl_xor(cm, o, 64));
    if (lane == 0 && cm) atomicMax(maxrow, cm);
  }
}

// Sort each row ascending.  One wave per chunk of 64 rows (grid-stride over
// chunks), the chunk's row offsets one per lane.  A row of up to 128 entries
// is sorted in registers by a bitonic network of P = the next power of two
// >= its length: lane l holds positions l and l + 64; exchanges at distance
// 64 stay in the lane, shorter ones go through cross-lane shuffles.  The
// next row's entries are loaded while the current one is sorted.  Rows with
// more than 128 entries (LONG launches only) use a wave-private LDS buffer.
constexpr int kSortBlock = 256;
constexpr int kSortWaves = kSortBlock / 64;

// v of lane `lane ^ j` (j a power of two up to 32, a constant once the
// networks are unrolled), without the LDS crossbar where a lane move does it:
// j = 1, 2 by a DPP quad permutation, j = 4, 8 by the two DPP row shifts and a
// select (a lane with bit j clear reads lane + j, one with it set lane - j,
// both in its row of 16), j = 16 by a swizzle within 32 lanes (bitmask mode,
// xor 16), j = 32 by a permute.  Every lane of the wave is active here.
__device__ __forceinline__ int32_t xor_lane(int32_t v, int j, int lane) {
  switch (j) {
    case 1: return __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false);  // quad_perm [1, 0, 3, 2]
    case 2: return __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false);  // quad_perm [2, 3, 0, 1]
    case 4: {
      const int32_t up = __builtin_amdgcn_update_dpp(v, v, 0x104, 0xF, 0xF, false);  // row_shl:4
      const int32_t dn = __builtin_amdgcn_update_dpp(v, v, 0x114, 0xF, 0xF, false);  // row_shr:4
      return (lane & 4) ? dn : up;
    }
    case 8: {
      const int32_t up = __builtin_amdgcn_update_dpp(v, v, 0x108, 0xF, 0xF, false);  // row_shl:8
      const int32_t dn = __builtin_amdgcn_update_dpp(v, v, 0x118, 0xF, 0xF, false);  // row_shr:8
      return (lane & 8) ? dn : up;
    }
    case 16: return __builtin_amdgcn_ds_swizzle(v, (16 << 10) | 0x1F);
    default: return __shfl_xor(v, j, 64);
  }
}

__device__ inline int32_t bitonic_pick(int32_t v, int32_t partner, int t, int j, int k) {
  const bool up = (t & k) == 0;     // direction of this k-sequence
  const bool lower = (t & j) == 0;  // t is the smaller position of its pair
  return (lower == up) ? min(v, partner) : max(v, partner);
}

// the bitonic network for P (power of two, <= 128) elements, unrolled
template <int P>
__device__ inline void sort_net(int32_t &v0, int32_t &v1, int lane) {
#pragma unroll
  for (int k = 2; k <= P; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j == 64) {
        const int32_t lo = min(v0, v1), hi = max(v0, v1);
        v0 = lo;
        v1 = hi;
      } else {
        v0 = bitonic_pick(v0, xor_lane(v0, j, lane), lane, j, k);
        if (P > 64) v1 = bitonic_pick(v1, xor_lane(v1, j, lane), lane + 64, j, k);
      }
    }
  }
}

// the bitonic network for 256 elements, four per lane (position lane + 64 r
// in v[r]): distances 128 and 64 compare registers of one lane, shorter ones
// exchange through the wave
__device__ inline void sort_net256(int32_t v[4], int lane) {
  auto cx = [](int32_t &a, int32_t &b, int t, int k) {  // a at position t, b at t + distance
    const bool up = (t & k) == 0;
    const int32_t lo = min(a, b), hi = max(a, b);
    a = up ? lo : hi;
    b = up ? hi : lo;
  };
#pragma unroll
  for (int k = 2; k <= 256; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j == 128) {
        cx(v[0], v[2], lane, k);
        cx(v[1], v[3], lane + 64, k);
      } else if (j == 64) {
        cx(v[0], v[1], lane, k);
        cx(v[2], v[3], lane + 128, k);
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = bitonic_pick(v[r], xor_lane(v[r], j, lane), lane + 64 * r, j, k);
      }
    }
  }
}

// STAGED: a row of at most sw entries is read from stage[i * sw ...]
// (the count pass's copy) and written, sorted, to its CSR place; a longer row
// (filled by the fill pass), or every row without STAGED, is sorted in place.
template <bool LONG, bool STAGED>
__global__ void __launch_bounds__(kSortBlock) k_row_sort(const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col,
                                                         const int32_t *__restrict__ stage, int sw, int64_t n) {
  extern __shared__ int32_t sort_buf[];  // LONG: kSortWaves x kMaxRow
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t nchunks = (n + 63) / 64;
  for (int64_t ch = (int64_t)blockIdx.x * kSortWaves + w; ch < nchunks; ch += (int64_t)gridDim.x * kSortWaves) {
    const int64_t i0 = ch * 64;
    const int nr = (int)min((int64_t)64, n - i0);
    int64_t rb = 0;
    int rl = 0;
    if (lane < nr) {
      rb = row_ptr[i0 + lane];
      rl = (int)(row_ptr[i0 + lane + 1] - rb);
    }
    auto src = [&](int r) -> const int32_t * {
      if (STAGED && __builtin_amdgcn_readlane(rl, r) <= sw) return stage + (i0 + r) * (int64_t)sw;
      return col + readlane64(rb, r);
    };
    // rows of up to kRegRow entries are held in registers (NV per lane)
    constexpr int NV = LONG ? 4 : 2;
    constexpr int kRegRow = 64 * NV;
    auto fetch = [&](int r, int32_t a[NV]) {
      const int32_t *sr = src(r);
      const int len = __builtin_amdgcn_readlane(rl, r);
#pragma unroll
      for (int q = 0; q < NV; ++q) a[q] = (len <= kRegRow && lane + 64 * q < len) ? sr[lane + 64 * q] : 0x7fffffff;
    };
    int32_t v[NV];
    fetch(0, v);
    for (int r = 0; r < nr; ++r) {
      const int64_t b = readlane64(rb, r);
      const int len = __builtin_amdgcn_readlane(rl, r);
      int32_t nx[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) nx[q] = 0x7fffffff;
      if (r + 1 < nr) fetch(r + 1, nx);
      if (STAGED && len == 1) {
        if (lane == 0) col[b] = v[0];
      } else if (len > 1 && len <= 128) {
        if (len <= 8) sort_net<8>(v[0], v[1], lane);
        else if (len <= 16) sort_net<16>(v[0], v[1], lane);
        else if (len <= 32) sort_net<32>(v[0], v[1], lane);
        else if (len <= 64) sort_net<64>(v[0], v[1], lane);
        else sort_net<128>(v[0], v[1], lane);
        if (lane < len) col[b + lane] = v[0];
        if (lane + 64 < len) col[b + lane + 64] = v[1];
      } else if (LONG && len > 128 && len <= kRegRow) {
        if constexpr (LONG) {
          sort_net256(v, lane);
#pragma unroll
          for (int q = 0; q < NV; ++q)
            if (lane + 64 * q < len) col[b + lane + 64 * q] = v[q];
        }
      } else if (LONG && len > kRegRow) {
        int32_t *bw = sort_buf + w * kMaxRow;
        const int32_t *sr = src(r);
        int P = 1;
        while (P < len) P <<= 1;
        for (int t = lane; t < P; t += 64) bw[t] = (t < len) ? sr[t] : 0x7fffffff;
        wave_fence();
        for (int k = 2; k <= P; k <<= 1) {
          for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < P; t += 64) {
              const int u = t ^ j;
              if (u > t) {
                const int32_t a = bw[t], c = bw[u];
                if ((a > c) == ((t & k) == 0)) { bw[t] = c; bw[u] = a; }
              }
            }
            wave_fence();
          }
        }
        for (int t = lane; t < len; t += 64) col[b + t] = bw[t];
        wave_fence();
      }
#pragma unroll
      for (int q = 0; q < NV; ++q) v[q] = nx[q];
    }
  }
}

// grouping: particles (in the given order) of group gsel, stable; the tiled
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

// One block per tile.  The tile's distinct indices go into an LDS hash set
// (open addressing, linear probing); a new key also takes the next place in
// ulist (one counter update per wave) and records where it sits in the
// table.  The distinct indices are ranked by counting (rank = number of
// smaller distinct indices), each rank is kept beside its key, the sorted list
// is written to uniq[ent_off[t] ...], and each entry's slot is the rank of its
// index, read at the table position its insertion found; cnt[t] = number of
// distinct indices.  Each wave takes whole rows (w, w + 8, ...), a lane at
// most two entries of each (rows hold at most kTileBandRow = 128 entries):
// its column indices are all requested at once and stay in registers, with
// their table positions, until the slots are written.  The result does not
// depend on the order of the insertions.
constexpr int kHashBits = 12;
constexpr int kHashSize = 1 << kHashBits;  // >= kTileEntries >= distinct keys: every probe ends
static_assert(kHashSize >= kTileEntries, "the hash set must hold every entry of a tile");

__device__ inline int hash_slot(int32_t j) { return (int)(((uint32_t)j * 2654435761u) >> (32 - kHashBits)); }

__global__ void __launch_bounds__(kTileThreads) k_tile_unique(TileGroups tg, const int64_t *__restrict__ row_ptr,
                                                              const int32_t *__restrict__ col,
                                                              const int32_t *__restrict__ grouped,
                                                              const int64_t *__restrict__ ent_off,
                                                              uint16_t *__restrict__ slot,
                                                              int32_t *__restrict__ uniq, int32_t *__restrict__ cnt,
                                                              int32_t *__restrict__ grp_max) {
  constexpr int NW = kTileThreads / 64;
  __shared__ int32_t hkey[kHashSize];
  __shared__ uint16_t hrank[kHashSize];
  __shared__ __attribute__((aligned(16))) int32_t ulist[kTileEntries];  // distinct indices, then sorted
  __shared__ uint16_t upos[kTileEntries];                                // table position of ulist[s]
  __shared__ int64_t rbase[kTileRows];
  __shared__ int32_t rlen[kTileRows];
  __shared__ int32_t ucount;
  const int64_t t = blockIdx.x;
  const int q = tile_group(tg, t);
  const int64_t r0 = (t - tg.tile_start[q]) * kTileRows;
  const int R = (int)min((int64_t)kTileRows, tg.nrows[q] - r0);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (tid < R) {
    const int32_t i = grouped[tg.row_start[q] + r0 + tid];
    rbase[tid] = row_ptr[i];
    rlen[tid] = (int)(row_ptr[i + 1] - row_ptr[i]);  // <= kTileBandRow: tiled rows
  }
  for (int h = tid; h < kHashSize; h += kTileThreads) hkey[h] = -1;
  if (tid == 0) ucount = 0;
  __syncthreads();
  // 1. distinct indices; entry c of a lane: row wave + NW (c / 2), entry lane + 64 (c % 2)
  static_assert(kTileRows == 4 * NW && kTileBandRow == 128, "four rows per wave, two entries per lane and row");
  constexpr int kC = 8;
  int32_t jj[kC];
  int hh[kC];
#pragma unroll
  for (int c = 0; c < kC; ++c) {
    const int r = wave + NW * (c >> 1), e = lane + 64 * (c & 1);
    jj[c] = (r < R && e < rlen[r]) ? col[rbase[r] + e] : -1;
  }
#pragma unroll
  for (int c = 0; c < kC; ++c) {
    {
      const int32_t j = jj[c];
      bool fresh = false;
      int h = 0;
      if (j >= 0) {
        h = hash_slot(j);
        while (true) {
          const int32_t prev = atomicCAS(&hkey[h], -1, j);
          if (prev == -1) {
            fresh = true;
            break;
          }
          if (prev == j) break;
          h = (h + 1) & (kHashSize - 1);
        }
      }
      hh[c] = h;
      const uint64_t m = __ballot(fresh);
      int ub = 0;
      if (lane == 0 && m) ub = atomicAdd(&ucount, __popcll(m));
      ub = __shfl(ub, 0, 64);
      if (fresh) {
        const int s = ub + __popcll(m & ((1ull << lane) - 1));
        ulist[s] = j;
        upos[s] = (uint16_t)h;
      }
    }
  }
  __syncthreads();
  const int U = ucount;
  // 2. rank of each distinct index = number of smaller distinct indices; the
  // list is read four at a time (padded to a multiple of four), every lane
  // of a wave reading the same address (an LDS broadcast).  The ranks go
  // beside the keys, and (after a barrier) the list is sorted in place.
  const int U4 = (U + 3) & ~3;
  for (int s = U + tid; s < U4; s += kTileThreads) ulist[s] = 0x7fffffff;
  __syncthreads();
  constexpr int kPer = kTileEntries / kTileThreads;
  int32_t vv[kPer];
  int rr[kPer];
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int s = tid + c * kTileThreads;
    rr[c] = -1;
    vv[c] = 0;
    if (s < U) {
      const int32_t v = ulist[s];
      int r = 0;
      const int4 *l4 = reinterpret_cast<const int4 *>(ulist);
      for (int c4 = 0; c4 < U4 / 4; ++c4) {
        const int4 w4 = l4[c4];
        r += (w4.x < v) + (w4.y < v) + (w4.z < v) + (w4.w < v);
      }
      vv[c] = v;
      rr[c] = r;
      hrank[upos[s]] = (uint16_t)r;
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < kPer; ++c)
    if (rr[c] >= 0) ulist[rr[c]] = vv[c];
  __syncthreads();
  // 3. the sorted distinct indices
  const int64_t ubase = ent_off[t];
  for (int s = tid; s < U; s += kTileThreads) uniq[ubase + s] = ulist[s];
  if (tid == 0) {
    cnt[t] = U;
    atomicMax(&grp_max[q], U);
  }
  // 4. slots: the rank kept beside each entry's index
#pragma unroll
  for (int c = 0; c < kC; ++c)
    if (jj[c] >= 0) {
      const int r = wave + NW * (c >> 1), e = lane + 64 * (c & 1);
      slot[rbase[r] + e] = hrank[hh[c]];
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
// (binary search in the sorted row j, -1 if i is not listed there); a team of
// kRevTeam lanes per row i, each lane running the searches of kRevU entries
// side by side, so that every step requests kRevU independent loads (a lone
// search waits for each of its ~log2 |S_j| steps in turn)
constexpr int kRevTeam = 8;
constexpr int kRevU = 4;
__global__ void __launch_bounds__(kBlock) k_rev(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                                int64_t n, int32_t *__restrict__ rev) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = gt / kRevTeam;
  if (i >= n) return;
  const int64_t b = row_ptr[i], e = row_ptr[i + 1];
  for (int64_t kb = b + gt % kRevTeam; kb < e; kb += kRevU * kRevTeam) {
    // entries past the row's end search for its last entry's twin and store nothing; a finished
    // search reads entry kb (in the row) so that no load is skipped
    int32_t jj[kRevU];
#pragma unroll
    for (int u = 0; u < kRevU; ++u) jj[u] = col[min(kb + u * kRevTeam, e - 1)];
    int64_t lo[kRevU], hi[kRevU], end[kRevU];
#pragma unroll
    for (int u = 0; u < kRevU; ++u) {
      lo[u] = row_ptr[jj[u]];
      hi[u] = end[u] = row_ptr[jj[u] + 1];
    }
    bool act = true;
    while (act) {
      int64_t mid[kRevU];
      int32_t v[kRevU];
#pragma unroll
      for (int u = 0; u < kRevU; ++u) {
        mid[u] = (lo[u] + hi[u]) >> 1;
        v[u] = col[lo[u] < hi[u] ? mid[u] : kb];
      }
      act = false;
#pragma unroll
      for (int u = 0; u < kRevU; ++u) {
        if (lo[u] < hi[u]) {
          if (v[u] < i) lo[u] = mid[u] + 1;
          else hi[u] = mid[u];
        }
        act |= lo[u] < hi[u];
      }
    }
    int32_t c[kRevU];
#pragma unroll
    for (int u = 0; u < kRevU; ++u) c[u] = col[lo[u] < end[u] ? lo[u] : kb];
#pragma unroll
    for (int u = 0; u < kRevU; ++u)
      if (kb + u * kRevTeam < e) rev[kb + u * kRevTeam] = (lo[u] < end[u] && c[u] == i) ? (int32_t)lo[u] : -1;
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
  if (nb->grow_ptr) (void)hipFree(nb->grow_ptr);
  if (nb->gpos) (void)hipFree(nb->gpos);
  if (nb->grev) (void)hipFree(nb->grev);
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

extern "C" gf_status gf_nbr_view(const gf_nbr *nbr, int64_t *nnz, const int64_t **row_ptr, const int32_t **col) {
  if (!nbr) return GF_EINVAL;
  if (nnz) *nnz = nbr->nnz;
  if (row_ptr) *row_ptr = nbr->row_ptr;
  if (col) *col = nbr->col;
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
__global__ void __launch_bounds__(kBlock) k_grouped_len(const int32_t *__restrict__ grouped,
                                                        const int64_t *__restrict__ row_ptr, int64_t n,
                                                        int32_t *__restrict__ len, int32_t *__restrict__ gpos) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int32_t i = grouped[t];
  len[t] = (int32_t)(row_ptr[i + 1] - row_ptr[i]);
  gpos[i] = (int32_t)t;
}
// grev for the rows in grouped order, a team of kRevTeam lanes per row
__global__ void __launch_bounds__(kBlock) k_grouped_rev(const int32_t *__restrict__ grouped,
                                                        const int64_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col,
                                                        const int32_t *__restrict__ rev,
                                                        const int64_t *__restrict__ grow_ptr,
                                                        const int32_t *__restrict__ gpos, int64_t n,
                                                        int32_t *__restrict__ grev) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t t = gt / kRevTeam;
  const int lane = (int)(gt % kRevTeam);
  if (t >= n) return;
  const int32_t i = grouped[t];
  const int64_t b = row_ptr[i], len = row_ptr[i + 1] - b, ob = grow_ptr[t];
  for (int64_t o = lane; o < len; o += kRevTeam) {
    const int32_t j = col[b + o];
    const int32_t kr = rev[b + o];
    grev[ob + o] = (j == i || kr < 0) ? -1 : (int32_t)(grow_ptr[gpos[j]] + (kr - row_ptr[j]));
  }
}
}  // namespace

gf_status ensure_grouped_rows(gf_ctx *ctx, gf_nbr *nbr) {
  if (nbr->grev) return GF_OK;
  gf_status st = ensure_rev(ctx, nbr);  // also checks that positions fit 32 bits
  if (st) return st;
  const int64_t n = nbr->n;
  if (hipMalloc(&nbr->grow_ptr, sizeof(int64_t) * (n + 1)) != hipSuccess ||
      hipMalloc(&nbr->gpos, sizeof(int32_t) * n) != hipSuccess ||
      hipMalloc(&nbr->grev, sizeof(int32_t) * std::max<int64_t>(nbr->nnz, 1)) != hipSuccess) {
    if (nbr->grow_ptr) (void)hipFree(nbr->grow_ptr);
    if (nbr->gpos) (void)hipFree(nbr->gpos);
    nbr->grow_ptr = nullptr;
    nbr->gpos = nullptr;
    nbr->grev = nullptr;
    return set_error(ctx, GF_ENOMEM, "grouped row offsets allocation failed");
  }
  Arena ar;
  if ((st = ensure_scratch(ctx, arena_bytes({sizeof(int32_t) * n, sizeof(int64_t) * scan_tmp_elems(n + 1)}), &ar)))
    return st;
  int32_t *len = ar.take<int32_t>(n);
  int64_t *tmp = ar.take<int64_t>(scan_tmp_elems(n + 1));
  hipLaunchKernelGGL(k_grouped_len, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, nbr->grouped,
                     nbr->row_ptr, n, len, nbr->gpos);
  GF_LAUNCH_CHECK(ctx);
  if ((st = scan_i32_to_i64(ctx, len, nbr->grow_ptr, n, tmp))) return st;
  hipLaunchKernelGGL(k_grouped_rev, dim3(grid_for(n * kRevTeam, kBlock)), dim3(kBlock), 0, ctx->stream, nbr->grouped,
                     nbr->row_ptr, nbr->col, nbr->rev, nbr->grow_ptr, nbr->gpos, n, nbr->grev);
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
  if (hipMalloc(&nb->slot, sizeof(uint16_t) * (nb->nnz + kQuadPad)) != hipSuccess ||
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
  {
    ProfScope prof(ctx, "nbr_tile_unique");
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, sm, grp_max, (int64_t)16, 0);
    hipLaunchKernelGGL(k_tile_entries, dim3(grid_for(nt, kBlock)), dim3(kBlock), 0, sm, tg, nb->row_ptr, nb->grouped,
                       ent);
    GF_LAUNCH_CHECK(ctx);
    if ((st = scan_i32_to_i64(ctx, ent, ent_off, nt, tmp64))) return st;
    hipLaunchKernelGGL(k_tile_unique, dim3((unsigned)nt), dim3(kTileThreads), 0, sm, tg, nb->row_ptr, nb->col,
                       nb->grouped, ent_off, nb->slot, uniq, cnt, grp_max);
    GF_LAUNCH_CHECK(ctx);
    if ((st = scan_i32_to_i64(ctx, cnt, nb->tile_off, nt, tmp64))) return st;
  }
  if ((st = ensure_host(ctx, 4096))) return st;
  char *hp = (char *)ctx->host_pinned;
  GF_HIP(ctx, hipMemcpyAsync(hp, grp_max, sizeof(int32_t) * 16, hipMemcpyDeviceToHost, sm));
  GF_HIP(ctx, hipMemcpyAsync(hp + 128, nb->tile_off + nt, sizeof(int64_t), hipMemcpyDeviceToHost, sm));
  GF_HIP(ctx, hipStreamSynchronize(sm));
  for (int q = 0; q < tg.nq; ++q) nb->tile_max[tg.gsel[q]] = ((int32_t *)hp)[q];  // per model
  const int64_t total = *(int64_t *)(hp + 128);
  if (hipMalloc(&nb->tile_u, sizeof(int32_t) * std::max<int64_t>(total, 1)) != hipSuccess)
    return set_error(ctx, GF_ENOMEM, "neighbour tile list allocation failed");
  ProfScope prof(ctx, "nbr_tile_compact");
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

// the grid of each model's last (smallest-support) level alone: every
// particle of the model falls in its cells, which hold few particles each
static Grid finest_grid(const Grid &g) {
  Grid g1;
  memset(&g1, 0, sizeof(g1));
  int ns = 0;
  int64_t base = 0;
  for (int m = 0; m < 2; ++m) {
    g1.slot0[m] = ns;
    if (g.slot0[m + 1] > g.slot0[m]) {
      const int s = g.slot0[m + 1] - 1;
      for (int d = 0; d < 3; ++d) {
        g1.lo[ns][d] = g.lo[s][d];
        g1.dim[ns][d] = g.dim[s][d];
        g1.bits[ns][d] = g.bits[s][d];
      }
      g1.inv_edge[ns] = g.inv_edge[s];
      g1.hcap[ns] = g.hcap[s];
      g1.base[ns] = base;
      base += (int64_t)1 << (g.bits[s][0] + g.bits[s][1] + g.bits[s][2]);
      ++ns;
    }
  }
  g1.slot0[2] = ns;
  g1.nslots = ns;
  g1.nkeys = base;
  return g1;
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
  static_assert(kBboxFin >= 1024, "one final thread per bounding-box block");
  hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(kBboxFin), 0, sm, part, bad_part, nblk, box, bad);
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

  // ---- grids: per model, levels with halving support caps (Grid); a grid's
  // edge is slightly above its cap so that rounding of the cell coordinate
  // never hides a neighbour
  Grid g;
  memset(&g, 0, sizeof(g));
  double lo[2][3], hi[2][3], hmx[2], hmn[2];
  for (int m = 0; m < 2; ++m) {
    for (int d = 0; d < 3; ++d) { lo[m][d] = bx[m * 8 + d]; hi[m][d] = bx[m * 8 + 3 + d]; }
    hmx[m] = bx[m * 8 + 6];
    hmn[m] = bx[m * 8 + 7];
  }
  const int64_t key_budget = std::max<int64_t>(4 * n, 1 << 16);  // per grid
  int64_t base = 0;
  int ns = 0;
  for (int m = 0; m < 2; ++m) {
    g.slot0[m] = ns;
    const bool empty = !(hmx[m] > 0.0);
    int L = 1;
    if (!empty)
      while (L < kMaxLevels && hmn[m] <= std::ldexp(hmx[m], -L)) ++L;
    for (int l = 0; l < L; ++l, ++ns) {
      g.hcap[ns] = empty ? 0.0 : std::ldexp(hmx[m], -l);
      double edge = empty ? 1.0 : g.hcap[ns] * (1.0 + 1e-9);
      for (int it = 0; it < 200; ++it) {
        int tb = 0;
        for (int d = 0; d < 3; ++d) {
          double span = empty ? 0.0 : hi[m][d] - lo[m][d];
          double dd = std::floor(span / edge) + 1.0;
          if (dd > 1e6) dd = 1e6;
          g.dim[ns][d] = (int)dd;
          g.bits[ns][d] = ceil_log2(g.dim[ns][d]);
          tb += g.bits[ns][d];
        }
        if (tb <= 30 && ((int64_t)1 << tb) <= key_budget) break;
        edge *= 1.5;
      }
      for (int d = 0; d < 3; ++d) g.lo[ns][d] = empty ? 0.0 : lo[m][d];
      g.inv_edge[ns] = 1.0 / edge;
      g.base[ns] = base;
      base += (int64_t)1 << (g.bits[ns][0] + g.bits[ns][1] + g.bits[ns][2]);
    }
  }
  g.slot0[2] = ns;
  g.nslots = ns;
  g.nkeys = base;
  if (g.nkeys >= (int64_t)0x7fffffff) return set_error(ctx, GF_ECAPACITY, "cell grid too large");

  // ---- sort particles into cells
  const int64_t K = g.nkeys;
  sz = {sizeof(int32_t) * n, sizeof(int32_t) * n, sizeof(int32_t) * (K + 1), sizeof(int32_t) * scan_tmp_elems(K + 1),
        sizeof(double4) * n, sizeof(int32_t) * n, sizeof(int64_t) * scan_tmp_elems(n + 1), sizeof(int32_t) * 32,
        sizeof(int32_t) * n, sizeof(int32_t) * (n + 1), sizeof(int32_t) * scan_tmp_elems(n + 1),
        sizeof(int32_t) * n, sizeof(int32_t) * n};
  // rows staged by the count pass (sw entries each, the widest that stays
  // under 8 GB); rows found longer are filled by a second search pass
  int sw = 0;
  for (int w : kStageWidths)
    if (sw == 0 && (double)n * w * sizeof(int32_t) <= 8e9) sw = w;
  const bool use_stage = sw > 0;
  if (use_stage) sz.push_back(sizeof(int32_t) * (size_t)n * sw);
  if ((st = ensure_scratch(ctx, arena_bytes(sz), &ar))) return st;
  int32_t *key = ar.take<int32_t>(n);
  int32_t *slot = ar.take<int32_t>(n);
  int32_t *cell_start = ar.take<int32_t>(K + 1);
  int32_t *tmp32 = ar.take<int32_t>(scan_tmp_elems(K + 1));
  double4 *sp = ar.take<double4>(n);
  int32_t *cnt = ar.take<int32_t>(n);
  int64_t *tmp64 = ar.take<int64_t>(scan_tmp_elems(n + 1));
  // hist[8], maxrow, -, queue counters of the two search passes [10], [11],
  // particles per grid [16 .. 16 + kMaxSlots); zeroed before use
  int32_t *small = ar.take<int32_t>(32);
  int32_t *slot_count = small + 16;
  int32_t *gflag = ar.take<int32_t>(n);
  int32_t *gpos = ar.take<int32_t>(n + 1);
  int32_t *tmpg = ar.take<int32_t>(scan_tmp_elems(n + 1));
  // list of non-empty cells (first sorted position of each); the cell heads
  // and their scan borrow the grouping arrays, which are free until the fill
  // pass has finished
  int32_t *cells = ar.take<int32_t>(n);
  int32_t *order1 = ar.take<int32_t>(n);  // model-wide cell order for the grouping (several levels)
  int32_t *stage = use_stage ? ar.take<int32_t>((size_t)n * sw) : nullptr;
  int32_t *head = gflag, *cpos = gpos;
  const int32_t *ncells = cpos + n;

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
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(kBlock), 0, sm, small, (int64_t)32, 0);
  hipLaunchKernelGGL(k_keys, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, sm, p->x, p->y, p->z, p->h, p->model, n, g,
                     key, slot, cell_start);
  if (hipGetLastError() != hipSuccess) return fail(set_error(ctx, GF_EHIP, "key kernel launch failed"));
  if ((st = scan_i32_to_i32(ctx, cell_start, cell_start, K, tmp32))) return fail(st);
  hipLaunchKernelGGL(k_slot_count, dim3(1), dim3(64), 0, sm, cell_start, g, slot_count);
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, sm, key, slot, cell_start, n, nb->order);
  hipLaunchKernelGGL(k_cell_heads, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, sm, nb->order, key, n, head);
  if ((st = scan_i32_to_i32(ctx, head, cpos, n, tmpg))) return fail(st);
  hipLaunchKernelGGL(k_cell_list, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, sm, head, cpos, n, cells);
  hipLaunchKernelGGL(k_cell_sort_reg, dim3((unsigned)std::min<int64_t>((n + kCellSortWaves - 1) / kCellSortWaves, 4096)),
                     dim3(64 * kCellSortWaves), 0, sm, cells, ncells, n, p->x, p->y, p->z, p->h, p->model, g,
                     nb->order);
  hipLaunchKernelGGL(k_cell_sort, dim3((unsigned)std::min<int64_t>(n, 2048)), dim3(64), 0, sm, cells, ncells, n,
                     p->x, p->y, p->z, p->h, p->model, g, nb->order);
  hipLaunchKernelGGL(k_gather_pos, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, sm, nb->order, p->x, p->y, p->z, p->h,
                     n, sp);
  }
  // one wave per non-empty cell from a queue; as many waves as fit at once
  const dim3 search_grid((unsigned)std::max<int64_t>(
      1, std::min<int64_t>((n + kSearchWaves - 1) / kSearchWaves, (int64_t)ctx->num_cu * kSearchWavesPerSimd)));
  {
  ProfScope prof_count(ctx, "nbr_count");
  hipLaunchKernelGGL(k_search<0>, search_grid, dim3(kSearchBlock), 0, sm, nb->order, sp, p->model, cell_start, cells,
                     ncells, slot_count, small + 10, n, n_rows, g, cross_model ? 1 : 0, cnt, small, small + 8,
                     (const int64_t *)nullptr, (int32_t *)nullptr, stage, sw);
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
  // staged rows need no fill pass; rows longer than sw (if any) are filled by one that
  // writes only those
  const bool staged = use_stage;
  if (!staged || nb->max_row > sw) {
    ProfScope prof_fill(ctx, "nbr_fill");
    hipLaunchKernelGGL(k_search<1>, search_grid, dim3(kSearchBlock), 0, sm, nb->order, sp, p->model, cell_start,
                       cells, ncells, slot_count, small + 11, n, n_rows, g, cross_model ? 1 : 0, (int32_t *)nullptr,
                       (int32_t *)nullptr, (int32_t *)nullptr, nb->row_ptr, nb->col, staged ? stage : (int32_t *)nullptr,
                       sw);
  }
  {
    // staged rows: sorted on their way into the CSR; else sorted in place
    ProfScope prof_sort(ctx, "nbr_row_sort");
    const int64_t nchunks = (n + 63) / 64;
    const dim3 sgrid((unsigned)std::max<int64_t>(1, std::min<int64_t>((nchunks + kSortWaves - 1) / kSortWaves, 4096)));
    const size_t lds = nb->max_row > 128 ? sizeof(int32_t) * kSortWaves * kMaxRow : 0;
    if (staged && nb->max_row > 128)
      hipLaunchKernelGGL((k_row_sort<true, true>), sgrid, dim3(kSortBlock), lds, sm, nb->row_ptr, nb->col, stage, sw,
                         n);
    else if (staged)
      hipLaunchKernelGGL((k_row_sort<false, true>), sgrid, dim3(kSortBlock), 0, sm, nb->row_ptr, nb->col, stage, sw,
                         n);
    else if (nb->max_row > 128)
      hipLaunchKernelGGL((k_row_sort<true, false>), sgrid, dim3(kSortBlock), lds, sm, nb->row_ptr, nb->col,
                         (const int32_t *)nullptr, 0, n);
    else
      hipLaunchKernelGGL((k_row_sort<false, false>), sgrid, dim3(kSortBlock), 0, sm, nb->row_ptr, nb->col,
                         (const int32_t *)nullptr, 0, n);
  }
  if (hipGetLastError() != hipSuccess) return fail(set_error(ctx, GF_EHIP, "fill/sort kernel launch failed"));

  // ---- groups by (model, band), Morton order kept inside each group.  The
  // cell order is level by level when a model has several support levels, so
  // a tile cut from it would gather particles of one level from a wide
  // region; the grouping then follows a model-wide order instead: the cells
  // of each model's smallest-support grid in Morton order, fine Morton key
  // inside each cell (the same kernels on a grid with one level per model).
  // The arrays of the first cell pass are free once the rows are written.
  const int32_t *gorder = nb->order;
  if (g.slot0[1] - g.slot0[0] > 1 || g.slot0[2] - g.slot0[1] > 1) {
    ProfScope prof_o(ctx, "nbr_order");
    const Grid g1 = finest_grid(g);
    const int64_t K1 = g1.nkeys;  // <= K: the slots of g1 are slots of g
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(K1 + 1, kBlock)), dim3(kBlock), 0, sm, cell_start, K1 + 1, 0);
    hipLaunchKernelGGL(k_keys, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, sm, p->x, p->y, p->z, p->h, p->model, n,
                       g1, key, slot, cell_start);
    if ((st = scan_i32_to_i32(ctx, cell_start, cell_start, K1, tmp32))) return fail(st);
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, sm, key, slot, cell_start, n, order1);
    hipLaunchKernelGGL(k_cell_heads, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, sm, order1, key, n, head);
    if ((st = scan_i32_to_i32(ctx, head, cpos, n, tmpg))) return fail(st);
    hipLaunchKernelGGL(k_cell_list, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, sm, head, cpos, n, cells);
    hipLaunchKernelGGL(k_cell_sort_reg,
                       dim3((unsigned)std::min<int64_t>((n + kCellSortWaves - 1) / kCellSortWaves, 4096)),
                       dim3(64 * kCellSortWaves), 0, sm, cells, ncells, n, p->x, p->y, p->z, p->h, p->model, g1,
                       order1);
    hipLaunchKernelGGL(k_cell_sort, dim3((unsigned)std::min<int64_t>(n, 2048)), dim3(64), 0, sm, cells, ncells, n,
                       p->x, p->y, p->z, p->h, p->model, g1, order1);
    if (hipGetLastError() != hipSuccess) return fail(set_error(ctx, GF_EHIP, "order kernels failed"));
    gorder = order1;
  }
  int64_t off = 0;
  {
  ProfScope prof_group(ctx, "nbr_group");
  for (int gsel = 0; gsel < 2 * GF_NBAND; ++gsel) {
    nb->group_start[gsel] = off;
    if (hist[gsel] == 0) continue;
    hipLaunchKernelGGL(k_group_flag, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, sm, gorder, cnt, p->model, n,
                       gsel, gflag);
    if ((st = scan_i32_to_i32(ctx, gflag, gpos, n, tmpg))) return fail(st);
    hipLaunchKernelGGL(k_group_scatter, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, sm, gorder, gflag, gpos, n,
                       off, nb->grouped);
    off += hist[gsel];
  }
  nb->group_start[2 * GF_NBAND] = off;
  }
  if (hipGetLastError() != hipSuccess) return fail(set_error(ctx, GF_EHIP, "grouping kernels failed"));
  if (off != n) return fail(set_error(ctx, GF_EHIP, "internal error: grouping covers %lld of %lld", (long long)off,
                                      (long long)n));
  if ((st = build_tiles(ctx, nb))) return fail(st);
  *out = nb;
  return GF_OK;
}
