// Implicit pressure-Poisson solve (projection scheme, Sec. 2.3) on the GFDM
// stencils: assembly of the matrix on the neighbour pattern, then
// right-preconditioned BiCGStab with the Jacobi preconditioner.
//
// The iteration runs as five fused kernels (direction update, SpMV + dot,
// intermediate update, SpMV + two dots, solution/residual update + two dots).
// Scalars (rho, alpha, omega, ...) stay on the device.  Every dot product is
// a deterministic two-level reduction: the kernels that produce it run a
// fixed grid of kRedBlocks blocks (grid-stride over the rows) and write one
// partial per block; a one-block kernel adds the partials in block order and
// updates the scalars.  The kernel boundary makes the partials visible (no
// device-scope fences: on a chip whose XCDs have separate L2 caches each such
// fence writes back an L2).  The host reads the residual norm every few
// iterations.
//
// Mixed modes.  mixed = 1: one BiCGStab run whose SpMV reads FP32 matrix
// values (4 instead of 8 bytes per entry) while the Krylov vectors, dots and
// updates stay FP64; its recursive residual tracks b - A32 x, so whenever it
// has fallen by kReplace since the last replacement (and when it reaches the
// tolerance) it is replaced by the FP64 residual b - A64 x (residual
// replacement, a form of iterative refinement that keeps the Krylov space:
// no restart).  mixed = 2: iterative refinement with restarts: the residual
// r = b - A64 x in FP64, then an inner BiCGStab on FP32 values and FP32
// vectors (dots accumulated in FP64) solves A32 d = r from d = 0 to a
// relative reduction inner_rtol, and x += d.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "stencil_common.h"

using namespace gfdm_dev;

namespace {
constexpr int kBlock = 256;
constexpr int kTeam = 8;
static_assert(kBlock / kTeam == kTileRows, "one team per row of a neighbour tile");

struct Scal {
  double rho, rho_old, alpha, omega, rv, ts, tt, rr, bb;
  int breakdown;
  int half;  // the half step solved the system (t = A shat = 0)
};

// ---------------------------------------------------------------- reductions
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double block_sum(double v) {
  __shared__ double sh[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) r += sh[w];
  return r;
}

constexpr int kRedBlocks = 2048;   // blocks of the reducing kernels
constexpr double kReplace = 1e-2;  // mixed = 1: residual replacement after this reduction
constexpr int kFinThreads = 1024;  // threads of the finishing kernels

// one partial per block and value: part[k * gridDim.x + blockIdx.x]
template <int NV>
__device__ inline void block_partials(const double v[NV], double *part) {
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double s = block_sum(v[k]);
    if (threadIdx.x == 0) part[(int64_t)k * gridDim.x + blockIdx.x] = s;
  }
}

// sums of the partials of nblk blocks, in block order, on every thread
template <int NV>
__device__ inline void finish_partials(const double *part, int nblk, double res[NV]) {
  __shared__ double sh[kFinThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kFinThreads) acc += part[(int64_t)k * nblk + b];
    acc = wave_sum(acc);
    __syncthreads();
    if (lane == 0) sh[wid] = acc;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < kFinThreads / 64; ++w) r += sh[w];
    res[k] = r;
  }
}

// ---------------------------------------------------------------- assembly
// One team of kTeam lanes per row (grid-stride): the row's values, its
// diagonal (found by the lane holding the self entry) and the Jacobi inverse.
__global__ void __launch_bounds__(kBlock) k_assemble(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                                     const double *__restrict__ w, const int8_t *__restrict__ row_type,
                                                     const double *__restrict__ h, const double *__restrict__ nx,
                                                     const double *__restrict__ ny, const double *__restrict__ nz,
                                                     double zeta, double a, int max_type, int64_t n,
                                                     double *__restrict__ val64,
                                                     float *__restrict__ val32, double *__restrict__ dinv64,
                                                     float *__restrict__ dinv32, int *__restrict__ bad) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = (int)(gt % kTeam);
  const int64_t nteams = (int64_t)gridDim.x * blockDim.x / kTeam;
  for (int64_t i = gt / kTeam; i < n; i += nteams) {
    const int rt = row_type[i];
    double nrm[3] = {0.0, 0.0, 0.0};
    if (rt == GF_ROW_NEUMANN_COMBINED || rt == GF_ROW_NEUMANN) { nrm[0] = nx[i]; nrm[1] = ny[i]; nrm[2] = nz[i]; }
    const double zf = zeta / h[i];
    double diag = 0.0;  // nonzero only on the lane that holds the self entry
    for (int64_t k = row_ptr[i] + lane; k < row_ptr[i + 1]; k += kTeam) {
      const double2 *p = reinterpret_cast<const double2 *>(w) + 2 * k;
      const double2 g01 = p[0], g23 = p[1];
      const double ngrad = nrm[0] * g01.x + nrm[1] * g01.y + nrm[2] * g23.x;
      const bool self = col[k] == i;
      double v;
      switch (rt) {
        case GF_ROW_INTERIOR: v = g23.y; break;
        case GF_ROW_DIRICHLET: v = self ? 1.0 : 0.0; break;
        case GF_ROW_NEUMANN_COMBINED: v = g23.y + zf * ngrad; break;
        case GF_ROW_IMPLICIT: v = (self ? 1.0 : 0.0) - a * g23.y; break;
        default: v = ngrad; break;
      }
      if (val64) val64[k] = v;
      if (val32) val32[k] = (float)v;
      if (self) diag = v;
    }
    diag = team_sum(diag, kTeam);  // exactly the self value: the other lanes add zeros
    if (lane == 0) {
      if (rt < 0 || rt > max_type || diag == 0.0 || !isfinite(diag)) atomicAdd(bad, 1);
      if (dinv64) dinv64[i] = (diag != 0.0) ? 1.0 / diag : 0.0;
      if (dinv32) dinv32[i] = (diag != 0.0) ? (float)(1.0 / diag) : 0.0f;
    }
  }
}

// ---------------------------------------------------------------- kernels
// Rows are taken by teams of kTeam lanes, grid-stride over the fixed grid.
#define GF_TEAM_ROWS(row)                                                              \
  const int64_t gt_ = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;                 \
  const int lane = (int)(gt_ % kTeam);                                                 \
  const int64_t nteams_ = (int64_t)gridDim.x * blockDim.x / kTeam;                     \
  for (int64_t row = gt_ / kTeam; row < n; row += nteams_)

// r = b - A x (FP64), optionally rhat = r; partials of (r,r) and (b,b)
__global__ void __launch_bounds__(kBlock) k_residual(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                                     const double *__restrict__ val, const double *__restrict__ b,
                                                     const double *__restrict__ x, int64_t n, double *__restrict__ r,
                                                     double *__restrict__ rhat, double *part) {
  double v[2] = {0.0, 0.0};
  GF_TEAM_ROWS(row) {
    double acc = 0.0;
    for (int64_t k = row_ptr[row] + lane; k < row_ptr[row + 1]; k += kTeam) acc += val[k] * x[col[k]];
    acc = team_sum(acc, kTeam);
    if (lane == 0) {
      const double ri = b[row] - acc;
      r[row] = ri;
      if (rhat) rhat[row] = ri;
      v[0] += ri * ri;
      v[1] += b[row] * b[row];
    }
  }
  block_partials<2>(v, part);
}

// residual replacement: r = b - A x with FP64 values; partials of (r, r) and
// (rhat, r), so that rho continues from the replaced residual
__global__ void __launch_bounds__(kBlock) k_residual_replace(const int64_t *__restrict__ row_ptr,
                                                             const int32_t *__restrict__ col,
                                                             const double *__restrict__ val, const double *__restrict__ b,
                                                             const double *__restrict__ x, const double *__restrict__ rhat,
                                                             int64_t n, double *__restrict__ r, double *part) {
  double v[2] = {0.0, 0.0};
  GF_TEAM_ROWS(row) {
    double acc = 0.0;
    for (int64_t k = row_ptr[row] + lane; k < row_ptr[row + 1]; k += kTeam) acc += val[k] * x[col[k]];
    acc = team_sum(acc, kTeam);
    if (lane == 0) {
      const double ri = b[row] - acc;
      r[row] = ri;
      v[0] += ri * ri;
      v[1] += rhat[row] * ri;
    }
  }
  block_partials<2>(v, part);
}

__global__ void __launch_bounds__(kFinThreads) k_fin_replace(const double *part, int nblk, Scal *S) {
  double res[2];
  finish_partials<2>(part, nblk, res);
  if (threadIdx.x != 0) return;
  S->rr = res[0];
  S->rho = res[1];  // rho_old keeps the value of the last iteration
  if (res[1] == 0.0 || !isfinite(res[1])) S->breakdown = 4;
}

// scalars after a residual: rr, bb; with reset, a fresh BiCGStab start (rhat = r)
__global__ void __launch_bounds__(kFinThreads) k_fin_residual(const double *part, int nblk, Scal *S, int reset) {
  double res[2];
  finish_partials<2>(part, nblk, res);
  if (threadIdx.x != 0) return;
  S->rr = res[0];
  S->bb = res[1];
  if (reset) {
    S->rho = res[0];
    S->rho_old = 1.0;
    S->alpha = 1.0;
    S->omega = 1.0;
    S->breakdown = 0;
    S->half = 0;
  }
}

// x32 = (float) r64; rhat32 = x32; p = v = 0; partial of (r,r)
template <typename XT>
__global__ void __launch_bounds__(kBlock) k_inner_init(const double *__restrict__ r64, int64_t n, XT *__restrict__ r,
                                                       XT *__restrict__ rhat, XT *__restrict__ p, XT *__restrict__ vv,
                                                       XT *__restrict__ x, double *part) {
  double v[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const XT ri = (XT)r64[i];
    r[i] = ri;
    rhat[i] = ri;
    p[i] = (XT)0;
    vv[i] = (XT)0;
    x[i] = (XT)0;
    v[0] += (double)ri * (double)ri;
  }
  block_partials<1>(v, part);
}

__global__ void __launch_bounds__(kFinThreads) k_fin_inner_init(const double *part, int nblk, Scal *S) {
  double res[1];
  finish_partials<1>(part, nblk, res);
  if (threadIdx.x != 0) return;
  S->rr = res[0];
  S->rho = res[0];
  S->rho_old = 1.0;
  S->alpha = 1.0;
  S->omega = 1.0;
  S->breakdown = 0;
  S->half = 0;
}

template <typename XT>
__global__ void __launch_bounds__(kBlock) k_zero_vecs(int64_t n, XT *a, XT *b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) { a[i] = (XT)0; b[i] = (XT)0; }
}

// p = r + beta (p - omega v); phat = p * dinv
template <typename XT>
__global__ void __launch_bounds__(kBlock) k_update_p(const XT *__restrict__ r, const XT *__restrict__ vv,
                                                     const XT *__restrict__ dinv, int64_t n, XT *__restrict__ p,
                                                     XT *__restrict__ phat, const Scal *__restrict__ S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || S->breakdown) return;
  const double beta = (S->rho / S->rho_old) * (S->alpha / S->omega);
  const double pi = (double)r[i] + beta * ((double)p[i] - S->omega * (double)vv[i]);
  p[i] = (XT)pi;
  phat[i] = (XT)(pi * (double)dinv[i]);
}

// y = A xin; partials of (other, y) and (y, y)
template <typename VT, typename XT>
__global__ void __launch_bounds__(kBlock) k_spmv_dot(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                                     const VT *__restrict__ val, const XT *__restrict__ xin, int64_t n,
                                                     XT *__restrict__ y, const XT *__restrict__ other, double *part,
                                                     const Scal *__restrict__ S) {
  double v[2] = {0.0, 0.0};
  if (!S->breakdown) {
    GF_TEAM_ROWS(row) {
      double acc = 0.0;
      for (int64_t k = row_ptr[row] + lane; k < row_ptr[row + 1]; k += kTeam) acc += (double)val[k] * (double)xin[col[k]];
      acc = team_sum(acc, kTeam);
      if (lane == 0) {
        const XT yi = (XT)acc;
        y[row] = yi;
        v[0] += (double)other[row] * (double)yi;
        v[1] += (double)yi * (double)yi;
      }
    }
  }
  block_partials<2>(v, part);
}

// two values in one load
template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

// Neighbour tiles of the matrix pattern (the neighbour handle's tiles): rows
// of tile t are grouped[row0[m] + (t - tile_start[m]) kTileRows ...] for the
// model m owning t; rows with more than kTileBandRow entries are listed per
// model in grouped[b3_start[m] .. + b3_n[m]).
struct SpmvTiles {
  const int64_t *toff;
  const int32_t *tu;
  const uint16_t *slot;
  const int32_t *grouped;
  int64_t tile_start[3];
  int64_t row0[2], nrows[2];
  int64_t b3_start[2], b3_n[2];
  int cap;  // LDS entries of the staged vector
};

// y = A xin over tiles.  The tiles are cut into eight contiguous slices,
// one per XCD (blocks are dealt to the XCDs in turn, so block b runs on
// XCD b mod 8 and neighbouring tiles, which share most of their lists,
// meet in one L2); the G = gridDim.x / 8 blocks of a slice walk it with
// stride G.  A tile's 32 rows (one team of kTeam lanes each) read the
// entries of xin it references from LDS through slot[]; tiles whose list
// exceeds the LDS capacity gather through col[].  Then the untiled rows.
// Partials of (other, y) and (y, y).
//
// The walk is software-pipelined so that a tile costs about one memory
// latency instead of the chain tile offset -> tile list -> xin gather and
// row index -> row extent -> values: while the rows of tile t are summed
// from one LDS buffer, the loads for the following tiles are in flight:
// the xin entries of t+G (held in registers, written to the other buffer
// at the end of the step), the tile lists of t+2G, the tile offsets of
// t+3G, the row extents of t+G and the row indices of t+2G.  None of them
// depends on a load of the same step.  One barrier per tile separates the
// buffers.
//
// A row's entries are read in aligned quads (4q .. 4q+3): lane l of the team
// takes the quads q0 + l, q0 + l + kTeam, ... (at most kQ of them for a row
// of kTileBandRow entries), all loaded before any is used, so one load moves
// 32 B of values or 8 B of slots instead of 8 B or 2 B.  A quad may reach
// up to three entries into the neighbouring rows: those are read (the value
// and slot arrays carry kQuadPad entries of padding) but not used.
// K = staged entries per thread (K * kBlock >= LDS capacity).
constexpr int kQ = kTileBandRow / (4 * kTeam) + 1;

template <typename VT, typename XT, int K>
__global__ void __launch_bounds__(kBlock) k_spmv_tiles(const int64_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ col, const VT *__restrict__ val,
                                                       const XT *__restrict__ xin, XT *__restrict__ y,
                                                       const XT *__restrict__ other, double *part,
                                                       const Scal *__restrict__ S, SpmvTiles tl) {
  extern __shared__ unsigned char s_raw[];
  XT *sb = reinterpret_cast<XT *>(s_raw);  // two buffers of tl.cap entries
  double v[2] = {0.0, 0.0};
  const int team = threadIdx.x / kTeam, lane = threadIdx.x % kTeam;
  auto finish_row = [&](int32_t row, double acc) {
    acc = team_sum(acc, kTeam);
    if (lane == 0) {
      const XT yi = (XT)acc;
      y[row] = yi;
      v[0] += (double)other[row] * (double)yi;
      v[1] += (double)yi * (double)yi;
    }
  };
  if (!S->breakdown) {
    const int nslice = gridDim.x % 8 == 0 ? 8 : 1;
    const int slice = blockIdx.x % nslice;
    const int64_t G = gridDim.x / nslice;
    const int64_t nt = tl.tile_start[2] * (slice + 1) / nslice;  // end of this block's slice
    const int cap = tl.cap;
    // list offset and length of tile t (length -1 past the last tile)
    auto extent = [&](int64_t t, int64_t &u0, int &cnt) {
      if (t < nt) {
        u0 = tl.toff[t];
        cnt = (int)(tl.toff[t + 1] - u0);
      } else {
        u0 = 0;
        cnt = -1;
      }
    };
    // this thread's share of a staged tile's list (-1: nothing)
    auto load_list = [&](int64_t u0, int cnt, int32_t idx[K]) {
      const bool staged = cnt >= 0 && cnt <= cap;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int s = threadIdx.x + j * kBlock;
        idx[j] = (staged && s < cnt) ? tl.tu[u0 + s] : -1;
      }
    };
    // this team's row of tile t (-1: none)
    auto team_row = [&](int64_t t) -> int32_t {
      if (t >= nt) return -1;  // (past the slice: the tile belongs to another one)
      const int m = (t >= tl.tile_start[1]) ? 1 : 0;
      const int64_t r = (t - tl.tile_start[m]) * kTileRows + team;
      return r < tl.nrows[m] ? tl.grouped[tl.row0[m] + r] : -1;
    };
    auto gather = [&](const int32_t idx[K], XT xv[K]) {
#pragma unroll
      for (int j = 0; j < K; ++j) xv[j] = idx[j] >= 0 ? xin[idx[j]] : (XT)0;
    };
    auto put = [&](XT *buf, const XT xv[K], int cnt) {
      if (cnt < 0 || cnt > cap) return;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const int s = threadIdx.x + j * kBlock;
        if (s < cnt) buf[s] = xv[j];
      }
    };

    // prologue: tile t staged, the loads of t+G and t+2G issued
    int64_t t = tl.tile_start[2] * slice / nslice + blockIdx.x / nslice;
    int64_t u0_0, u0_1, u0_2;
    int c0, c1, c2;
    extent(t, u0_0, c0);
    extent(t + G, u0_1, c1);
    extent(t + 2 * G, u0_2, c2);
    int32_t idx1[K];
    {
      int32_t idx0[K];
      XT x0[K];
      load_list(u0_0, c0, idx0);
      gather(idx0, x0);
      put(sb, x0, c0);
    }
    load_list(u0_1, c1, idx1);
    int32_t row_c = team_row(t), row_n = team_row(t + G);
    int64_t b_c = 0, e_c = 0;
    if (row_c >= 0) {
      b_c = row_ptr[row_c];
      e_c = row_ptr[row_c + 1];
    }
    __syncthreads();
    int cur = 0;
    for (; t < nt; t += G) {
      XT xn[K];
      gather(idx1, xn);  // entries of t+G
      int32_t idx2[K];
      load_list(u0_2, c2, idx2);  // list of t+2G
      int64_t u0_3;
      int c3;
      extent(t + 3 * G, u0_3, c3);
      int64_t b_n = 0, e_n = 0;
      if (row_n >= 0) {  // row extent of t+G
        b_n = row_ptr[row_n];
        e_n = row_ptr[row_n + 1];
      }
      const int32_t row_nn = team_row(t + 2 * G);
      if (row_c >= 0) {
        double acc = 0.0;
        if (c0 <= cap) {
          const XT *buf = sb + cur * cap;
          typename Vec2<VT>::type va[kQ], vb[kQ];
          ushort4 ss[kQ];
          const int64_t q0 = (b_c >> 2) + lane;
#pragma unroll
          for (int j = 0; j < kQ; ++j) {
            const int64_t k = 4 * (q0 + j * kTeam);
            if (k < e_c) {
              va[j] = *reinterpret_cast<const typename Vec2<VT>::type *>(val + k);
              vb[j] = *reinterpret_cast<const typename Vec2<VT>::type *>(val + k + 2);
              ss[j] = *reinterpret_cast<const ushort4 *>(tl.slot + k);
            }
          }
#pragma unroll
          for (int j = 0; j < kQ; ++j) {
            const int64_t k = 4 * (q0 + j * kTeam);
            if (k < e_c) {
              if (k >= b_c) acc += (double)va[j].x * (double)buf[ss[j].x];
              if (k + 1 >= b_c && k + 1 < e_c) acc += (double)va[j].y * (double)buf[ss[j].y];
              if (k + 2 >= b_c && k + 2 < e_c) acc += (double)vb[j].x * (double)buf[ss[j].z];
              if (k + 3 < e_c) acc += (double)vb[j].y * (double)buf[ss[j].w];
            }
          }
        } else {
          for (int64_t k = b_c + lane; k < e_c; k += kTeam) acc += (double)val[k] * (double)xin[col[k]];
        }
        finish_row(row_c, acc);
      }
      put(sb + (cur ^ 1) * cap, xn, c1);
      __syncthreads();
      cur ^= 1;
      c0 = c1;
      u0_1 = u0_2; c1 = c2;
      u0_2 = u0_3; c2 = c3;
#pragma unroll
      for (int j = 0; j < K; ++j) idx1[j] = idx2[j];
      row_c = row_n; b_c = b_n; e_c = e_n;
      row_n = row_nn;
    }
    // untiled rows: teams grid-stride over each model's list
    const int64_t gteam = (int64_t)blockIdx.x * (blockDim.x / kTeam) + team;
    const int64_t nteams = (int64_t)gridDim.x * (blockDim.x / kTeam);
    for (int m = 0; m < 2; ++m) {
      for (int64_t q = gteam; q < tl.b3_n[m]; q += nteams) {
        const int32_t row = tl.grouped[tl.b3_start[m] + q];
        double acc = 0.0;
        for (int64_t k = row_ptr[row] + lane; k < row_ptr[row + 1]; k += kTeam) acc += (double)val[k] * (double)xin[col[k]];
        finish_row(row, acc);
      }
    }
  }
  block_partials<2>(v, part);
}

// STAGE 0: alpha = rho / (rhat, v);  STAGE 1: omega = (t, s) / (t, t)
template <int STAGE>
__global__ void __launch_bounds__(kFinThreads) k_fin_spmv(const double *part, int nblk, Scal *S) {
  double res[2];
  finish_partials<2>(part, nblk, res);
  if (threadIdx.x != 0 || S->breakdown) return;
  if (STAGE == 0) {
    const double rv = res[0];
    S->rv = rv;
    if (rv == 0.0 || !isfinite(rv)) S->breakdown = 1;
    else S->alpha = S->rho / rv;
  } else {
    S->ts = res[0];
    S->tt = res[1];
    if (res[1] == 0.0) {
      // t = A shat = 0, so s = 0 for a nonsingular A: x + alpha phat already
      // solves the system.  Take that step (omega = 0) and restart from the
      // true residual afterwards (code 5).
      S->omega = 0.0;
      S->half = 1;
    } else if (!isfinite(res[1])) {
      S->breakdown = 2;
    } else {
      S->omega = res[0] / res[1];
      if (S->omega == 0.0) S->breakdown = 3;
    }
  }
}

// s = r - alpha v; shat = s * dinv
template <typename XT>
__global__ void __launch_bounds__(kBlock) k_update_s(const XT *__restrict__ r, const XT *__restrict__ vv,
                                                     const XT *__restrict__ dinv, int64_t n, XT *__restrict__ s,
                                                     XT *__restrict__ shat, const Scal *__restrict__ S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || S->breakdown) return;
  const double si = (double)r[i] - S->alpha * (double)vv[i];
  s[i] = (XT)si;
  shat[i] = (XT)(si * (double)dinv[i]);
}

// x += alpha phat + omega shat; r = s - omega t; partials of (rhat, r), (r, r)
template <typename XT>
__global__ void __launch_bounds__(kBlock) k_update_xr(const XT *__restrict__ phat, const XT *__restrict__ shat,
                                                      const XT *__restrict__ s, const XT *__restrict__ t,
                                                      const XT *__restrict__ rhat, int64_t n, XT *__restrict__ x,
                                                      XT *__restrict__ r, double *part, const Scal *__restrict__ S) {
  double v[2] = {0.0, 0.0};
  if (!S->breakdown) {
    const double al = S->alpha, om = S->omega;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
      x[i] = (XT)((double)x[i] + al * (double)phat[i] + om * (double)shat[i]);
      const double ri = (double)s[i] - om * (double)t[i];
      r[i] = (XT)ri;
      v[0] += (double)rhat[i] * (double)(XT)ri;
      v[1] += (double)(XT)ri * (double)(XT)ri;
    }
  }
  block_partials<2>(v, part);
}

__global__ void __launch_bounds__(kFinThreads) k_fin_xr(const double *part, int nblk, Scal *S) {
  double res[2];
  finish_partials<2>(part, nblk, res);
  if (threadIdx.x != 0 || S->breakdown) return;
  S->rho_old = S->rho;
  S->rho = res[0];
  S->rr = res[1];
  if (S->half) S->breakdown = 5;
  else if (res[0] == 0.0 || !isfinite(res[0])) S->breakdown = 4;
}

template <typename XT>
__global__ void __launch_bounds__(kBlock) k_add_corr(double *__restrict__ x, const XT *__restrict__ d, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += (double)d[i];
}

__global__ void k_reset_counter(unsigned *c) {
  if (threadIdx.x == 0) *c = 0u;
}

struct Solver {
  gf_ctx *ctx;
  const gf_nbr *nbr;
  int64_t n;
  double *part;  // [2 * kRedBlocks]
  Scal *S;
  Scal *hS;
  unsigned grid_row;
  bool tiled;    // the SpMV runs on the neighbour tiles
  SpmvTiles tl;
  int tiles_grid[3] = {0, 0, 0};  // blocks of the tiled SpMV (FP64; FP32 values; FP32 values and vectors), set at first use
  double *x_out = nullptr;        // the solution (refinement adds each inner correction here)
};

// staged-vector capacity of the tiled SpMV (entries)
constexpr int kSpmvCap = 2048;
static_assert(kSpmvCap <= 8 * kBlock, "the tiled SpMV stages at most 8 entries per thread");

void init_spmv_tiles(Solver &sv) {
  const gf_nbr *nb = sv.nbr;
  sv.tiled = nb->ntiles > 0 && nb->slot && nb->tile_u && nb->tile_off;
  SpmvTiles &t = sv.tl;
  t.toff = nb->tile_off; t.tu = nb->tile_u; t.slot = nb->slot; t.grouped = nb->grouped;
  for (int k = 0; k < 3; ++k) t.tile_start[k] = nb->tile_start[k];
  int cap = 0;
  for (int m = 0; m < 2; ++m) {
    t.row0[m] = nb->group_start[m * GF_NBAND];
    t.nrows[m] = nb->group_start[m * GF_NBAND + kTileBand + 1] - t.row0[m];
    t.b3_start[m] = nb->group_start[m * GF_NBAND + kTileBand + 1];
    t.b3_n[m] = nb->group_start[(m + 1) * GF_NBAND] - t.b3_start[m];
    cap = std::max(cap, nb->tile_max[m]);
  }
  t.cap = std::min(cap, tile_capacity(sv.ctx, kSpmvCap));
}

// Blocks of the tiled SpMV: as many as are resident at once (a block walks
// its tiles to the end, so a block that waits for a slot would add its whole
// walk to the time), a multiple of 8, at most kRedBlocks.
template <typename VT, typename XT, int K>
int spmv_tiles_grid(const Solver &sv, size_t lds) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_spmv_tiles<VT, XT, K>, kBlock, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return std::max(8, std::min(kRedBlocks, per_cu * sv.ctx->num_cu) / 8 * 8);
}

// y = A xin with the partials of (other, y), (y, y); returns the number of
// partials (blocks) written
template <typename VT, typename XT, int K>
int launch_spmv_tiles(Solver &sv, const VT *val, const XT *xin, XT *y, const XT *other) {
  const size_t lds = 2 * sizeof(XT) * (size_t)sv.tl.cap;
  int &grid = sv.tiles_grid[sizeof(VT) == 8 ? 0 : (sizeof(XT) == 8 ? 1 : 2)];
  if (grid == 0) grid = spmv_tiles_grid<VT, XT, K>(sv, lds);
  hipLaunchKernelGGL((k_spmv_tiles<VT, XT, K>), dim3(grid), dim3(kBlock), lds, sv.ctx->stream, sv.nbr->row_ptr,
                     sv.nbr->col, val, xin, y, other, sv.part, sv.S, sv.tl);
  return grid;
}

template <typename VT, typename XT>
int launch_spmv(Solver &sv, const VT *val, const XT *xin, XT *y, const XT *other) {
  if (sv.tiled) {
    const int k = (sv.tl.cap + kBlock - 1) / kBlock;
    if (k <= 1) return launch_spmv_tiles<VT, XT, 1>(sv, val, xin, y, other);
    if (k <= 2) return launch_spmv_tiles<VT, XT, 2>(sv, val, xin, y, other);
    if (k <= 3) return launch_spmv_tiles<VT, XT, 3>(sv, val, xin, y, other);
    if (k <= 4) return launch_spmv_tiles<VT, XT, 4>(sv, val, xin, y, other);
    return launch_spmv_tiles<VT, XT, 8>(sv, val, xin, y, other);
  }
  hipLaunchKernelGGL((k_spmv_dot<VT, XT>), dim3(kRedBlocks), dim3(kBlock), 0, sv.ctx->stream, sv.nbr->row_ptr,
                     sv.nbr->col, val, xin, sv.n, y, other, sv.part, sv.S);
  return kRedBlocks;
}

gf_status read_scal(Solver &sv) {
  GF_HIP(sv.ctx, hipMemcpyAsync(sv.hS, sv.S, sizeof(Scal), hipMemcpyDeviceToHost, sv.ctx->stream));
  GF_HIP(sv.ctx, hipStreamSynchronize(sv.ctx->stream));
  return GF_OK;
}

template <typename VT, typename XT>
struct Vecs {
  const VT *val;
  const XT *dinv;
  XT *x, *r, *rhat, *p, *v, *phat, *s, *shat, *t;
};

// r = b - A x (and rhat = r with reset) followed by its scalar update
void launch_residual(Solver &sv, const double *val64, const double *rhs, const double *x, double *r, double *rhat,
                     int reset) {
  hipStream_t sm = sv.ctx->stream;
  hipLaunchKernelGGL(k_residual, dim3(kRedBlocks), dim3(kBlock), 0, sm, sv.nbr->row_ptr, sv.nbr->col, val64, rhs, x,
                     sv.n, r, rhat, sv.part);
  hipLaunchKernelGGL(k_fin_residual, dim3(1), dim3(kFinThreads), 0, sm, sv.part, kRedBlocks, sv.S, reset);
}

// one BiCGStab iteration (5 launches + 3 one-block finishers)
template <typename VT, typename XT>
gf_status bicgstab_iter(Solver &sv, const Vecs<VT, XT> &V) {
  hipStream_t sm = sv.ctx->stream;
  const int64_t n = sv.n;
  ProfScope prof(sv.ctx, sizeof(VT) == 8 ? "bicgstab_iter_f64"
                        : (sizeof(XT) == 8 ? "bicgstab_iter_f32val" : "bicgstab_iter_f32"));
  hipLaunchKernelGGL((k_update_p<XT>), dim3(sv.grid_row), dim3(kBlock), 0, sm, V.r, V.v, V.dinv, n, V.p, V.phat, sv.S);
  int nb = launch_spmv<VT, XT>(sv, V.val, V.phat, V.v, V.rhat);
  hipLaunchKernelGGL((k_fin_spmv<0>), dim3(1), dim3(kFinThreads), 0, sm, sv.part, nb, sv.S);
  hipLaunchKernelGGL((k_update_s<XT>), dim3(sv.grid_row), dim3(kBlock), 0, sm, V.r, V.v, V.dinv, n, V.s, V.shat, sv.S);
  nb = launch_spmv<VT, XT>(sv, V.val, V.shat, V.t, V.s);
  hipLaunchKernelGGL((k_fin_spmv<1>), dim3(1), dim3(kFinThreads), 0, sm, sv.part, nb, sv.S);
  hipLaunchKernelGGL((k_update_xr<XT>), dim3(kRedBlocks), dim3(kBlock), 0, sm, V.phat, V.shat, V.s, V.t, V.rhat, n,
                     V.x, V.r, sv.part, sv.S);
  hipLaunchKernelGGL(k_fin_xr, dim3(1), dim3(kFinThreads), 0, sm, sv.part, kRedBlocks, sv.S);
  GF_LAUNCH_CHECK(sv.ctx);
  return GF_OK;
}

// One inner solve of the refinement: A32 d = r64 from d = 0 by Jacobi-BiCGStab
// on FP32 matrix values, until the recursive residual is below inner_target
// (or the iteration limits); then x += d.  `total` counts every iteration.
template <typename XT>
gf_status inner_solve(Solver &sv, const Vecs<float, XT> &V, const double *r64, double inner_target,
                      const gf_solve_params &prm, int &total, gf_solve_stats &sts) {
  gf_ctx *ctx = sv.ctx;
  hipStream_t sm = ctx->stream;
  hipLaunchKernelGGL(k_inner_init<XT>, dim3(kRedBlocks), dim3(kBlock), 0, sm, r64, sv.n, V.r, V.rhat, V.p, V.v, V.x,
                     sv.part);
  hipLaunchKernelGGL(k_fin_inner_init, dim3(1), dim3(kFinThreads), 0, sm, sv.part, kRedBlocks, sv.S);
  GF_LAUNCH_CHECK(ctx);
  gf_status st;
  int it = 0;
  while (it < prm.inner_maxit && total < prm.maxit) {
    if ((st = bicgstab_iter<float, XT>(sv, V))) return st;
    ++it;
    ++total;
    if (it % prm.check_every != 0) continue;
    if ((st = read_scal(sv))) return st;
    if (sv.hS->breakdown) { ++sts.restarts; break; }
    if (std::sqrt(sv.hS->rr) <= inner_target) break;
  }
  hipLaunchKernelGGL(k_add_corr<XT>, dim3(sv.grid_row), dim3(kBlock), 0, sm, sv.x_out, V.x, sv.n);
  GF_LAUNCH_CHECK(ctx);
  return GF_OK;
}
}  // namespace

extern "C" void gf_solve_params_default(gf_solve_params *p) {
  if (!p) return;
  p->rtol = 1e-8;
  p->maxit = 20000;
  p->mixed = 0;
  p->inner_rtol = 1e-4;
  p->inner_maxit = 2000;
  p->zeta = 0.3;
  p->check_every = 4;
  p->implicit_a = 0.0;
}

// a: coefficient of GF_ROW_IMPLICIT rows; max_type: largest row type accepted
static gf_status assemble_common(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr, const double *w64,
                                 const int8_t *row_type, double zeta, double a, int max_type, double *val64,
                                 float *val32, double *dinv64, float *dinv32, int *bad) {
  hipLaunchKernelGGL(k_assemble, dim3(kRedBlocks), dim3(kBlock), 0, ctx->stream, nbr->row_ptr, nbr->col,
                     w64, row_type, p->h, p->nx, p->ny, p->nz, zeta, a, max_type, p->n, val64, val32, dinv64, dinv32,
                     bad);
  GF_LAUNCH_CHECK(ctx);
  return GF_OK;
}

static gf_status check_solve_args(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr, const double *w64,
                                  const int8_t *row_type) {
  gf_status st = check_particles(ctx, p, false, false);
  if (st) return st;
  if ((st = check_nbr(ctx, nbr, p->n))) return st;
  if (nbr->cross) return set_error(ctx, GF_EINVAL, "the pressure system lives on same-model neighbourhoods");
  if (!w64 || !row_type) return set_error(ctx, GF_EINVAL, "w64 and row_type are required");
  return GF_OK;
}

extern "C" gf_status gf_poisson_assemble(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr, const double *w64,
                                         const int8_t *row_type, double zeta, double *val_out) {
  if (!ctx) return GF_EINVAL;
  gf_status st = check_solve_args(ctx, p, nbr, w64, row_type);
  if (st) return st;
  if (!val_out) return set_error(ctx, GF_EINVAL, "val_out is NULL");
  if (!p->nx || !p->ny || !p->nz) return set_error(ctx, GF_EINVAL, "normals are required for Neumann rows");
  Arena ar;
  if ((st = ensure_scratch(ctx, arena_bytes({64}), &ar))) return st;
  int *bad = ar.take<int>(16);
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, ctx->stream, (unsigned *)bad);
  return assemble_common(ctx, p, nbr, w64, row_type, zeta, 0.0, GF_ROW_NEUMANN, val_out, nullptr, nullptr, nullptr,
                         bad);
}

extern "C" gf_status gf_poisson_solve(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr, const double *w64,
                                      const int8_t *row_type, const double *rhs, double *p_inout,
                                      const gf_solve_params *params, gf_solve_stats *stats) {
  if (!ctx) return GF_EINVAL;
  gf_status st = check_solve_args(ctx, p, nbr, w64, row_type);
  if (st) return st;
  if (!rhs || !p_inout) return set_error(ctx, GF_EINVAL, "rhs and p_inout are required");
  if (!p->nx || !p->ny || !p->nz) return set_error(ctx, GF_EINVAL, "normals are required for Neumann rows");
  gf_solve_params prm;
  gf_solve_params_default(&prm);
  if (params) prm = *params;
  if (!(prm.rtol > 0.0) || prm.maxit <= 0 || prm.check_every <= 0 || prm.mixed < 0 || prm.mixed > 2 ||
      (prm.mixed && (!(prm.inner_rtol > 0.0) || prm.inner_maxit <= 0)))
    return set_error(ctx, GF_EINVAL, "invalid solver parameters");
  gf_solve_stats sts;
  memset(&sts, 0, sizeof(sts));
  const auto t_start = std::chrono::steady_clock::now();
  auto elapsed = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count(); };
  const int64_t n = p->n, nnz = nbr->nnz;
  const bool mixed = prm.mixed != 0;
  const bool vec32 = prm.mixed == 2;  // FP32 Krylov vectors in the inner solve
  Arena ar;
  const int nblk_row = (int)grid_for(n, kBlock);
  std::vector<size_t> sz = {sizeof(double) * (nnz + kQuadPad), sizeof(double) * n, sizeof(double) * 2 * kRedBlocks + 64,
                            sizeof(Scal), 64};
  for (int k = 0; k < 9; ++k) sz.push_back(sizeof(double) * n);
  if (mixed) {
    sz.push_back(sizeof(float) * (nnz + kQuadPad));
    sz.push_back(sizeof(float) * n);
    if (vec32)
      for (int k = 0; k < 9; ++k) sz.push_back(sizeof(float) * n);
  }
  if ((st = ensure_scratch(ctx, arena_bytes(sz), &ar))) return st;
  double *val64 = ar.take<double>(nnz + kQuadPad);
  double *dinv64 = ar.take<double>(n);
  double *part = ar.take<double>(2 * kRedBlocks + 8);
  Scal *S = ar.take<Scal>(1);
  int *bad = ar.take<int>(16);
  double *vec64[9];
  for (int k = 0; k < 9; ++k) vec64[k] = ar.take<double>(n);
  float *val32 = nullptr, *dinv32 = nullptr, *v32[9] = {nullptr};
  if (mixed) {
    val32 = ar.take<float>(nnz + kQuadPad);
    dinv32 = ar.take<float>(n);
    if (vec32)
      for (int k = 0; k < 9; ++k) v32[k] = ar.take<float>(n);
  }
  if ((st = ensure_host(ctx, 4096))) return st;
  hipStream_t sm = ctx->stream;
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, sm, (unsigned *)bad);
  if ((st = assemble_common(ctx, p, nbr, w64, row_type, prm.zeta, prm.implicit_a, GF_ROW_IMPLICIT, val64, val32,
                            dinv64, dinv32, bad)))
    return st;
  Solver sv;
  sv.ctx = ctx; sv.nbr = nbr; sv.n = n; sv.part = part; sv.S = S;
  sv.hS = (Scal *)ctx->host_pinned;
  sv.grid_row = (unsigned)nblk_row;
  sv.x_out = p_inout;
  init_spmv_tiles(sv);
  int *hbad = (int *)((char *)ctx->host_pinned + 1024);
  GF_HIP(ctx, hipMemcpyAsync(hbad, bad, sizeof(int), hipMemcpyDeviceToHost, sm));
  // FP64 work vectors: x is the caller's array
  Vecs<double, double> V64;
  V64.val = val64; V64.dinv = dinv64; V64.x = p_inout;
  V64.r = vec64[0]; V64.rhat = vec64[1]; V64.p = vec64[2]; V64.v = vec64[3]; V64.phat = vec64[4];
  V64.s = vec64[5]; V64.shat = vec64[6]; V64.t = vec64[7];
  // initial residual
  launch_residual(sv, val64, rhs, p_inout, V64.r, V64.rhat, 1);
  hipLaunchKernelGGL(k_zero_vecs<double>, dim3(sv.grid_row), dim3(kBlock), 0, sm, n, V64.p, V64.v);
  GF_LAUNCH_CHECK(ctx);
  if ((st = read_scal(sv))) return st;
  if (*hbad > 0) return set_error(ctx, GF_EINVAL, "%d rows have an unknown row type or a zero/non-finite diagonal", *hbad);
  const double bnorm = std::sqrt(sv.hS->bb);
  double rnorm = std::sqrt(sv.hS->rr);
  if (bnorm == 0.0) {
    // the solution of A p = 0 is p = 0
    hipLaunchKernelGGL(k_zero_vecs<double>, dim3(sv.grid_row), dim3(kBlock), 0, sm, n, p_inout, V64.r);
    GF_LAUNCH_CHECK(ctx);
    sts.converged = 1;
    sts.seconds = elapsed();
    if (stats) *stats = sts;
    return GF_OK;
  }
  const double target = prm.rtol * bnorm;
  int total = 0;
  if (!mixed) {
    sts.outer_its = 1;
    // true residual at the last restart; restarts that no longer reduce it
    // mean the tolerance is below the attainable accuracy
    double restart_rnorm = rnorm;
    int stagnant = 0;
    while (rnorm > target && total < prm.maxit) {
      if ((st = bicgstab_iter<double, double>(sv, V64))) return st;
      ++total;
      if (total % prm.check_every != 0 && total < prm.maxit) continue;
      if ((st = read_scal(sv))) return st;
      if (sv.hS->breakdown) {
        if (++sts.restarts > 50) {
          sts.inner_its_total = total;
          sts.seconds = elapsed();
    if (stats) *stats = sts;
          return set_error(ctx, GF_EBREAKDOWN, "BiCGStab broke down repeatedly (code %d)", sv.hS->breakdown);
        }
        launch_residual(sv, val64, rhs, p_inout, V64.r, V64.rhat, 1);
        hipLaunchKernelGGL(k_zero_vecs<double>, dim3(sv.grid_row), dim3(kBlock), 0, sm, n, V64.p, V64.v);
        if ((st = read_scal(sv))) return st;
        rnorm = std::sqrt(sv.hS->rr);
        stagnant = rnorm < 0.9 * restart_rnorm ? 0 : stagnant + 1;
        restart_rnorm = std::min(restart_rnorm, rnorm);
        if (stagnant >= 3) break;
        continue;
      }
      rnorm = std::sqrt(sv.hS->rr);
      if (rnorm <= target) {
        // replace the recursive residual by the true one
        launch_residual(sv, val64, rhs, p_inout, V64.r, nullptr, 0);
        if ((st = read_scal(sv))) return st;
        rnorm = std::sqrt(sv.hS->rr);
      }
    }
  } else if (!vec32) {
    // FP32 matrix values, FP64 vectors, residual replacement with the FP64 matrix
    Vecs<float, double> V1 = {val32, dinv64, p_inout, V64.r, V64.rhat, V64.p, V64.v, V64.phat, V64.s, V64.shat, V64.t};
    sts.outer_its = 1;
    double last_true = rnorm;  // true residual at the last replacement (or restart)
    int stagnant = 0;
    while (rnorm > target && total < prm.maxit) {
      if ((st = bicgstab_iter<float, double>(sv, V1))) return st;
      ++total;
      if (total % prm.check_every != 0 && total < prm.maxit) continue;
      if ((st = read_scal(sv))) return st;
      if (sv.hS->breakdown) {
        if (++sts.restarts > 50) {
          sts.inner_its_total = total;
          sts.seconds = elapsed();
          if (stats) *stats = sts;
          return set_error(ctx, GF_EBREAKDOWN, "BiCGStab broke down repeatedly (code %d)", sv.hS->breakdown);
        }
        launch_residual(sv, val64, rhs, p_inout, V64.r, V64.rhat, 1);
        hipLaunchKernelGGL(k_zero_vecs<double>, dim3(sv.grid_row), dim3(kBlock), 0, sm, n, V64.p, V64.v);
        if ((st = read_scal(sv))) return st;
        rnorm = std::sqrt(sv.hS->rr);
        stagnant = rnorm < 0.9 * last_true ? 0 : stagnant + 1;
        last_true = std::min(last_true, rnorm);
        if (stagnant >= 3) break;
        continue;
      }
      const double rrec = std::sqrt(sv.hS->rr);
      if (rrec > std::max(target, kReplace * last_true)) {
        rnorm = rrec;
        continue;
      }
      // replace the recursive residual by the FP64 one
      hipLaunchKernelGGL(k_residual_replace, dim3(kRedBlocks), dim3(kBlock), 0, sm, nbr->row_ptr, nbr->col, val64,
                         rhs, p_inout, V64.rhat, n, V64.r, part);
      hipLaunchKernelGGL(k_fin_replace, dim3(1), dim3(kFinThreads), 0, sm, part, kRedBlocks, S);
      GF_LAUNCH_CHECK(ctx);
      if ((st = read_scal(sv))) return st;
      rnorm = std::sqrt(sv.hS->rr);
      ++sts.outer_its;
      // replacements that no longer cut the true residual: the tolerance is below what the FP32 matrix allows
      stagnant = rnorm < 0.9 * last_true ? 0 : stagnant + 1;
      last_true = rnorm;
      if (stagnant >= 3) break;
    }
  } else {
    // iterative refinement with restarts, FP32 inner vectors
    Vecs<float, float> Vf;
    Vf.val = val32; Vf.dinv = dinv32; Vf.x = v32[8];
    Vf.r = v32[0]; Vf.rhat = v32[1]; Vf.p = v32[2]; Vf.v = v32[3]; Vf.phat = v32[4];
    Vf.s = v32[5]; Vf.shat = v32[6]; Vf.t = v32[7];
    while (rnorm > target && total < prm.maxit) {
      ++sts.outer_its;
      // inner solve of A32 d = r64 from d = 0; the last one need not go below half the overall target
      const double inner_target = std::max(prm.inner_rtol * rnorm, 0.5 * target);
      if ((st = inner_solve<float>(sv, Vf, V64.r, inner_target, prm, total, sts))) return st;
      launch_residual(sv, val64, rhs, p_inout, V64.r, nullptr, 0);
      GF_LAUNCH_CHECK(ctx);
      if ((st = read_scal(sv))) return st;
      const double prev = rnorm;
      rnorm = std::sqrt(sv.hS->rr);
      if (sts.restarts > 50) break;
      if (!(rnorm < prev) && sts.outer_its > 3) break;  // refinement stagnated
    }
  }
  sts.inner_its_total = total;
  sts.final_rel_res = rnorm / bnorm;
  sts.converged = rnorm <= target;
  sts.seconds = elapsed();
  if (stats) *stats = sts;
  if (!sts.converged)
    return set_error(ctx, GF_ENOTCONV, "not converged: relative residual %.3e after %d iterations", sts.final_rel_res, total);
  return GF_OK;
}
