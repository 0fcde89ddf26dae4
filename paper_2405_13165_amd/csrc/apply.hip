// Stencil application (Eq. GFDM_Definition, differenced form) and its
// transpose.  Rows are taken in the grouped Morton order of the neighbour
// handle; a team of T lanes strides over a row's entries so one wave
// instruction reads T consecutive 16-byte (FP32) or 32-byte (FP64) weight
// records; partial sums are combined by a butterfly over the team and
// accumulated in FP64.
#include <algorithm>

#include "stencil_common.h"

using namespace gfdm_dev;

namespace {
constexpr int kBlock = 256;

template <typename WT>
struct W4;
template <>
struct W4<float> {
  static __device__ inline void load(const void *w, int64_t k, double c[4]) {
    const float4 v = reinterpret_cast<const float4 *>(w)[k];
    c[0] = v.x; c[1] = v.y; c[2] = v.z; c[3] = v.w;
  }
};
template <>
struct W4<double> {
  static __device__ inline void load(const void *w, int64_t k, double c[4]) {
    const double2 *p = reinterpret_cast<const double2 *>(w) + 2 * k;
    const double2 a = p[0], b = p[1];
    c[0] = a.x; c[1] = a.y; c[2] = b.x; c[3] = b.y;
  }
};

template <int T, typename WT, typename IOT>
__global__ void __launch_bounds__(kBlock) k_apply(const int32_t *__restrict__ sched, int64_t nrows,
                                                  const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                                  const void *__restrict__ w, unsigned mask,
                                                  const IOT *__restrict__ u, IOT *__restrict__ out, int64_t n) {
  const int64_t gt = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t team = gt / T;
  const int lane = (int)(gt % T);
  if (team >= nrows) return;
  const int32_t i = sched[team];
  const int64_t b = row_ptr[i], e = row_ptr[i + 1];
  const double ui = (double)u[i];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t k = b + lane; k < e; k += T) {
    const int32_t j = col[k];
    double c[4];
    W4<WT>::load(w, k, c);
    const double du = (j != i) ? (double)u[j] - ui : 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[s] += c[s] * du;
  }
  if constexpr (T > 1) {
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[s] = team_sum(acc[s], T);
  }
  if (lane == 0) {
    int q = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (mask & (1u << s)) out[(int64_t)(q++) * n + i] = (IOT)acc[s];
  }
}

// Tiled application (rows of the tiled bands): one block per neighbour tile;
// the field values of the tile's distinct neighbours are staged in LDS and
// each entry reads its value through slot[] (2 bytes) instead of col[]
// (4 bytes) plus a gather.  The diagonal entry contributes u_i - u_i = 0.
template <int T, typename WT, typename IOT>
__global__ void __launch_bounds__(kTileRows * T) k_apply_tile(const int32_t *__restrict__ sched, int64_t nrows,
                                                              const int64_t *__restrict__ row_ptr,
                                                              const int32_t *__restrict__ col,
                                                              const uint16_t *__restrict__ slot,
                                                              const int64_t *__restrict__ toff,
                                                              const int32_t *__restrict__ tu, int64_t tile0, int cap,
                                                              const void *__restrict__ w, unsigned mask,
                                                              const IOT *__restrict__ u, IOT *__restrict__ out,
                                                              int64_t n) {
  extern __shared__ double s_u[];
  const int64_t tl = xcd_block(blockIdx.x, gridDim.x);
  const int team = threadIdx.x / T, lane = threadIdx.x % T;
  const int64_t r = tl * kTileRows + team;
  // row prologue first: its loads overlap the staging below
  const bool live = r < nrows;
  const int32_t i = live ? sched[r] : 0;
  const int64_t b = live ? row_ptr[i] : 0, e = live ? row_ptr[i + 1] : 0;
  const double ui = (double)u[i];
  const int64_t u0 = toff[tile0 + tl];
  const int cnt = (int)(toff[tile0 + tl + 1] - u0);
  const bool staged = cnt <= cap;
  if (staged)
    for (int s = threadIdx.x; s < cnt; s += blockDim.x) s_u[s] = (double)u[tu[u0 + s]];
  __syncthreads();
  if (!live) return;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (staged) {
#pragma unroll 4
    for (int64_t k = b + lane; k < e; k += T) {
      double c[4];
      W4<WT>::load(w, k, c);
      const double du = s_u[slot[k]] - ui;
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[s] += c[s] * du;
    }
  } else {
    for (int64_t k = b + lane; k < e; k += T) {
      double c[4];
      W4<WT>::load(w, k, c);
      const double du = (double)u[col[k]] - ui;
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[s] += c[s] * du;
    }
  }
  if constexpr (T > 1) {
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[s] = team_sum(acc[s], T);
  }
  if (lane == 0) {
    int q = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (mask & (1u << s)) out[(int64_t)(q++) * n + i] = (IOT)acc[s];
  }
}

// field values a tiled apply block may stage
constexpr int kApplyCap = 2048;

// A stencil record (four operators of one entry) as loaded, converted to
// FP64 only where it is used: a conversion right after the load would wait
// for it there.
template <typename WT>
struct WRec;
template <>
struct WRec<float> {
  float4 v;
  __device__ inline void load(const void *w, int64_t k) { v = reinterpret_cast<const float4 *>(w)[k]; }
  __device__ inline double get(int s) const { return s == 0 ? v.x : s == 1 ? v.y : s == 2 ? v.z : v.w; }
};
template <>
struct WRec<double> {
  double2 a, b;
  __device__ inline void load(const void *w, int64_t k) {
    const double2 *p = reinterpret_cast<const double2 *>(w) + 2 * k;
    a = p[0];
    b = p[1];
  }
  __device__ inline double get(int s) const { return s == 0 ? a.x : s == 1 ? a.y : s == 2 ? b.x : b.y; }
};

// ubar_j = sum_{i : j in S_i, i != j} c_ij ybar_i - ybar_j sum_{k in S_j, k != j} c_jk,
// the first sum gathered through the reverse-edge map (entry (i,j) sits at
// rev[k] for the entry k = (j,i) of row j); an entry of row j without a twin
// (towards a ghost particle, which has no row) adds only its own term.
// One team of adj_team lanes per row j (the lanes stride over the row), K the
// number of selected operators.  Each lane takes adj_unroll entries per step: their
// columns and twin positions, then their two stencil records (c_ij of row i,
// c_ji of row j) and seeds ybar_i are all requested before the first is used,
// in one straight block (so that no load is moved down to its use); entries
// past the row's end read its last entry and an entry without a twin reads
// the stencil record 0 (both valid, added as zero), so no load is skipped.
// Team width and entries per step, as measured on the mixed cloud (FP32
// stencils: 8 x 4 took 572 / 631 us for one / four operators, 8 x 8 461 / 626,
// 16 x 4 495 / 569); FP64 records are twice as large and keep 8 x 4.
template <typename WT>
__host__ __device__ constexpr int adj_team(int K) { return (sizeof(WT) == 4 && K >= 3) ? 16 : 8; }
template <typename WT>
__host__ __device__ constexpr int adj_unroll(int K) { return (sizeof(WT) == 4 && K <= 2) ? 8 : 4; }
template <typename WT, int K>
__global__ void __launch_bounds__(kBlock) k_apply_adjoint(const int64_t *__restrict__ row_ptr,
                                                          const int32_t *__restrict__ col,
                                                          const int32_t *__restrict__ rev, const void *__restrict__ w,
                                                          unsigned mask, const double *__restrict__ ybar, int64_t n,
                                                          double *__restrict__ ubar) {
  constexpr int kAdjTeam = adj_team<WT>(K), kAU = adj_unroll<WT>(K);
  const int64_t gt = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t j = gt / kAdjTeam;
  const int lane = (int)(gt % kAdjTeam);
  if (j >= n) return;
  int sel[K];  // the selected operators in ascending order
  unsigned m = mask;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    sel[q] = K == 4 ? q : __builtin_ctz(m);
    m &= m - 1;
  }
  double yj[K];
#pragma unroll
  for (int q = 0; q < K; ++q) yj[q] = ybar[(int64_t)q * n + j];
  double acc = 0.0;
  const int64_t b = row_ptr[j], e = row_ptr[j + 1], kl = e - 1;
#pragma unroll 1
  for (int64_t kb = b + lane; kb < e; kb += kAU * kAdjTeam) {
    int32_t ci[kAU], kr[kAU];
#pragma unroll
    for (int u = 0; u < kAU; ++u) {
      const int64_t kk = min(kb + u * kAdjTeam, kl);
      ci[u] = col[kk];
      kr[u] = rev[kk];
    }
    WRec<WT> win[kAU], wout[kAU];
    double y[kAU][K];
#pragma unroll
    for (int u = 0; u < kAU; ++u) {
      win[u].load(w, kr[u] >= 0 ? kr[u] : 0);
      wout[u].load(w, min(kb + u * kAdjTeam, kl));
#pragma unroll
      for (int q = 0; q < K; ++q) y[u][q] = ybar[(int64_t)q * n + ci[u]];
    }
#pragma unroll
    for (int u = 0; u < kAU; ++u) {
      const bool on = kb + u * kAdjTeam < e && ci[u] != j;
#pragma unroll
      for (int q = 0; q < K; ++q) {
        const double t = (kr[u] >= 0 ? win[u].get(sel[q]) * y[u][q] : 0.0) - wout[u].get(sel[q]) * yj[q];
        acc += on ? t : 0.0;
      }
    }
  }
  acc = team_sum(acc, kAdjTeam);
  if (lane == 0) ubar[j] = acc;
}

template <typename WT, typename IOT>
gf_status launch_apply(gf_ctx *ctx, const gf_nbr *nbr, const void *w, unsigned mask, const void *u, void *out,
                       int only_unit = -1, int team_override = 0) {
  LaunchUnit units[2 * GF_NBAND];
  const int nu = launch_units(nbr, units);
  const IOT *uu = (const IOT *)u;
  IOT *oo = (IOT *)out;
  for (int q = 0; q < nu; ++q) {
    if (only_unit >= 0 && q != only_unit) continue;
    const LaunchUnit &lu = units[q];
    const int T = team_override > 0 ? team_override : ctx->ateam[lu.model][lu.band];
    const int32_t *sched = nbr->grouped + lu.row0;
    const int64_t nrows = lu.nrows;
    ProfScope prof(ctx, lu.model == 0 ? "apply_3d" : "apply_film");
    if (lu.tiled) {
      const int cap = std::min(lu.tile_max, tile_capacity(ctx, kApplyCap));
      const dim3 tgrid(grid_for(lu.ntiles, 1)), tblock(kTileRows * std::min(T, 32));
      const size_t lds = sizeof(double) * cap;
#define GF_APPLY_TILE(TT)                                                                                           \
  hipLaunchKernelGGL((k_apply_tile<TT, WT, IOT>), tgrid, tblock, lds, ctx->stream, sched, nrows, nbr->row_ptr,      \
                     nbr->col, nbr->slot, nbr->tile_off, nbr->tile_u, lu.tile0, cap, w, mask, uu, oo, nbr->n)
      switch (std::min(T, 32)) {
        case 4: GF_APPLY_TILE(4); break;
        case 8: GF_APPLY_TILE(8); break;
        case 16: GF_APPLY_TILE(16); break;
        default: GF_APPLY_TILE(32); break;
      }
#undef GF_APPLY_TILE
      GF_LAUNCH_CHECK(ctx);
      continue;
    }
    const dim3 grid(grid_for(nrows * T, kBlock)), block(kBlock);
    switch (T) {
      case 4: hipLaunchKernelGGL((k_apply<4, WT, IOT>), grid, block, 0, ctx->stream, sched, nrows, nbr->row_ptr, nbr->col, w, mask, uu, oo, nbr->n); break;
      case 8: hipLaunchKernelGGL((k_apply<8, WT, IOT>), grid, block, 0, ctx->stream, sched, nrows, nbr->row_ptr, nbr->col, w, mask, uu, oo, nbr->n); break;
      case 16: hipLaunchKernelGGL((k_apply<16, WT, IOT>), grid, block, 0, ctx->stream, sched, nrows, nbr->row_ptr, nbr->col, w, mask, uu, oo, nbr->n); break;
      case 32: hipLaunchKernelGGL((k_apply<32, WT, IOT>), grid, block, 0, ctx->stream, sched, nrows, nbr->row_ptr, nbr->col, w, mask, uu, oo, nbr->n); break;
      default: hipLaunchKernelGGL((k_apply<64, WT, IOT>), grid, block, 0, ctx->stream, sched, nrows, nbr->row_ptr, nbr->col, w, mask, uu, oo, nbr->n); break;
    }
    GF_LAUNCH_CHECK(ctx);
  }
  return GF_OK;
}
}  // namespace

// Team-size search for the application kernel (FP64 field), per launch unit.
gf_status tune_apply(gf_ctx *ctx, const gf_nbr *nbr, const void *w, gf_dtype wtype) {
  double *u = nullptr, *out = nullptr;
  if (hipMalloc(&u, sizeof(double) * nbr->n) != hipSuccess) return set_error(ctx, GF_ENOMEM, "tuning buffer");
  if (hipMalloc(&out, sizeof(double) * 4 * nbr->n) != hipSuccess) {
    (void)hipFree(u);
    return set_error(ctx, GF_ENOMEM, "tuning buffer");
  }
  (void)hipMemsetAsync(u, 0, sizeof(double) * nbr->n, ctx->stream);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int sizes[5] = {4, 8, 16, 32, 64};
  gf_status st = GF_OK;
  LaunchUnit units[2 * GF_NBAND];
  const int nu = launch_units(nbr, units);
  for (int q = 0; q < nu && !st; ++q) {
    float best = INFINITY;
    int bestT = ctx->ateam[units[q].model][units[q].band];
    // tiled blocks hold kTileRows teams: at most 32 lanes each
    const int nsizes = units[q].tiled ? 4 : 5;
    for (int t = 0; t < nsizes && !st; ++t) {
      float times[3];
      for (int rep = -1; rep < 3 && !st; ++rep) {
        if (rep >= 0) (void)hipEventRecord(e0, ctx->stream);
        st = (wtype == GF_F32) ? launch_apply<float, double>(ctx, nbr, w, 0xF, u, out, q, sizes[t])
                               : launch_apply<double, double>(ctx, nbr, w, 0xF, u, out, q, sizes[t]);
        if (rep >= 0) {
          (void)hipEventRecord(e1, ctx->stream);
          (void)hipEventSynchronize(e1);
          (void)hipEventElapsedTime(&times[rep], e0, e1);
        }
      }
      if (st) break;
      std::sort(times, times + 3);
      if (times[1] < best) { best = times[1]; bestT = sizes[t]; }
    }
    ctx->ateam[units[q].model][units[q].band] = bestT;
  }
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(u);
  (void)hipFree(out);
  return st;
}

extern "C" gf_status gf_apply_stencil(gf_ctx *ctx, const gf_nbr *nbr, gf_dtype wtype, const void *w, unsigned op_mask,
                                      gf_dtype io, const void *u, void *out) {
  if (!ctx) return GF_EINVAL;
  if (!nbr) return set_error(ctx, GF_EINVAL, "neighbour handle is NULL");
  gf_status st = check_nbr(ctx, nbr, nbr->n);
  if (st) return st;
  if (nbr->cross) return set_error(ctx, GF_EINVAL, "stencils live on same-model neighbourhoods");
  if (!w || !u || !out) return set_error(ctx, GF_EINVAL, "w, u and out are required");
  if (reinterpret_cast<uintptr_t>(w) & 15) return set_error(ctx, GF_EINVAL, "w must be 16-byte aligned");
  if ((op_mask & 0xF) == 0 || (op_mask & ~0xFu)) return set_error(ctx, GF_EINVAL, "op_mask must select 1..4 operators");
  if ((wtype != GF_F32 && wtype != GF_F64) || (io != GF_F32 && io != GF_F64))
    return set_error(ctx, GF_EINVAL, "unknown dtype");
  GF_HIP(ctx, hipSetDevice(ctx->device));
  if (wtype == GF_F32) {
    return io == GF_F64 ? launch_apply<float, double>(ctx, nbr, w, op_mask, u, out)
                        : launch_apply<float, float>(ctx, nbr, w, op_mask, u, out);
  }
  return io == GF_F64 ? launch_apply<double, double>(ctx, nbr, w, op_mask, u, out)
                      : launch_apply<double, float>(ctx, nbr, w, op_mask, u, out);
}

extern "C" gf_status gf_apply_stencil_adjoint(gf_ctx *ctx, const gf_nbr *nbr, gf_dtype wtype, const void *w,
                                              unsigned op_mask, const double *ybar, double *ubar) {
  if (!ctx) return GF_EINVAL;
  if (!nbr) return set_error(ctx, GF_EINVAL, "neighbour handle is NULL");
  gf_status st = check_nbr(ctx, nbr, nbr->n);
  if (st) return st;
  if (nbr->cross) return set_error(ctx, GF_EINVAL, "stencils live on same-model neighbourhoods");
  if (!w || !ybar || !ubar) return set_error(ctx, GF_EINVAL, "w, ybar and ubar are required");
  if (reinterpret_cast<uintptr_t>(w) & 15) return set_error(ctx, GF_EINVAL, "w must be 16-byte aligned");
  if ((op_mask & 0xF) == 0 || (op_mask & ~0xFu)) return set_error(ctx, GF_EINVAL, "op_mask must select 1..4 operators");
  if (wtype != GF_F32 && wtype != GF_F64) return set_error(ctx, GF_EINVAL, "unknown dtype");
  GF_HIP(ctx, hipSetDevice(ctx->device));
  if ((st = ensure_rev(ctx, const_cast<gf_nbr *>(nbr)))) return st;
  const dim3 block(kBlock);
  ProfScope prof(ctx, "apply_adjoint");
#define GF_ADJ(WT, K)                                                                                            \
  hipLaunchKernelGGL((k_apply_adjoint<WT, K>), dim3(grid_for(nbr->n * adj_team<WT>(K), kBlock)), block, 0,         \
                     ctx->stream, nbr->row_ptr, nbr->col, nbr->rev, w, op_mask, ybar, nbr->n, ubar)
#define GF_ADJ_K(WT)                       \
  switch (__builtin_popcount(op_mask)) {   \
    case 1: GF_ADJ(WT, 1); break;          \
    case 2: GF_ADJ(WT, 2); break;          \
    case 3: GF_ADJ(WT, 3); break;          \
    default: GF_ADJ(WT, 4); break;         \
  }
  if (wtype == GF_F32) {
    GF_ADJ_K(float)
  } else {
    GF_ADJ_K(double)
  }
#undef GF_ADJ_K
#undef GF_ADJ
  GF_LAUNCH_CHECK(ctx);
  return GF_OK;
}
