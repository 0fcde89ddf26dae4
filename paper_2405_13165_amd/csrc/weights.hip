// Second-order GFDM stencils (Eq. GFDM_Definition) and their fused
// application.
//
// Batched path: particles are grouped by model (10 monomials in 3D, 6 on the
// film) and by neighbour-count band; inside a group they are taken in Morton
// order.  Each particle is handled by a team of T lanes of a wave: the lanes
// stride over the neighbours, accumulate their share of the packed FP64 Gram
// matrix G = M^T W M in registers, and a butterfly sum gives every lane the
// full G.  The team factors G (LDL^T), spreads the columns of G^{-1} over
// its lanes to get the exact 1-norm condition number and the four target
// solutions, and a second pass over the neighbours writes
// c_j = w_j phi_j^T lambda (and, fused, applies the stencils to a field).
// Particles whose condition number exceeds kappa_max, or whose pivots are not
// positive, are queued and re-solved by a Householder QR of sqrt(W) M (one
// wave per particle), which also decides rank deficiency.
//
// Plain path: one work-item per particle in the caller's order, the same
// FP64 arithmetic, FP64 output.
#include "stencil_common.h"

using namespace gfdm_dev;

namespace {
constexpr int kBlock = 256;
constexpr int kQrBlock = 64;
constexpr int kQrStride = 15;  // per neighbour: 10 columns, 4 targets, sqrt(w)

struct WArgs {
  const double *x, *y, *z, *h, *nx, *ny, *nz;
  const int8_t *model;
  const int64_t *row_ptr;
  const int32_t *col;
  const int32_t *sched;
  int64_t nrows;
  int64_t n;
  WeightFn wf;
  double kappa_max;
  void *w_out;
  int8_t *status;
  float *kappa_out;
  int32_t *queue;
  int32_t *qcount;
  const double *u;
  double *y_out;
  unsigned mask;
};

template <int OUT>
__device__ inline void store_w(void *w, int64_t k, double c0, double c1, double c2, double c3) {
  if constexpr (OUT == GF_F32) {
    reinterpret_cast<float4 *>(w)[k] = make_float4((float)c0, (float)c1, (float)c2, (float)c3);
  } else {
    double2 *p = reinterpret_cast<double2 *>(w) + 2 * k;
    p[0] = make_double2(c0, c1);
    p[1] = make_double2(c2, c3);
  }
}

__device__ inline void store_fused(const WArgs &a, int32_t i, const double acc[4]) {
  int q = 0;
  for (int s = 0; s < 4; ++s)
    if (a.mask & (1u << s)) a.y_out[(int64_t)(q++) * a.n + i] = acc[s];
}

template <int M>
__device__ inline void row_geom(const WArgs &a, int32_t i, RowGeom &g) {
  g.xi = a.x[i]; g.yi = a.y[i]; g.zi = a.z[i]; g.hi = a.h[i];
  g.inv_h = 1.0 / g.hi;
  if constexpr (M == 6) tangent_frame(a.nx[i], a.ny[i], a.nz[i], g.t1, g.t2);
}

template <int M, int T, int OUT, bool FUSED, bool FASTW>
__device__ void weights_row(const WArgs &a, int32_t i, int lane) {
  const int64_t b = a.row_ptr[i];
  const int n = (int)(a.row_ptr[i + 1] - b);
  if (n < M) {
    if (a.w_out)
      for (int k = lane; k < n; k += T) store_w<OUT>(a.w_out, b + k, 0.0, 0.0, 0.0, 0.0);
    if (lane == 0) {
      if (a.status) a.status[i] = 3;
      if (a.kappa_out) a.kappa_out[i] = 0.0f;
      if constexpr (FUSED) {
        const double z[4] = {0.0, 0.0, 0.0, 0.0};
        store_fused(a, i, z);
      }
    }
    return;
  }
  RowGeom g;
  row_geom<M>(a, i, g);
  constexpr int NP = npack(M);
  double G[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) G[p] = 0.0;
#pragma unroll 1
  for (int k = lane; k < n; k += T) {
    const int32_t j = a.col[b + k];
    const double dx = a.x[j] - g.xi, dy = a.y[j] - g.yi, dz = a.z[j] - g.zi;
    const double r = 0.5 * (g.hi + a.h[j]);
    const double w = support_weight<FASTW>(dx * dx + dy * dy + dz * dz, r, a.wf);
    double phi[M];
    monomials<M>(g, dx, dy, dz, phi);
    gram_add<M>(G, phi, w);
  }
  if constexpr (T > 1) {
#pragma unroll
    for (int p = 0; p < NP; ++p) G[p] = team_sum(G[p], T);
  }
  double lam[4][M];
  double kappa;
  const bool ok = team_solve<M, T>(G, lane, lam, &kappa);
  if (lane == 0 && a.kappa_out) a.kappa_out[i] = (float)kappa;
  if (!ok || !(kappa <= a.kappa_max)) {
    if (lane == 0) {
      if (a.status) a.status[i] = 1;
      const int32_t q = atomicAdd(a.qcount, 1);
      a.queue[q] = i;
    }
    return;
  }
  // physical scaling: first derivatives / h, Laplacian / h^2
  const double ih2 = g.inv_h * g.inv_h;
#pragma unroll
  for (int r = 0; r < M; ++r) {
    lam[0][r] *= g.inv_h; lam[1][r] *= g.inv_h; lam[2][r] *= g.inv_h; lam[3][r] *= ih2;
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  double ui = 0.0;
  if constexpr (FUSED) ui = a.u[i];
#pragma unroll 1
  for (int k = lane; k < n; k += T) {
    const int32_t j = a.col[b + k];
    const double dx = a.x[j] - g.xi, dy = a.y[j] - g.yi, dz = a.z[j] - g.zi;
    const double r = 0.5 * (g.hi + a.h[j]);
    const double w = support_weight<FASTW>(dx * dx + dy * dy + dz * dz, r, a.wf);
    double phi[M];
    monomials<M>(g, dx, dy, dz, phi);
    double c[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < M; ++q) t += phi[q] * lam[s][q];
      c[s] = w * t;
    }
    if constexpr (M == 6) {
      const double cu = c[0], cv = c[1];
      c[0] = g.t1[0] * cu + g.t2[0] * cv;
      c[1] = g.t1[1] * cu + g.t2[1] * cv;
      c[2] = g.t1[2] * cu + g.t2[2] * cv;
    }
    if (a.w_out) store_w<OUT>(a.w_out, b + k, c[0], c[1], c[2], c[3]);
    if constexpr (FUSED) {
      if (j != i) {
        double du = a.u[j] - ui;
        if constexpr (OUT == GF_F32) {
          // apply the weights as stored
#pragma unroll
          for (int s = 0; s < 4; ++s) acc[s] += (double)(float)c[s] * du;
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s) acc[s] += c[s] * du;
        }
      }
    }
  }
  if constexpr (FUSED) {
    if constexpr (T > 1) {
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[s] = team_sum(acc[s], T);
    }
    if (lane == 0) store_fused(a, i, acc);
  }
  if (lane == 0 && a.status) a.status[i] = 0;
}

template <int M, int T, int OUT, bool FUSED, bool FASTW>
__global__ void __launch_bounds__(kBlock) k_weights_team(WArgs a) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t team = gt / T;
  const int lane = (int)(gt % T);
  if (team >= a.nrows) return;
  weights_row<M, T, OUT, FUSED, FASTW>(a, a.sched[team], lane);
}

__global__ void __launch_bounds__(kBlock) k_weights_plain(WArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.nrows) return;
  if (a.model[i] == GF_MODEL_FILM)
    weights_row<6, 1, GF_F64, false, false>(a, (int32_t)i, 0);
  else
    weights_row<10, 1, GF_F64, false, false>(a, (int32_t)i, 0);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Householder QR of A = sqrt(W) M for the queued particles: one wave each.
// Columns live in a per-block slice of global scratch (column-major, n rows).
template <int OUT, bool FUSED, bool FASTW>
__global__ void __launch_bounds__(kQrBlock) k_weights_qr(WArgs a, double *scratch, int64_t slice) {
  const int lane = threadIdx.x;
  double *A = scratch + (int64_t)blockIdx.x * slice;
  __shared__ double R[10][10];
  __shared__ double vtv[10];
  __shared__ double zt[4][10];
  const int qn = *a.qcount;
  for (int q = blockIdx.x; q < qn; q += gridDim.x) {
    const int32_t i = a.queue[q];
    const int64_t b = a.row_ptr[i];
    const int n = (int)(a.row_ptr[i + 1] - b);
    const bool film = a.model[i] == GF_MODEL_FILM;
    const int M = film ? 6 : 10;
    RowGeom g;
    g.xi = a.x[i]; g.yi = a.y[i]; g.zi = a.z[i]; g.hi = a.h[i]; g.inv_h = 1.0 / g.hi;
    if (film) tangent_frame(a.nx[i], a.ny[i], a.nz[i], g.t1, g.t2);
    double *SW = A + 14 * (int64_t)n;
    for (int r = lane; r < n; r += kQrBlock) {
      const int32_t j = a.col[b + r];
      const double dx = a.x[j] - g.xi, dy = a.y[j] - g.yi, dz = a.z[j] - g.zi;
      const double rr = 0.5 * (g.hi + a.h[j]);
      const double w = support_weight<FASTW>(dx * dx + dy * dy + dz * dz, rr, a.wf);
      const double sw = sqrt(w);
      SW[r] = sw;
      double phi[10];
      if (film) monomials<6>(g, dx, dy, dz, phi); else monomials<10>(g, dx, dy, dz, phi);
      for (int c = 0; c < M; ++c) A[(int64_t)c * n + r] = sw * phi[c];
    }
    __syncthreads();
    for (int k = 0; k < M; ++k) {
      double part = 0.0;
      for (int r = k + lane; r < n; r += kQrBlock) part += A[(int64_t)k * n + r] * A[(int64_t)k * n + r];
      const double nrm2 = wave_sum(part);
      const double akk = A[(int64_t)k * n + k];
      const double alpha = (akk > 0.0) ? -sqrt(nrm2) : sqrt(nrm2);
      const double vv = 2.0 * (nrm2 - akk * alpha);
      __syncthreads();
      if (lane == 0) {
        A[(int64_t)k * n + k] = akk - alpha;
        R[k][k] = alpha;
        vtv[k] = vv;
      }
      __syncthreads();
      for (int c = k + 1; c < M; ++c) {
        double sp = 0.0;
        for (int r = k + lane; r < n; r += kQrBlock) sp += A[(int64_t)k * n + r] * A[(int64_t)c * n + r];
        const double s = wave_sum(sp);
        if (vv > 0.0) {
          const double f = 2.0 * s / vv;
          for (int r = k + lane; r < n; r += kQrBlock) A[(int64_t)c * n + r] -= f * A[(int64_t)k * n + r];
        }
      }
      __syncthreads();
    }
    for (int t = lane; t < M * M; t += kQrBlock) {
      const int rr = t / M, cc = t % M;
      if (cc > rr) R[rr][cc] = A[(int64_t)cc * n + rr];
      else if (cc < rr) R[rr][cc] = 0.0;
    }
    __syncthreads();
    double rmax = 0.0, rmin = INFINITY;
    for (int k = 0; k < M; ++k) {
      rmax = fmax(rmax, fabs(R[k][k]));
      rmin = fmin(rmin, fabs(R[k][k]));
    }
    const bool full_rank = rmin > 1e-12 * rmax;
    if (!full_rank) {
      if (a.w_out)
        for (int r = lane; r < n; r += kQrBlock) store_w<OUT>(a.w_out, b + r, 0.0, 0.0, 0.0, 0.0);
      if (lane == 0) {
        if (a.status) a.status[i] = 2;
        if constexpr (FUSED) {
          const double z[4] = {0.0, 0.0, 0.0, 0.0};
          store_fused(a, i, z);
        }
      }
      __syncthreads();
      continue;
    }
    // z_s = R^{-T} d_s (lanes 0..3, one target each)
    if (lane < 4) {
      const int s = lane;
      double d[10];
      for (int r = 0; r < 10; ++r) d[r] = 0.0;
      if (!film) {
        if (s < 3) d[s + 1] = 1.0; else { d[4] = 2.0; d[5] = 2.0; d[6] = 2.0; }
      } else {
        if (s < 2) d[s + 1] = 1.0; else if (s == 3) { d[3] = 2.0; d[4] = 2.0; }
      }
      for (int r = 0; r < M; ++r) {
        double t = d[r];
        for (int c = 0; c < r; ++c) t -= R[c][r] * zt[s][c];
        zt[s][r] = t / R[r][r];
      }
    }
    __syncthreads();
    double *Y = A + 10 * (int64_t)n;
    for (int r = lane; r < n; r += kQrBlock)
      for (int s = 0; s < 4; ++s) Y[(int64_t)s * n + r] = (r < M) ? zt[s][r] : 0.0;
    __syncthreads();
    // y_s = H_0 H_1 ... H_{M-1} [z_s; 0]
    for (int k = M - 1; k >= 0; --k) {
      const double vv = vtv[k];
      double sp[4] = {0.0, 0.0, 0.0, 0.0};
      for (int r = k + lane; r < n; r += kQrBlock) {
        const double v = A[(int64_t)k * n + r];
        for (int s = 0; s < 4; ++s) sp[s] += v * Y[(int64_t)s * n + r];
      }
      double f[4];
      for (int s = 0; s < 4; ++s) f[s] = (vv > 0.0) ? 2.0 * wave_sum(sp[s]) / vv : 0.0;
      for (int r = k + lane; r < n; r += kQrBlock) {
        const double v = A[(int64_t)k * n + r];
        for (int s = 0; s < 4; ++s) Y[(int64_t)s * n + r] -= f[s] * v;
      }
      __syncthreads();
    }
    const double ih = g.inv_h, ih2 = g.inv_h * g.inv_h;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    double ui = 0.0;
    if constexpr (FUSED) ui = a.u[i];
    for (int r = lane; r < n; r += kQrBlock) {
      const double sw = SW[r];
      double c[4];
      c[0] = sw * Y[r] * ih;
      c[1] = sw * Y[(int64_t)n + r] * ih;
      c[2] = sw * Y[2 * (int64_t)n + r] * ih;
      c[3] = sw * Y[3 * (int64_t)n + r] * ih2;
      if (film) {
        const double cu = c[0], cv = c[1];
        c[0] = g.t1[0] * cu + g.t2[0] * cv;
        c[1] = g.t1[1] * cu + g.t2[1] * cv;
        c[2] = g.t1[2] * cu + g.t2[2] * cv;
      }
      if (a.w_out) store_w<OUT>(a.w_out, b + r, c[0], c[1], c[2], c[3]);
      if constexpr (FUSED) {
        const int32_t j = a.col[b + r];
        if (j != i) {
          const double du = a.u[j] - ui;
          for (int s = 0; s < 4; ++s) acc[s] += ((OUT == GF_F32) ? (double)(float)c[s] : c[s]) * du;
        }
      }
    }
    if constexpr (FUSED) {
      for (int s = 0; s < 4; ++s) acc[s] = wave_sum(acc[s]);
      if (lane == 0) store_fused(a, i, acc);
    }
    if (lane == 0 && a.status) a.status[i] = 1;
    __syncthreads();
  }
}

__global__ void k_zero_i32(int32_t *p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

// counts of each status and the largest finite condition estimate
__global__ void __launch_bounds__(1024) k_ls_stats(const int8_t *__restrict__ status, const float *__restrict__ kappa,
                                                   int64_t n, long long *out_counts, double *out_kmax) {
  __shared__ long long cnt[4];
  __shared__ double km[1024];
  if (threadIdx.x < 4) cnt[threadIdx.x] = 0;
  __syncthreads();
  long long c[4] = {0, 0, 0, 0};
  double k = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    int s = status[i];
    if (s >= 0 && s < 4) c[s]++;
    if (kappa) {
      double kv = kappa[i];
      if (isfinite(kv)) k = fmax(k, kv);
    }
  }
  for (int s = 0; s < 4; ++s) atomicAdd((unsigned long long *)&cnt[s], (unsigned long long)c[s]);
  km[threadIdx.x] = k;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) km[threadIdx.x] = fmax(km[threadIdx.x], km[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x < 4) out_counts[threadIdx.x] = cnt[threadIdx.x];
  if (threadIdx.x == 0) *out_kmax = km[0];
}

// team size per (model, neighbour-count band)
int team_for(int model, int band) {
  static const int bulk[GF_NBAND] = {4, 8, 8, 16};
  static const int film[GF_NBAND] = {4, 4, 8, 16};
  return model ? film[band] : bulk[band];
}

const char *team_kernel_name(int M, int T, bool fused) {
  if (M == 10) {
    if (fused) return T == 4 ? "weights_apply_3d_t4" : T == 8 ? "weights_apply_3d_t8" : "weights_apply_3d_t16";
    return T == 4 ? "weights_3d_t4" : T == 8 ? "weights_3d_t8" : "weights_3d_t16";
  }
  if (fused) return T == 4 ? "weights_apply_film_t4" : T == 8 ? "weights_apply_film_t8" : "weights_apply_film_t16";
  return T == 4 ? "weights_film_t4" : T == 8 ? "weights_film_t8" : "weights_film_t16";
}

template <int M, int OUT, bool FUSED, bool FASTW>
gf_status launch_team(gf_ctx *ctx, const WArgs &a, int T) {
  ProfScope prof(ctx, team_kernel_name(M, T, FUSED));
  const int64_t threads = a.nrows * (int64_t)T;
  const dim3 grid(grid_for(threads, kBlock)), block(kBlock);
  switch (T) {
    case 4: hipLaunchKernelGGL((k_weights_team<M, 4, OUT, FUSED, FASTW>), grid, block, 0, ctx->stream, a); break;
    case 8: hipLaunchKernelGGL((k_weights_team<M, 8, OUT, FUSED, FASTW>), grid, block, 0, ctx->stream, a); break;
    case 16: hipLaunchKernelGGL((k_weights_team<M, 16, OUT, FUSED, FASTW>), grid, block, 0, ctx->stream, a); break;
    default: return set_error(ctx, GF_EINVAL, "unsupported team size %d", T);
  }
  GF_LAUNCH_CHECK(ctx);
  return GF_OK;
}

template <int OUT, bool FUSED, bool FASTW>
gf_status launch_batched(gf_ctx *ctx, const gf_nbr *nbr, WArgs a) {
  for (int m = 0; m < 2; ++m) {
    for (int band = 0; band < GF_NBAND; ++band) {
      const int gsel = m * GF_NBAND + band;
      const int64_t s0 = nbr->group_start[gsel], s1 = nbr->group_start[gsel + 1];
      if (s1 <= s0) continue;
      a.sched = nbr->grouped + s0;
      a.nrows = s1 - s0;
      const int T = team_for(m, band);
      gf_status st = (m == 0) ? launch_team<10, OUT, FUSED, FASTW>(ctx, a, T) : launch_team<6, OUT, FUSED, FASTW>(ctx, a, T);
      if (st) return st;
    }
  }
  return GF_OK;
}

struct WeightsScratch {
  int32_t *queue, *qcount;
  double *qr;
  int64_t qr_slice;
  int qr_blocks;
  int8_t *status;
  float *kappa;
  long long *counts;
  double *kmax;
};

gf_status weights_common(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr, gf_prec prec,
                         const gf_ls_params *params, gf_dtype wtype, void *w_out, int8_t *status_n, float *kappa_n,
                         gf_ls_stats *stats, bool fused, unsigned op_mask, const double *u, double *out) {
  gf_status st = check_particles(ctx, p, false, false);
  if (st) return st;
  if ((st = check_nbr(ctx, nbr, p->n))) return st;
  if (nbr->cross) return set_error(ctx, GF_EINVAL, "stencils need same-model neighbourhoods");
  if (prec != GF_PLAIN_F64 && prec != GF_BATCHED) return set_error(ctx, GF_EINVAL, "unknown precision mode %d", (int)prec);
  if (wtype != GF_F64 && wtype != GF_F32) return set_error(ctx, GF_EINVAL, "unknown weight type %d", (int)wtype);
  if (prec == GF_PLAIN_F64 && wtype != GF_F64) return set_error(ctx, GF_EINVAL, "GF_PLAIN_F64 writes FP64 weights");
  if (!w_out && !fused) return set_error(ctx, GF_EINVAL, "w_out is NULL");
  if (fused && (!u || !out || (op_mask & 0xF) == 0 || (op_mask & ~0xFu)))
    return set_error(ctx, GF_EINVAL, "fused application needs u, out and a non-empty op mask");
  gf_ls_params prm;
  gf_ls_params_default(&prm);
  if (params) prm = *params;
  if (!(prm.alpha_w > 0.0) || !(prm.kappa_max > 0.0)) return set_error(ctx, GF_EINVAL, "alpha_w and kappa_max must be positive");
  bool has_film = nbr->group_start[2 * GF_NBAND] > nbr->group_start[GF_NBAND];
  if (has_film && (!p->nx || !p->ny || !p->nz)) return set_error(ctx, GF_EINVAL, "film particles need normals");
  const int64_t n = p->n;
  const int qr_blocks = (int)std::min<int64_t>(1024, n);
  const int64_t slice = (int64_t)kQrStride * std::max(nbr->max_row, 1);
  Arena ar;
  if ((st = ensure_scratch(ctx, arena_bytes({sizeof(int32_t) * n, 64, sizeof(double) * slice * qr_blocks, (size_t)n,
                                             sizeof(float) * n, 64, 64}),
                           &ar)))
    return st;
  WeightsScratch ws;
  ws.queue = ar.take<int32_t>(n);
  ws.qcount = ar.take<int32_t>(16);
  ws.qr = ar.take<double>(slice * qr_blocks);
  ws.status = ar.take<int8_t>(n);
  ws.kappa = ar.take<float>(n);
  ws.counts = ar.take<long long>(4);
  ws.kmax = ar.take<double>(1);
  WArgs a;
  a.x = p->x; a.y = p->y; a.z = p->z; a.h = p->h; a.nx = p->nx; a.ny = p->ny; a.nz = p->nz; a.model = p->model;
  a.row_ptr = nbr->row_ptr; a.col = nbr->col; a.sched = nullptr; a.nrows = n; a.n = n;
  a.wf = make_weight_fn(prm.alpha_w);
  a.kappa_max = prm.kappa_max;
  a.w_out = w_out;
  a.status = status_n ? status_n : ((stats) ? ws.status : nullptr);
  a.kappa_out = kappa_n ? kappa_n : ((stats) ? ws.kappa : nullptr);
  a.queue = ws.queue;
  a.qcount = ws.qcount;
  a.u = u; a.y_out = out; a.mask = op_mask;
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, ctx->stream, ws.qcount, 16);
  GF_LAUNCH_CHECK(ctx);
  const bool f32 = wtype == GF_F32;
  if (prec == GF_PLAIN_F64) {
    ProfScope prof(ctx, "weights_plain_f64");
    hipLaunchKernelGGL(k_weights_plain, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, a);
    GF_LAUNCH_CHECK(ctx);
  } else if (!fused) {
    st = f32 ? launch_batched<GF_F32, false, true>(ctx, nbr, a) : launch_batched<GF_F64, false, false>(ctx, nbr, a);
    if (st) return st;
  } else {
    st = f32 ? launch_batched<GF_F32, true, true>(ctx, nbr, a) : launch_batched<GF_F64, true, false>(ctx, nbr, a);
    if (st) return st;
  }
  // fallback queue (sized on the device; the grid loops over it)
  ProfScope prof_qr(ctx, "weights_qr_fallback");
  if (!fused) {
    if (f32) hipLaunchKernelGGL((k_weights_qr<GF_F32, false, true>), dim3(qr_blocks), dim3(kQrBlock), 0, ctx->stream, a, ws.qr, slice);
    else hipLaunchKernelGGL((k_weights_qr<GF_F64, false, false>), dim3(qr_blocks), dim3(kQrBlock), 0, ctx->stream, a, ws.qr, slice);
  } else {
    if (f32) hipLaunchKernelGGL((k_weights_qr<GF_F32, true, true>), dim3(qr_blocks), dim3(kQrBlock), 0, ctx->stream, a, ws.qr, slice);
    else hipLaunchKernelGGL((k_weights_qr<GF_F64, true, false>), dim3(qr_blocks), dim3(kQrBlock), 0, ctx->stream, a, ws.qr, slice);
  }
  GF_LAUNCH_CHECK(ctx);
  if (stats) {
    hipLaunchKernelGGL(k_ls_stats, dim3(1), dim3(1024), 0, ctx->stream, a.status, a.kappa_out, n, ws.counts, ws.kmax);
    GF_LAUNCH_CHECK(ctx);
    if ((st = ensure_host(ctx, 4096))) return st;
    GF_HIP(ctx, hipMemcpyAsync(ctx->host_pinned, ws.counts, 4 * sizeof(long long), hipMemcpyDeviceToHost, ctx->stream));
    GF_HIP(ctx, hipMemcpyAsync((char *)ctx->host_pinned + 64, ws.kmax, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    GF_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const long long *hc = (const long long *)ctx->host_pinned;
    stats->n_ok = hc[0];
    stats->n_fallback = hc[1];
    stats->n_rank_deficient = hc[2];
    stats->n_too_few = hc[3];
    stats->kappa_max_seen = *(const double *)((const char *)ctx->host_pinned + 64);
  }
  return GF_OK;
}
}  // namespace

extern "C" void gf_ls_params_default(gf_ls_params *p) {
  if (!p) return;
  p->alpha_w = 8.0;
  p->kappa_max = 1e5;
}

extern "C" gf_status gf_gfdm_weights(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr, gf_prec prec,
                                     const gf_ls_params *params, gf_dtype wtype, void *w_out, int8_t *status_n,
                                     float *kappa_n, gf_ls_stats *stats) {
  if (!ctx) return GF_EINVAL;
  return weights_common(ctx, p, nbr, prec, params, wtype, w_out, status_n, kappa_n, stats, false, 0, nullptr, nullptr);
}

extern "C" gf_status gf_gfdm_weights_apply(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr,
                                           const gf_ls_params *params, gf_dtype wtype, void *w_out, unsigned op_mask,
                                           const double *u, double *out, int8_t *status_n) {
  if (!ctx) return GF_EINVAL;
  return weights_common(ctx, p, nbr, GF_BATCHED, params, wtype, w_out, status_n, nullptr, nullptr, true, op_mask, u,
                        out);
}
