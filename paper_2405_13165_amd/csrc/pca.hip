// Local PCA of every neighbourhood and the transition flags of Sec. 4.
//
// A team of kTeam lanes per particle builds the 3x3 covariance in two passes
// (centroid, then centred second moments) from offsets relative to the
// particle itself, so an exactly planar neighbourhood yields an exactly zero
// third eigenvalue.  Rows with at most 128 neighbours are processed by
// neighbour tiles: a block takes kPcaTiles consecutive tiles, stages each
// tile's distinct neighbours (position, index and kind) in LDS in turn, and
// keeps the covariances and neighbour-kind counts of all its rows in LDS;
// then every thread of the block runs the eigen solve and the classification
// of one row, so the serial 3x3 Jacobi solves use every lane.  Rows with more
// neighbours gather from global memory, and one lane of the team solves.
#include "stencil_common.h"

using namespace gfdm_dev;

namespace {
constexpr int kBlock = 256;
constexpr int kTeam = 4;

// Symmetric 3x3 eigen-decomposition by Jacobi rotations (each rotation
// annihilates one off-diagonal entry; sweeps until the off-diagonal mass is
// negligible).  a: packed symmetric [a00 a01 a02 a11 a12 a22].
__device__ void sym3_eigen(double a00, double a01, double a02, double a11, double a12, double a22,
                           double lam[3], double V[3][3]) {
  double A[3][3] = {{a00, a01, a02}, {a01, a11, a12}, {a02, a12, a22}};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) V[r][c] = (r == c) ? 1.0 : 0.0;
  const double scale = sqrt(a00 * a00 + a11 * a11 + a22 * a22 + 2.0 * (a01 * a01 + a02 * a02 + a12 * a12));
  for (int sweep = 0; sweep < 32; ++sweep) {
    double off = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
    if (off == 0.0 || off <= 1e-17 * scale) break;
    for (int t = 0; t < 3; ++t) {
      const int p = (t == 2) ? 1 : 0;
      const int q = (t == 0) ? 1 : 2;
      const double apq = A[p][q];
      if (apq == 0.0) continue;
      // tan of the rotation angle, smaller root of t^2 + 2 t cot(2phi) - 1 = 0
      const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
      const double tn = copysign(1.0, tau) / (fabs(tau) + sqrt(1.0 + tau * tau));
      const double c = 1.0 / sqrt(1.0 + tn * tn);
      const double s = tn * c;
      for (int k = 0; k < 3; ++k) {
        const double akp = A[k][p], akq = A[k][q];
        A[k][p] = c * akp - s * akq;
        A[k][q] = s * akp + c * akq;
      }
      for (int k = 0; k < 3; ++k) {
        const double apk = A[p][k], aqk = A[q][k];
        A[p][k] = c * apk - s * aqk;
        A[q][k] = s * apk + c * aqk;
      }
      A[p][q] = 0.0;
      A[q][p] = 0.0;
      for (int k = 0; k < 3; ++k) {
        const double vkp = V[k][p], vkq = V[k][q];
        V[k][p] = c * vkp - s * vkq;
        V[k][q] = s * vkp + c * vkq;
      }
    }
  }
  lam[0] = A[0][0];
  lam[1] = A[1][1];
  lam[2] = A[2][2];
}

struct PcaArgs {
  const double *x, *y, *z;
  const int8_t *model, *kind;
  const double *nx, *ny, *nz;
  const int64_t *row_ptr;
  const int32_t *col;
  const int32_t *sched;  // rows of the launch (a range of the grouped order)
  int64_t nrows;
  const double *film_height, *h3d;
  const uint8_t *prev, *user;
  double eps_max, cos_theta;
  int literal;
  double *lam, *w3, *eps;
  uint8_t *raw;
};

// eigen decomposition of the covariance, outputs and the flags of particle i
__device__ void pca_finish(const PcaArgs &a, int32_t i, int n_int, int n_fs, double c00, double c01, double c02,
                           double c11, double c12, double c22) {
  double lam[3], V[3][3];
  sym3_eigen(c00, c01, c02, c11, c12, c22, lam, V);
  // order descending; equal values keep their original order
  int o0 = 0, o1 = 1, o2 = 2, t;
  if (lam[o0] < lam[o1]) { t = o0; o0 = o1; o1 = t; }
  if (lam[o1] < lam[o2]) { t = o1; o1 = o2; o2 = t; }
  if (lam[o0] < lam[o1]) { t = o0; o0 = o1; o1 = t; }
  double w[3] = {V[0][o2], V[1][o2], V[2][o2]};
  const double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  int big = 0;
  if (fabs(w[1]) > fabs(w[big])) big = 1;
  if (fabs(w[2]) > fabs(w[big])) big = 2;
  const double sg = (w[big] < 0.0) ? -1.0 : 1.0;
  for (int r = 0; r < 3; ++r) w[r] = sg * w[r] / wn;
  const double l0 = lam[o0], l1 = lam[o1], l2 = lam[o2];
  const double den = l0 + l1;
  const double epsl = (den == 0.0) ? INFINITY : 2.0 * l2 / den;
  if (a.lam) { a.lam[3 * i] = l0; a.lam[3 * i + 1] = l1; a.lam[3 * i + 2] = l2; }
  if (a.w3) { a.w3[3 * i] = w[0]; a.w3[3 * i + 1] = w[1]; a.w3[3 * i + 2] = w[2]; }
  if (a.eps) a.eps[i] = epsl;
  if (!a.raw) return;
  // ---- transition detection (Alg. 2, Eq. 2Dto3Dcond), smoothing rule 2
  uint8_t f = 0;
  const bool user = a.user && a.user[i];
  const int m = a.model[i];
  if (m == GF_MODEL_BULK && a.kind[i] == GF_KIND_WALL) {
    if (n_fs > 0) {
      const double nd = fabs(a.nx[i] * w[0] + a.ny[i] * w[1] + a.nz[i] * w[2]);
      const bool eig_ok = epsl < a.eps_max;
      const bool vec_ok = a.literal ? (nd < a.cos_theta) : (nd >= a.cos_theta);
      if ((eig_ok && vec_ok) || user) f = 1;
    } else if (n_int == 0) {
      f = 1;
    }
  } else if (m == GF_MODEL_FILM) {
    const bool hcrit = (a.film_height && a.h3d) ? (a.film_height[i] >= a.h3d[i]) : false;
    if (hcrit || user) f = 2;
  }
  if (a.prev && a.prev[i]) f = 0;
  a.raw[i] = f;
}

// A neighbour as (x, y, z, 4 index + kind code): the index and the code
// (kind 0..2, anything else 3) are exact in the FP64 field.
__device__ inline double pca_code(const PcaArgs &a, int32_t j) {
  const int k = a.kind ? (int)a.kind[j] : 0;
  return (double)(4 * (int64_t)j + ((k >= 0 && k <= 2) ? k : 3));
}
struct PcaTile {   // staged in LDS, addressed by slot[]
  const double4 *sp;
  const uint16_t *slot;
  __device__ double4 operator()(const PcaArgs &, int64_t k) const { return sp[slot[k]]; }
};
struct PcaGlobal {
  __device__ double4 operator()(const PcaArgs &a, int64_t k) const {
    const int32_t j = a.col[k];
    return make_double4(a.x[j], a.y[j], a.z[j], pca_code(a, j));
  }
};

// covariance (c00 c01 c02 c11 c12 c22) and the counts of interior and
// free-surface neighbours of row i, complete on every lane of the team
template <class F>
__device__ void pca_cov(const PcaArgs &a, int32_t i, int lane, const F &fetch, double c[6], int &n_int, int &n_fs) {
  const int64_t b = a.row_ptr[i], e = a.row_ptr[i + 1];
  const double xi = a.x[i], yi = a.y[i], zi = a.z[i];
  const bool need_kinds = a.raw && a.kind;
  double mx = 0.0, my = 0.0, mz = 0.0;
  n_int = 0;
  n_fs = 0;
  for (int64_t k = b + lane; k < e; k += kTeam) {
    const double4 pj = fetch(a, k);
    mx += pj.x - xi;
    my += pj.y - yi;
    mz += pj.z - zi;
    if (need_kinds) {
      const int64_t code = (int64_t)pj.w;
      if ((code >> 2) != i) {
        const int kj = (int)(code & 3);
        n_int += (kj == GF_KIND_INTERIOR);
        n_fs += (kj == GF_KIND_FREE_SURFACE);
      }
    }
  }
  mx = team_sum(mx, kTeam);
  my = team_sum(my, kTeam);
  mz = team_sum(mz, kTeam);
  n_int = team_sum(n_int, kTeam);
  n_fs = team_sum(n_fs, kTeam);
  const double inv = 1.0 / (double)(e - b);
  mx *= inv; my *= inv; mz *= inv;
#pragma unroll
  for (int q = 0; q < 6; ++q) c[q] = 0.0;
  for (int64_t k = b + lane; k < e; k += kTeam) {
    const double4 pj = fetch(a, k);
    const double dx = (pj.x - xi) - mx, dy = (pj.y - yi) - my, dz = (pj.z - zi) - mz;
    c[0] += dx * dx; c[1] += dx * dy; c[2] += dx * dz;
    c[3] += dy * dy; c[4] += dy * dz; c[5] += dz * dz;
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) c[q] = team_sum(c[q], kTeam);
}

// Tiled rows: kPcaTiles consecutive neighbour tiles per block (kTileRows
// teams of kTeam lanes, so a block has as many threads as its rows).
constexpr int kPcaTiles = kTeam;
constexpr int kPcaRows = kTileRows * kPcaTiles;  // rows of a block = its threads
__global__ void __launch_bounds__(kTileRows * kTeam) k_pca_tile(PcaArgs a, const int64_t *__restrict__ toff,
                                                                const int32_t *__restrict__ tu,
                                                                const uint16_t *__restrict__ slot, int64_t tile0,
                                                                int64_t ntiles, int cap) {
  extern __shared__ double4 s_pos[];
  __shared__ double s_cov[6][kPcaRows];
  __shared__ int s_cnt[2][kPcaRows];
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int team = threadIdx.x / kTeam, lane = threadIdx.x % kTeam;
  for (int q = 0; q < kPcaTiles; ++q) {
    const int64_t tl = blk * kPcaTiles + q;
    if (tl >= ntiles) break;  // uniform over the block
    const int64_t u0 = toff[tile0 + tl];
    const int cnt = (int)(toff[tile0 + tl + 1] - u0);
    const bool staged = cnt <= cap;
    if (staged) {
      for (int s = threadIdx.x; s < cnt; s += blockDim.x) {
        const int32_t j = tu[u0 + s];
        s_pos[s] = make_double4(a.x[j], a.y[j], a.z[j], pca_code(a, j));
      }
    }
    __syncthreads();
    const int64_t r = tl * kTileRows + team;
    if (r < a.nrows) {
      double c[6];
      int n_int, n_fs;
      if (staged) pca_cov(a, a.sched[r], lane, PcaTile{s_pos, slot}, c, n_int, n_fs);
      else pca_cov(a, a.sched[r], lane, PcaGlobal{}, c, n_int, n_fs);
      if (lane == 0) {
        const int t = q * kTileRows + team;
#pragma unroll
        for (int k = 0; k < 6; ++k) s_cov[k][t] = c[k];
        s_cnt[0][t] = n_int;
        s_cnt[1][t] = n_fs;
      }
    }
    __syncthreads();  // the staging buffer is rewritten by the next tile
  }
  // one row per thread: eigen solve and classification
  const int t = threadIdx.x;
  const int64_t r = blk * kPcaRows + t;
  if (r >= a.nrows) return;
  pca_finish(a, a.sched[r], s_cnt[0][t], s_cnt[1][t], s_cov[0][t], s_cov[1][t], s_cov[2][t], s_cov[3][t],
             s_cov[4][t], s_cov[5][t]);
}

// untiled rows: teams over the rows of the launch, gathers from global memory
__global__ void __launch_bounds__(kBlock) k_pca_flags(PcaArgs a) {
  const int64_t gt = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t r = gt / kTeam;
  if (r >= a.nrows) return;
  const int32_t i = a.sched[r];
  double c[6];
  int n_int, n_fs;
  pca_cov(a, i, (int)(gt % kTeam), PcaGlobal{}, c, n_int, n_fs);
  if (gt % kTeam == 0) pca_finish(a, i, n_int, n_fs, c[0], c[1], c[2], c[3], c[4], c[5]);
}

// smoothing rule 1 over the cross-model neighbourhood
__global__ void __launch_bounds__(kBlock) k_smooth(const uint8_t *__restrict__ raw, const int8_t *__restrict__ model,
                                                   const int64_t *__restrict__ xrow, const int32_t *__restrict__ xcol,
                                                   int64_t n, uint8_t *__restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint8_t f = raw[i];
  if (f != 0 && xrow) {
    const int target = (f == 1) ? GF_MODEL_FILM : GF_MODEL_BULK;
    bool ok = false;
    for (int64_t k = xrow[i]; k < xrow[i + 1] && !ok; ++k) {
      const int32_t j = xcol[k];
      if (j == i) continue;
      ok = (model[j] == target) || (raw[j] == f);
    }
    if (!ok) f = 0;
  }
  flag[i] = f;
}

// neighbour positions a tile block may stage (larger tiles gather)
constexpr int kPcaCap = 1024;
}  // namespace

extern "C" void gf_pca_params_default(gf_pca_params *p) {
  if (!p) return;
  p->eps_lambda_max = 0.15;
  p->theta_star = 3.14159265358979323846 / 6.0;
  p->literal_rule = 0;
}

extern "C" gf_status gf_classify_pca(gf_ctx *ctx, const gf_particles *p, const gf_nbr *same, const gf_nbr *cross,
                                     const double *film_height, const double *h3d, const uint8_t *prev_transitioned,
                                     const uint8_t *user_flag, const gf_pca_params *params, double *lam_3n,
                                     double *w3_3n, double *eps_n, uint8_t *flag_n) {
  gf_status st = check_particles(ctx, p, flag_n != nullptr, flag_n != nullptr);
  if (st) return st;
  if ((st = check_nbr(ctx, same, p->n))) return st;
  if (same->cross) return set_error(ctx, GF_EINVAL, "`same` must hold same-model neighbourhoods");
  if (cross) {
    if ((st = check_nbr(ctx, cross, p->n))) return st;
    if (!cross->cross) return set_error(ctx, GF_EINVAL, "`cross` must hold cross-model neighbourhoods");
  }
  gf_pca_params prm;
  gf_pca_params_default(&prm);
  if (params) prm = *params;
  const int64_t n = p->n;
  Arena ar;
  if ((st = ensure_scratch(ctx, arena_bytes({(size_t)n}), &ar))) return st;
  uint8_t *raw = flag_n ? ar.take<uint8_t>(n) : nullptr;
  PcaArgs a;
  a.x = p->x; a.y = p->y; a.z = p->z; a.model = p->model; a.kind = p->kind;
  a.nx = p->nx; a.ny = p->ny; a.nz = p->nz;
  a.row_ptr = same->row_ptr; a.col = same->col;
  a.film_height = film_height; a.h3d = h3d; a.prev = prev_transitioned; a.user = user_flag;
  a.eps_max = prm.eps_lambda_max; a.cos_theta = std::cos(prm.theta_star); a.literal = prm.literal_rule;
  a.lam = lam_3n; a.w3 = w3_3n; a.eps = eps_n; a.raw = raw;
  ProfScope prof(ctx, "pca_flags");
  LaunchUnit units[2 * GF_NBAND];
  const int nu = launch_units(same, units);
  for (int q = 0; q < nu; ++q) {
    const LaunchUnit &u = units[q];
    a.sched = same->grouped + u.row0;
    a.nrows = u.nrows;
    if (u.tiled) {
      const int cap = std::min(u.tile_max, tile_capacity(ctx, kPcaCap));
      hipLaunchKernelGGL(k_pca_tile, dim3(grid_for(u.ntiles, kPcaTiles)), dim3(kTileRows * kTeam),
                         sizeof(double4) * cap, ctx->stream, a, same->tile_off, same->tile_u, same->slot, u.tile0,
                         u.ntiles, cap);
    } else {
      hipLaunchKernelGGL(k_pca_flags, dim3(grid_for(u.nrows * kTeam, kBlock)), dim3(kBlock), 0, ctx->stream, a);
    }
    GF_LAUNCH_CHECK(ctx);
  }
  if (flag_n) {
    ProfScope prof_s(ctx, "pca_smooth");
    hipLaunchKernelGGL(k_smooth, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, raw, p->model,
                       cross ? cross->row_ptr : nullptr, cross ? cross->col : nullptr, n, flag_n);
    GF_LAUNCH_CHECK(ctx);
  }
  return GF_OK;
}
