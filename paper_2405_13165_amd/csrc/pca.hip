// Local PCA of every neighbourhood and the transition flags of Sec. 4.
//
// A team of kTeam lanes per particle.  Rows with at most 128 neighbours run
// one neighbour tile per block: the tile's distinct neighbours (position and
// kind) are staged in LDS and read through the tile slots, which each lane
// loads in aligned quads, all before the first is used; rows with more
// neighbours gather from global memory.  One pass accumulates the sums of
// the offsets d = x_j - x_i and of their products, and the covariance about
// the centroid follows as sum d d^T - (sum d)(sum d)^T / n: offsets relative
// to the particle itself keep an exactly planar neighbourhood exactly planar
// (its third eigenvalue is exactly zero), and with |d| <= h the subtraction
// loses no more than a few ulp of the largest eigenvalue.  The neighbour
// kinds are counted in 16-bit fields of one integer.  The team writes the
// covariance and the counts of its row (one 64-byte record), and a second
// kernel runs the eigen solve and the classification with one particle per
// lane: inside the team kernel only one lane of each team would do that
// work while the other three idle.
#include "stencil_common.h"

using namespace gfdm_dev;

namespace {
constexpr int kBlock = 256;
constexpr int kTeam = 4;
static_assert(kTeam == 4, "a team writes its row's 64-byte record as 16 bytes per lane");

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
  double2 *cov;  // [n][4]: c00 c01 | c02 c11 | c12 c22 | counts, 0
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

// A neighbour as (x, y, z, 16 * kind code), the code being the kind 0..2 or 3
// for anything else: the shift that counts it in its 16-bit field.
__device__ inline double pca_code(const PcaArgs &a, int32_t j) {
  const int k = a.kind ? (int)a.kind[j] : 0;
  return (double)(16 * ((k >= 0 && k <= 2) ? k : 3));
}
// The tile's neighbours in LDS as (x, y) 16-byte records, z and the kind
// code in arrays of their own: 25 bytes per neighbour instead of a 32-byte
// record, so that more blocks fit a CU (the kernel is bound by latency and
// LDS-limited in occupancy), and the (x, y) reads start at one of 8 offsets
// in a 128-byte bank row.
struct PcaRec {
  const double2 *xy;
  const double *zz;
  const uint8_t *cc;
  __device__ double4 operator[](int s) const {
    const double2 p = xy[s];
    return make_double4(p.x, p.y, zz[s], (double)cc[s]);
  }
};
struct PcaTile {   // staged in LDS, addressed by slot[]
  static constexpr bool kQuads = true;
  PcaRec sp;
  const uint16_t *slot;
  __device__ double4 operator()(const PcaArgs &, int64_t k) const { return sp[slot[k]]; }
};
struct PcaGlobal {
  static constexpr bool kQuads = false;
  __device__ double4 operator()(const PcaArgs &a, int64_t k) const {
    const int32_t j = a.col[k];
    return make_double4(a.x[j], a.y[j], a.z[j], pca_code(a, j));
  }
};

constexpr int kPq = 128 / (4 * kTeam) + 1;  // quads per lane for rows of at most 128 entries
template <class F>
__device__ void pca_row(const PcaArgs &a, int32_t i, int lane, const F &fetch) {
  const int64_t b = a.row_ptr[i], e = a.row_ptr[i + 1];
  const double xi = a.x[i], yi = a.y[i], zi = a.z[i];
  const bool need_kinds = a.raw && a.kind;
  double c[6];
  int n_int = 0, n_fs = 0;
  uint64_t kinds = 0;
  double mx = 0.0, my = 0.0, mz = 0.0;
  double sxx = 0.0, sxy = 0.0, sxz = 0.0, syy = 0.0, syz = 0.0, szz = 0.0;
  auto visit = [&](const double4 &pj) {
    const double dx = pj.x - xi, dy = pj.y - yi, dz = pj.z - zi;
    mx += dx; my += dy; mz += dz;
    sxx += dx * dx; sxy += dx * dy; sxz += dx * dz;
    syy += dy * dy; syz += dy * dz; szz += dz * dz;
    if (need_kinds) kinds += (uint64_t)1 << (int)pj.w;
  };
  if constexpr (F::kQuads) {
    // entries 4q .. 4q+3 of the aligned quads q0 + lane, q0 + lane + kTeam, ...; a quad may reach
    // up to three entries into the neighbouring rows (padded slot array): those are skipped
    const int64_t q0 = (b >> 2) + lane;
    ushort4 ss[kPq];
#pragma unroll
    for (int j = 0; j < kPq; ++j) {
      const int64_t k = 4 * (q0 + j * kTeam);
      if (k < e) ss[j] = *reinterpret_cast<const ushort4 *>(fetch.slot + k);
    }
#pragma unroll
    for (int j = 0; j < kPq; ++j) {
      const int64_t k = 4 * (q0 + j * kTeam);
      if (k < e) {
        if (k >= b) visit(fetch.sp[ss[j].x]);
        if (k + 1 >= b && k + 1 < e) visit(fetch.sp[ss[j].y]);
        if (k + 2 >= b && k + 2 < e) visit(fetch.sp[ss[j].z]);
        if (k + 3 < e) visit(fetch.sp[ss[j].w]);
      }
    }
  } else {
    for (int64_t k = b + lane; k < e; k += kTeam) visit(fetch(a, k));
  }
  mx = team_sum(mx, kTeam);
  my = team_sum(my, kTeam);
  mz = team_sum(mz, kTeam);
  if (need_kinds) {
    kinds = team_sum(kinds, kTeam);
    // i is in S_i once: remove its own kind
    const int ko = (int)a.kind[i];
    kinds -= (uint64_t)1 << (16 * ((ko >= 0 && ko <= 2) ? ko : 3));
    n_int = (int)(kinds & 0xFFFF);
    n_fs = (int)((kinds >> 16) & 0xFFFF);
  }
  sxx = team_sum(sxx, kTeam); sxy = team_sum(sxy, kTeam); sxz = team_sum(sxz, kTeam);
  syy = team_sum(syy, kTeam); syz = team_sum(syz, kTeam); szz = team_sum(szz, kTeam);
  const double inv = 1.0 / (double)(e - b);
  const double cx = mx * inv, cy = my * inv, cz = mz * inv;
  c[0] = sxx - mx * cx; c[1] = sxy - mx * cy; c[2] = sxz - mx * cz;
  c[3] = syy - my * cy; c[4] = syz - my * cz; c[5] = szz - mz * cz;
  // every lane holds the sums: lane l writes 16 bytes of the row's record
  const double cnt = __builtin_bit_cast(double, (uint64_t)(uint32_t)n_int | ((uint64_t)(uint32_t)n_fs << 32));
  const double2 v = lane == 0 ? make_double2(c[0], c[1])
                  : lane == 1 ? make_double2(c[2], c[3])
                  : lane == 2 ? make_double2(c[4], c[5]) : make_double2(cnt, 0.0);
  a.cov[4 * (int64_t)i + lane] = v;
}

// eigen solve and classification, one particle per lane
__global__ void __launch_bounds__(kBlock) k_pca_finish(PcaArgs a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 r0 = a.cov[4 * i], r1 = a.cov[4 * i + 1], r2 = a.cov[4 * i + 2], r3 = a.cov[4 * i + 3];
  const uint64_t cnt = __builtin_bit_cast(uint64_t, r3.x);
  pca_finish(a, (int32_t)i, (int)(uint32_t)cnt, (int)(uint32_t)(cnt >> 32), r0.x, r0.y, r1.x, r1.y, r2.x, r2.y);
}

// tiled rows: one neighbour tile per block, kTileRows teams
__global__ void __launch_bounds__(kTileRows * kTeam) k_pca_tile(PcaArgs a, const int64_t *__restrict__ toff,
                                                                const int32_t *__restrict__ tu,
                                                                const uint16_t *__restrict__ slot, int64_t tile0,
                                                                int cap) {
  extern __shared__ double2 s_rec[];  // (x, y)[cap], then z[cap], then code[cap]
  double *s_z = reinterpret_cast<double *>(s_rec + cap);
  uint8_t *s_c = reinterpret_cast<uint8_t *>(s_z + cap);
  const int64_t tl = xcd_block(blockIdx.x, gridDim.x);
  const int64_t u0 = toff[tile0 + tl];
  const int cnt = (int)(toff[tile0 + tl + 1] - u0);
  const bool staged = cnt <= cap;
  if (staged) {
    for (int s = threadIdx.x; s < cnt; s += blockDim.x) {
      const int32_t j = tu[u0 + s];
      s_rec[s] = make_double2(a.x[j], a.y[j]);
      s_z[s] = a.z[j];
      s_c[s] = (uint8_t)pca_code(a, j);
    }
  }
  __syncthreads();
  const int team = threadIdx.x / kTeam, lane = threadIdx.x % kTeam;
  const int64_t r = tl * kTileRows + team;
  if (r >= a.nrows) return;
  const int32_t i = a.sched[r];
  if (staged) pca_row(a, i, lane, PcaTile{PcaRec{s_rec, s_z, s_c}, slot});
  else pca_row(a, i, lane, PcaGlobal{});
}

// untiled rows: teams over the rows of the launch, gathers from global memory
__global__ void __launch_bounds__(kBlock) k_pca_flags(PcaArgs a) {
  const int64_t gt = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t r = gt / kTeam;
  if (r >= a.nrows) return;
  pca_row(a, a.sched[r], (int)(gt % kTeam), PcaGlobal{});
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
  if ((st = ensure_scratch(ctx, arena_bytes({(size_t)n, 64 * (size_t)n}), &ar))) return st;
  uint8_t *raw = flag_n ? ar.take<uint8_t>(n) : nullptr;
  double2 *cov = ar.take<double2>(4 * (size_t)n);
  PcaArgs a;
  a.x = p->x; a.y = p->y; a.z = p->z; a.model = p->model; a.kind = p->kind;
  a.nx = p->nx; a.ny = p->ny; a.nz = p->nz;
  a.row_ptr = same->row_ptr; a.col = same->col;
  a.film_height = film_height; a.h3d = h3d; a.prev = prev_transitioned; a.user = user_flag;
  a.eps_max = prm.eps_lambda_max; a.cos_theta = std::cos(prm.theta_star); a.literal = prm.literal_rule;
  a.lam = lam_3n; a.w3 = w3_3n; a.eps = eps_n; a.raw = raw; a.cov = cov;
  {
  ProfScope prof(ctx, "pca_cov");
  LaunchUnit units[2 * GF_NBAND];
  const int nu = launch_units(same, units);
  for (int q = 0; q < nu; ++q) {
    const LaunchUnit &u = units[q];
    a.sched = same->grouped + u.row0;
    a.nrows = u.nrows;
    if (u.tiled) {
      const int cap = std::min(u.tile_max, tile_capacity(ctx, kPcaCap));
      hipLaunchKernelGGL(k_pca_tile, dim3(grid_for(u.ntiles, 1)), dim3(kTileRows * kTeam), (sizeof(double2) + sizeof(double) + 1) * (size_t)cap,
                         ctx->stream, a, same->tile_off, same->tile_u, same->slot, u.tile0, cap);
    } else {
      hipLaunchKernelGGL(k_pca_flags, dim3(grid_for(u.nrows * kTeam, kBlock)), dim3(kBlock), 0, ctx->stream, a);
    }
    GF_LAUNCH_CHECK(ctx);
  }
  }
  {
    ProfScope prof(ctx, "pca_finish");
    hipLaunchKernelGGL(k_pca_finish, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, a, n);
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
