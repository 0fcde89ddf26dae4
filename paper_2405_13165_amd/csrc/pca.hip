// Local PCA of every neighbourhood and the transition flags of Sec. 4.
//
// Rows with at most 128 neighbours get a team of kTeam lanes each and run
// one neighbour tile per block: the tile's distinct neighbours (position and
// kind) are staged in LDS and read through the tile slots, which each lane
// loads in aligned quads, all before the first is used; rows with more
// neighbours gather from global memory, with teams of kTeamWide lanes that
// keep four entries each in flight.  One pass accumulates the sums of
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

// One Jacobi rotation in the (p, q) plane of a symmetric 3x3 matrix, r being
// the third index: annihilates a_pq.  tan(phi) is the root of smaller
// magnitude of t^2 + 2 t cot(2 phi) - 1 = 0, cot(2 phi) = (a_qq - a_pp) / (2 a_pq),
// written as 2 a_pq sign(a_qq - a_pp) / (|a_qq - a_pp| + sqrt((a_qq - a_pp)^2 + 4 a_pq^2))
// so that it takes one division and one square root; cos(phi) = 1 / sqrt(1 + t^2).
// Only the entries the rotation changes are updated, a_pp and a_qq in the
// form a_pp - t a_pq, a_qq + t a_pq; vp and vq are columns p and q of the
// accumulated rotation.
__device__ __forceinline__ void jacobi_rotate(double &app, double &aqq, double &apq, double &arp, double &arq,
                                              double vp[3], double vq[3]) {
  if (apq == 0.0) return;
  const double d = aqq - app, two = 2.0 * apq;
  const double r = sqrt(d * d + two * two);
  const double den = fabs(d) + r;
  if (!(den > 0.0)) return;  // both squares underflowed with d == 0: leave a_pq for the next sweep
  const double t = copysign(1.0, d) * two / den;
  const double c = rsqrt(1.0 + t * t);
  const double s = t * c;
  const double ta = t * apq;
  app -= ta;
  aqq += ta;
  apq = 0.0;
  const double xp = arp, xq = arq;
  arp = c * xp - s * xq;
  arq = s * xp + c * xq;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double up = vp[k], uq = vq[k];
    vp[k] = c * up - s * uq;
    vq[k] = s * up + c * uq;
  }
}

// Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations over the
// planes (0, 1), (0, 2), (1, 2), sweeping until the off-diagonal mass is
// negligible.  lam: the diagonal at the end; V[k][c]: component k of the
// eigenvector of lam[c].
__device__ void sym3_eigen(double a00, double a01, double a02, double a11, double a12, double a22,
                           double lam[3], double V[3][3]) {
  double v0[3] = {1.0, 0.0, 0.0}, v1[3] = {0.0, 1.0, 0.0}, v2[3] = {0.0, 0.0, 1.0};
  const double scale = sqrt(a00 * a00 + a11 * a11 + a22 * a22 + 2.0 * (a01 * a01 + a02 * a02 + a12 * a12));
  for (int sweep = 0; sweep < 32; ++sweep) {
    const double off = fabs(a01) + fabs(a02) + fabs(a12);
    if (off == 0.0 || off <= 1e-17 * scale) break;
    jacobi_rotate(a00, a11, a01, a02, a12, v0, v1);  // p, q, r = 0, 1, 2
    jacobi_rotate(a00, a22, a02, a01, a12, v0, v2);  // p, q, r = 0, 2, 1
    jacobi_rotate(a11, a22, a12, a01, a02, v1, v2);  // p, q, r = 1, 2, 0
  }
  lam[0] = a00;
  lam[1] = a11;
  lam[2] = a22;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    V[k][0] = v0[k];
    V[k][1] = v1[k];
    V[k][2] = v2[k];
  }
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
__device__ inline double pca_code_of(int k) { return (double)(16 * ((k >= 0 && k <= 2) ? k : 3)); }
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
};
struct PcaGlobal {  // gathered from global memory
  static constexpr bool kQuads = false;
};

// lanes per row for rows that gather from global memory (rows of more than
// 128 neighbours): each lane keeps four entries in flight
constexpr int kTeamWide = 16;

template <int T, class F>
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
    // entries 4q .. 4q+3 of the aligned quads q0 + lane, q0 + lane + T, ...; a quad may reach
    // up to three entries into the neighbouring rows (padded slot array): those are skipped
    constexpr int kPq = 128 / (4 * T) + 1;  // quads per lane for rows of at most 128 entries
    const int64_t q0 = (b >> 2) + lane;
    ushort4 ss[kPq];
#pragma unroll
    for (int j = 0; j < kPq; ++j) {
      const int64_t k = 4 * (q0 + j * T);
      if (k < e) ss[j] = *reinterpret_cast<const ushort4 *>(fetch.slot + k);
    }
#pragma unroll
    for (int j = 0; j < kPq; ++j) {
      const int64_t k = 4 * (q0 + j * T);
      if (k < e) {
        if (k >= b) visit(fetch.sp[ss[j].x]);
        if (k + 1 >= b && k + 1 < e) visit(fetch.sp[ss[j].y]);
        if (k + 2 >= b && k + 2 < e) visit(fetch.sp[ss[j].z]);
        if (k + 3 < e) visit(fetch.sp[ss[j].w]);
      }
    }
  } else {
    // entries k0, k0 + T, k0 + 2T, k0 + 3T per step, every load of a step issued before the first
    // is used; an entry past the row's end reads particle i itself, whose offset d = 0 adds
    // nothing to the sums, and is left out of the kind counts.  The kind byte is read without a
    // branch (from the model array when there are no kinds, whose codes then go unused), so that
    // no load waits for the one before it.
    const int8_t *kp = a.kind ? a.kind : a.model;
    for (int64_t k0 = b + lane; k0 < e; k0 += 4 * T) {
      int32_t jj[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int32_t c = a.col[min(k0 + u * T, e - 1)];
        jj[u] = k0 + u * T < e ? c : i;
      }
      double4 pj[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) pj[u] = make_double4(a.x[jj[u]], a.y[jj[u]], a.z[jj[u]], pca_code_of(kp[jj[u]]));
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double dx = pj[u].x - xi, dy = pj[u].y - yi, dz = pj[u].z - zi;
        mx += dx; my += dy; mz += dz;
        sxx += dx * dx; sxy += dx * dy; sxz += dx * dz;
        syy += dy * dy; syz += dy * dz; szz += dz * dz;
        if (need_kinds && k0 + u * T < e) kinds += (uint64_t)1 << (int)pj[u].w;
      }
    }
  }
  mx = team_sum(mx, T);
  my = team_sum(my, T);
  mz = team_sum(mz, T);
  if (need_kinds) {
    kinds = team_sum(kinds, T);
    // i is in S_i once: remove its own kind
    const int ko = (int)a.kind[i];
    kinds -= (uint64_t)1 << (16 * ((ko >= 0 && ko <= 2) ? ko : 3));
    n_int = (int)(kinds & 0xFFFF);
    n_fs = (int)((kinds >> 16) & 0xFFFF);
  }
  sxx = team_sum(sxx, T); sxy = team_sum(sxy, T); sxz = team_sum(sxz, T);
  syy = team_sum(syy, T); syz = team_sum(syz, T); szz = team_sum(szz, T);
  const double inv = 1.0 / (double)(e - b);
  const double cx = mx * inv, cy = my * inv, cz = mz * inv;
  c[0] = sxx - mx * cx; c[1] = sxy - mx * cy; c[2] = sxz - mx * cz;
  c[3] = syy - my * cy; c[4] = syz - my * cz; c[5] = szz - mz * cz;
  // every lane holds the sums: lane l < 4 writes 16 bytes of the row's record
  if (lane >= 4) return;
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
    const int8_t *kp = a.kind ? a.kind : a.model;  // codes unused without kinds; no branch per load
    for (int s = threadIdx.x; s < cnt; s += blockDim.x) {
      const int32_t j = tu[u0 + s];
      s_rec[s] = make_double2(a.x[j], a.y[j]);
      s_z[s] = a.z[j];
      s_c[s] = (uint8_t)pca_code_of(kp[j]);
    }
  }
  __syncthreads();
  const int team = threadIdx.x / kTeam, lane = threadIdx.x % kTeam;
  const int64_t r = tl * kTileRows + team;
  if (r >= a.nrows) return;
  const int32_t i = a.sched[r];
  if (staged) pca_row<kTeam>(a, i, lane, PcaTile{PcaRec{s_rec, s_z, s_c}, slot});
  else pca_row<kTeam>(a, i, lane, PcaGlobal{});
}

// untiled rows: teams of kTeamWide lanes over the rows of the launch, gathers from global memory
__global__ void __launch_bounds__(kBlock) k_pca_flags(PcaArgs a) {
  const int64_t gt = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t r = gt / kTeamWide;
  if (r >= a.nrows) return;
  pca_row<kTeamWide>(a, a.sched[r], (int)(gt % kTeamWide), PcaGlobal{});
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
      hipLaunchKernelGGL(k_pca_flags, dim3(grid_for(u.nrows * kTeamWide, kBlock)), dim3(kBlock), 0, ctx->stream, a);
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
