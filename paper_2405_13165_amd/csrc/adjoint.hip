// Gradient of L(out), out_i^s = sum_{j != i} c_ij^s (u_j - u_i), with respect
// to particle positions through the stencil weights.
//
// For particle i, with G = sum_j w_j phi_j phi_j^T, lambda_s = G^{-1} d_s and
// chat_j = w_j phi_j . lambda_s, the chain rule gives, for the adjoint
// chatbar_js of the dimensionless stencil,
//   mu_s     = G^{-1} sum_j chatbar_js w_j phi_j
//   wbar_j   = sum_s chatbar_js (phi_j . lambda_s) - (mu_s . phi_j)(phi_j . lambda_s)
//   phibar_j = sum_s chatbar_js w_j lambda_s - w_j (mu_s (phi_j . lambda_s)
//                                                   + lambda_s (mu_s . phi_j))
//   dbar_j   = (d phi / d d)^T phibar_j + wbar_j dw/dd,   d = x_j - x_i,
// and x_j gains dbar_j, x_i loses it.  The stencils are recomputed (nothing
// is stored but the neighbour lists).  Per-entry contributions go to scratch
// with the rows laid out in grouped (Morton) order and are gathered per
// particle, in the same order, through the reverse-edge map: the twin entry
// (j, i) of (i, j) lies in a Morton-near row, so the gather stays in L2.  No
// atomics: the result is deterministic.  The Gram system is solved by LDL^T in FP64.
// Rows whose forward stencils are zero (status 2 or 3 of the stencil call,
// when the caller passes those statuses) contribute nothing, and so do rows
// whose Gram matrix is not positive definite.
#include "stencil_common.h"

using namespace gfdm_dev;

namespace {
constexpr int kBlock = 256;
constexpr int kT = 8;

struct AArgs {
  const double *x, *y, *z, *h, *nx, *ny, *nz;
  const double4 *pos;  // (x, y, z, h) packed per particle
  const int64_t *row_ptr;
  const int32_t *col;
  const int32_t *sched;
  int64_t nrows, n;
  WeightFn wf;
  unsigned mask;
  const double *u, *ybar;
  const int8_t *status;  // forward stencil statuses (may be NULL)
  double *dbar;  // [nnz][3], rows in grouped order
  double *xbar;  // [n][3]: each row subtracts its own entries' sum here
  const int64_t *gbase;  // per team: offset of its row in dbar (grouped row offsets)
};

// SEL: the stencils (bits of the op mask) the kernel carries; stencils
// outside SEL have no adjoint (ybar = 0) and their terms are not formed.
// The general kernel carries all four; the common single-operator cases
// (Laplacian, gradient) get their own, with far fewer registers.
//
// A team of kT lanes per particle, in the form of the batched stencil kernel:
// G from the weighted moments of the offsets (team sum through LDS), its
// inverse by team Gauss-Jordan (lane owns rows lane + q kT), lambda_s and
// mu_s shared through the team's LDS area.  Everything is written in the
// unscaled offsets d (monomials of d, physical targets), where lambda_s are
// the coefficients of the physical stencils as they stand; the weights leave
// out their normalising factor 1 / (1 - e^{-a}): a common factor of the
// weights cancels from the stencils and from every term below (G and v_s
// scale with it, lambda_s and mu_s with its inverse, dw/dd with it).
template <int M>
constexpr int adj_lds_doubles() {  // per team: reduction / moments / pivot row, then lambda (4M), mu (4M)
  return ((cmax(cmax(nmom<M>(), red_lanes(kT) * red_lanes(kT)), cmax(M + 1, 8 * M)) + 1) & ~1);
}

// Visit the entries k = lane, lane + T, ... of a row of n >= 1 entries at CSR
// entry b, calling body(k, j, position of j, field value of j (FIELD)); the
// column two steps ahead and the position (and field value) one step ahead
// are in flight during the arithmetic.  Loads past the row's end read its
// last entry (valid, never used), so every load is unconditional.
template <int T, bool FIELD, class Body>
__device__ inline void adj_walk(const AArgs &a, int64_t b, int n, int lane, Body &&body) {
  const int kmax = n - 1;
  int32_t jc = a.col[b + min(lane, kmax)];
  int32_t jn = a.col[b + min(lane + T, kmax)];
  double4 pc = a.pos[jc];
  double uc = FIELD ? a.u[jc] : 0.0;
#pragma unroll 1
  for (int k = lane; k < n; k += T) {
    const int32_t j = jc;
    const double4 pj = pc;
    const double uj = uc;
    jc = jn;
    pc = a.pos[jn];
    if constexpr (FIELD) uc = a.u[jn];
    jn = a.col[b + min(k + 2 * T, kmax)];
    body(k, j, pj, uj);
  }
}

template <int M, unsigned SEL>
__device__ void adjoint_row(const AArgs &a, int32_t i, int64_t ob, int lane, double *sm) {
  constexpr int T = kT;
  constexpr int NM = nmom<M>();
  constexpr int NR = (M + T - 1) / T;
  const int64_t b = a.row_ptr[i];
  const int n = (int)(a.row_ptr[i + 1] - b);
  RowGeom g;
  g.xi = a.x[i]; g.yi = a.y[i]; g.zi = a.z[i]; g.hi = a.h[i]; g.inv_h = 1.0;  // unscaled monomials
  if constexpr (M == 6) tangent_frame(a.nx[i], a.ny[i], a.nz[i], g.t1, g.t2);
  auto zero_out = [&]() {
    for (int k = lane; k < n; k += T) {
      double *d = a.dbar + 3 * (ob + k);
      d[0] = 0.0; d[1] = 0.0; d[2] = 0.0;
    }
  };
  // n < M (status 3) and rank-deficient rows (status 2) have constant zero stencils
  if (n < M || (a.status && a.status[i] >= 2)) {
    zero_out();
    return;
  }
  // unnormalised weight e^{-a q^2} - e^{-a}, q^2 = |d|^2 / r^2, r = (h_i + h_j) / 2;
  // e = e^{-a q^2} and ir2 = 1 / r^2 give dw/dd = -2 a e ir2 d.  Equal
  // supports take the row's 1 / h_i^2; others 1 / r^2 from the reciprocal
  // estimate and two Newton steps
  const double ir2_row = 1.0 / (g.hi * g.hi);
  auto weight = [&](double hj, double d2, double &e, double &ir2) {
    if (hj == g.hi) {
      ir2 = ir2_row;
    } else {
      const double r = 0.5 * (g.hi + hj), rr = r * r;
      double q = __builtin_amdgcn_rcp(rr);
      q = fma(q, fma(-rr, q, 1.0), q);
      ir2 = fma(q, fma(-rr, q, 1.0), q);
    }
    e = exp(-a.wf.alpha * (d2 * ir2));
    return e - a.wf.ea;
  };
  // ---- pass 1: moments
  double mom[NM];
#pragma unroll
  for (int p = 0; p < NM; ++p) mom[p] = 0.0;
  adj_walk<T, false>(a, b, n, lane, [&](int, int32_t, const double4 &pj, double) {
    const double dx = pj.x - g.xi, dy = pj.y - g.yi, dz = pj.z - g.zi;
    double e, ir2;
    const double w = weight(pj.w, fma(dz, dz, fma(dy, dy, dx * dx)), e, ir2);
    double X, Y, Z;
    local_raw<M>(g, dx, dy, dz, X, Y, Z);
    moments_add_raw<M>(mom, w, X, Y, Z);
  });
  team_moment_sum<M, T>(mom, lane, sm);
  // ---- G^{-1}
  double row[NR][M];
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int r = lane + q * T;
    const bool own = r < M;
#pragma unroll
    for (int c = 0; c < M; ++c) {
      const int mi = own ? (M == 10 ? kGram3.v[r][c] : kGram2.v[r][c]) : 0;
      row[q][c] = own ? sm[mi] : 0.0;
    }
  }
  wave_sync();  // the pivot rows overwrite the moments
  if (!team_gauss_jordan<M, T>(row, lane, sm)) {  // G not positive definite (same on every lane)
    zero_out();
    return;
  }
  // lambda_s = G^{-1} t_s (the target of stencil s), row r on the lane that owns it
  double *s_lam = sm, *s_mu = sm + 4 * M;
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int r = lane + q * T;
    if (r < M) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (!((SEL >> s) & 1u)) continue;
        double v = 0.0;
#pragma unroll
        for (int c = 1; c < M; ++c) {
          const double cf = target_coef<M>(s, c);
          if (cf != 0.0) v += cf * row[q][c];
        }
        s_lam[s * M + r] = v;
      }
    }
  }
  // ybar of this row, per stencil s (zero if not selected)
  double yb[4] = {0.0, 0.0, 0.0, 0.0};
  {
    int q = 0;
    for (int s = 0; s < 4; ++s)
      if (a.mask & (1u << s)) yb[s] = a.ybar[(int64_t)(q++) * a.n + i];
  }
  const double ui = a.u[i];
  // chatbar_js = dL / dc_js for the stencils the kernel forms (on a film the
  // tangential ones, s = 0, 1, of which the stored x, y, z stencils are the
  // combinations t1 c_0 + t2 c_1)
  auto chatbar = [&](int32_t j, double uj, double cb[4]) {
    const double du = (j != i) ? (uj - ui) : 0.0;
    if constexpr (M == 10) {
      cb[0] = yb[0] * du; cb[1] = yb[1] * du; cb[2] = yb[2] * du;
    } else {
      const double gx = yb[0] * du, gy = yb[1] * du, gz = yb[2] * du;
      cb[0] = g.t1[0] * gx + g.t1[1] * gy + g.t1[2] * gz;
      cb[1] = g.t2[0] * gx + g.t2[1] * gy + g.t2[2] * gz;
      cb[2] = 0.0;
    }
    cb[3] = yb[3] * du;
  };
  // ---- pass 2: v_s = sum_j chatbar_js w_j phi_j
  double v[4][M];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int r = 0; r < M; ++r) v[s][r] = 0.0;  // (entries outside SEL are never read)
  adj_walk<T, true>(a, b, n, lane, [&](int, int32_t j, const double4 &pj, double uj) {
    const double dx = pj.x - g.xi, dy = pj.y - g.yi, dz = pj.z - g.zi;
    double e, ir2;
    const double w = weight(pj.w, fma(dz, dz, fma(dy, dy, dx * dx)), e, ir2);
    double phi[M], cb[4];
    monomials<M>(g, dx, dy, dz, phi);
    chatbar(j, uj, cb);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (!((SEL >> s) & 1u)) continue;
      const double cw = cb[s] * w;
#pragma unroll
      for (int r = 0; r < M; ++r) v[s][r] = fma(cw, phi[r], v[s][r]);
    }
  });
  // ---- mu_s = G^{-1} v_s, row r on the lane that owns it
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (!((SEL >> s) & 1u)) continue;
#pragma unroll
    for (int r = 0; r < M; ++r) v[s][r] = team_sum(v[s][r], T);
  }
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int r = lane + q * T;
    if (r < M) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (!((SEL >> s) & 1u)) continue;
        double m = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) m = fma(row[q][c], v[s][c], m);
        s_mu[s * M + r] = m;
      }
    }
  }
  wave_sync();
  double lam[4][M], mu[4][M];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (!((SEL >> s) & 1u)) continue;
#pragma unroll
    for (int r = 0; r < M; ++r) {
      lam[s][r] = s_lam[s * M + r];
      mu[s][r] = s_mu[s * M + r];
    }
  }
  // ---- pass 3: dbar_j per entry
  double own[3] = {0.0, 0.0, 0.0};  // this lane's share of sum_j dbar(i, j)
  // each entry's dbar is stored one step late, at the start of the next
  // step: a load and a store in flight count against one counter, and the
  // wait for the next entry's column would otherwise wait for the store
  double po[3] = {0.0, 0.0, 0.0};
  int kp = -1;
  auto flush_prev = [&]() {
    if (kp >= 0) {
      double *out = a.dbar + 3 * (ob + kp);
      out[0] = po[0]; out[1] = po[1]; out[2] = po[2];
    }
  };
  adj_walk<T, true>(a, b, n, lane, [&](int k, int32_t j, const double4 &pj, double uj) {
    flush_prev();
    kp = k;
    if (j == i) {
      po[0] = 0.0; po[1] = 0.0; po[2] = 0.0;
      return;
    }
    const double dx = pj.x - g.xi, dy = pj.y - g.yi, dz = pj.z - g.zi;
    double e, ir2;
    const double w = weight(pj.w, fma(dz, dz, fma(dy, dy, dx * dx)), e, ir2);
    double phi[M], cb[4];
    monomials<M>(g, dx, dy, dz, phi);
    chatbar(j, uj, cb);
    double wb = 0.0, pb[M];
#pragma unroll
    for (int q = 0; q < M; ++q) pb[q] = 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (!((SEL >> s) & 1u)) continue;
      double pl = 0.0, mp = 0.0;
#pragma unroll
      for (int q = 0; q < M; ++q) { pl = fma(phi[q], lam[s][q], pl); mp = fma(mu[s][q], phi[q], mp); }
      wb += (cb[s] - mp) * pl;
#pragma unroll
      for (int q = 0; q < M; ++q) pb[q] += w * ((cb[s] - mp) * lam[s][q] - pl * mu[s][q]);
    }
    double dd[3];
    monomials_grad_dot<M>(g, dx, dy, dz, pb, dd);
    const double f = wb * (-2.0 * a.wf.alpha * e * ir2);
    po[0] = dd[0] + f * dx;
    po[1] = dd[1] + f * dy;
    po[2] = dd[2] + f * dz;
    own[0] += po[0];
    own[1] += po[1];
    own[2] += po[2];
  });
  flush_prev();
  // x_i loses every dbar(i, j), whether or not (j, i) is listed
#pragma unroll
  for (int c = 0; c < 3; ++c) own[c] = team_sum(own[c], T);
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) a.xbar[3 * (int64_t)i + c] -= own[c];
  }
}

// The Laplacian-only kernels (the common case) are held at 4 (film) and 3
// (3D) waves per SIMD, a few registers spilled; the others take what they need.
template <int M, unsigned SEL>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(SEL == 8u ? (M == 6 ? 4 : 3) : 1))) k_adjoint_x(AArgs a) {
  __shared__ double smem[(kBlock / kT) * adj_lds_doubles<M>()];
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t team = gt / kT;
  const int lane = (int)(gt % kT);
  if (team >= a.nrows) return;
  adjoint_row<M, SEL>(a, a.sched[team], a.gbase[team], lane,
                      smem + (threadIdx.x / kT) * adj_lds_doubles<M>());
}

template <int M>
void launch_adjoint_x(hipStream_t sm, dim3 grid, dim3 block, const AArgs &a) {
  if (a.mask == 8u) hipLaunchKernelGGL((k_adjoint_x<M, 8u>), grid, block, 0, sm, a);       // Laplacian
  else if (a.mask == 7u) hipLaunchKernelGGL((k_adjoint_x<M, 7u>), grid, block, 0, sm, a);  // gradient
  else hipLaunchKernelGGL((k_adjoint_x<M, 15u>), grid, block, 0, sm, a);
}

// xbar_j += sum over entries (j, i) of row j, i != j, of dbar(i, j) (x_j gains
// what row i differentiated with respect to it; the row's own entries were
// subtracted by the row kernel); rows in grouped order, a team of kGT lanes
// per row; the twin dbar(i, j) sits at grev[g] (a Morton-near row).  An entry
// (j, i) without a twin (i a ghost particle whose row holds only itself)
// adds nothing.
constexpr int kGT = 8;  // lanes per row of the gather
// entries per lane and step of the gather (lanes x entries on the mixed cloud:
// 8 x 8 481 us, 8 x 4 497, 16 x 4 488, 4 x 8 526)
constexpr int kGU = 8;
__global__ void __launch_bounds__(kBlock) k_adjoint_gather(const int32_t *__restrict__ grouped,
                                                           const int64_t *__restrict__ grow_ptr,
                                                           const int32_t *__restrict__ grev,
                                                           const double *__restrict__ dbar, int64_t n,
                                                           double *__restrict__ xbar) {
  const int64_t gt = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t t = gt / kGT;
  const int lane = (int)(gt % kGT);
  if (t >= n) return;
  const int32_t j = grouped[t];
  const int64_t g0 = grow_ptr[t], g1 = grow_ptr[t + 1];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  // kGU entries per lane and step: every twin position of the step, then
  // every dbar record, is requested before the first is used (a straight
  // block, so none of the loads is moved down to its use); reads past the
  // row's end take its last entry, an entry without a twin reads record 0
  // (both valid, neither added)
  const int64_t gl = g1 - 1;  // a step starts only at gk < g1: gl is in the row
#pragma unroll 1
  for (int64_t gk = g0 + lane; gk < g1; gk += kGU * kGT) {
    int32_t tw[kGU];
#pragma unroll
    for (int u = 0; u < kGU; ++u) tw[u] = grev[min(gk + u * kGT, gl)];
    double da[kGU], db[kGU], dc[kGU];
#pragma unroll
    for (int u = 0; u < kGU; ++u) {
      const int64_t q = 3 * (int64_t)(tw[u] >= 0 ? tw[u] : 0);
      da[u] = dbar[q];
      db[u] = dbar[q + 1];
      dc[u] = dbar[q + 2];
    }
#pragma unroll
    for (int u = 0; u < kGU; ++u) {  // in entry order
      const bool on = tw[u] >= 0 && gk + u * kGT < g1;
      s0 += on ? da[u] : 0.0;
      s1 += on ? db[u] : 0.0;
      s2 += on ? dc[u] : 0.0;
    }
  }
  s0 = team_sum(s0, kGT);
  s1 = team_sum(s1, kGT);
  s2 = team_sum(s2, kGT);
  if (lane == 0) {
    xbar[3 * j] += s0;
    xbar[3 * j + 1] += s1;
    xbar[3 * j + 2] += s2;
  }
}
}  // namespace

extern "C" gf_status gf_gfdm_weights_adjoint(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr,
                                             const gf_ls_params *params, unsigned op_mask, const double *u,
                                             const double *ybar, const int8_t *status_n, double *xbar_3n) {
  if (!ctx) return GF_EINVAL;
  gf_status st = check_particles(ctx, p, false, false);
  if (st) return st;
  if ((st = check_nbr(ctx, nbr, p->n))) return st;
  if (nbr->cross) return set_error(ctx, GF_EINVAL, "stencils need same-model neighbourhoods");
  if (!u || !ybar || !xbar_3n) return set_error(ctx, GF_EINVAL, "u, ybar and xbar are required");
  if ((op_mask & 0xF) == 0 || (op_mask & ~0xFu)) return set_error(ctx, GF_EINVAL, "op_mask must select 1..4 operators");
  const bool has_film = nbr->group_start[2 * GF_NBAND] > nbr->group_start[GF_NBAND];
  if (has_film && (!p->nx || !p->ny || !p->nz)) return set_error(ctx, GF_EINVAL, "film particles need normals");
  gf_ls_params prm;
  gf_ls_params_default(&prm);
  if (params) prm = *params;
  if ((st = ensure_grouped_rows(ctx, const_cast<gf_nbr *>(nbr)))) return st;
  Arena ar;
  if ((st = ensure_scratch(ctx, arena_bytes({sizeof(double) * 3 * (size_t)std::max<int64_t>(nbr->nnz, 1),
                                             sizeof(double4) * (size_t)p->n}), &ar)))
    return st;
  AArgs a;
  a.x = p->x; a.y = p->y; a.z = p->z; a.h = p->h; a.nx = p->nx; a.ny = p->ny; a.nz = p->nz;
  a.row_ptr = nbr->row_ptr; a.col = nbr->col; a.n = p->n;
  a.wf = make_weight_fn(prm.alpha_w);
  a.mask = op_mask; a.u = u; a.ybar = ybar; a.status = status_n;
  a.dbar = ar.take<double>(3 * (size_t)std::max<int64_t>(nbr->nnz, 1));
  double4 *pos = ar.take<double4>(p->n);
  {
    ProfScope prof(ctx, "pack_positions");
    hipLaunchKernelGGL(k_pack_pos, dim3(grid_for(p->n, 256)), dim3(256), 0, ctx->stream, p->x, p->y, p->z, p->h, p->n,
                       pos);
    GF_LAUNCH_CHECK(ctx);
  }
  a.pos = pos;
  a.xbar = xbar_3n;
  for (int m = 0; m < 2; ++m) {
    const int64_t s0 = nbr->group_start[m * GF_NBAND], s1 = nbr->group_start[(m + 1) * GF_NBAND];
    if (s1 <= s0) continue;
    a.sched = nbr->grouped + s0;
    a.gbase = nbr->grow_ptr + s0;
    a.nrows = s1 - s0;
    const dim3 grid(grid_for(a.nrows * kT, kBlock)), block(kBlock);
    ProfScope prof(ctx, m == 0 ? "weights_adjoint_3d" : "weights_adjoint_film");
    if (m == 0) launch_adjoint_x<10>(ctx->stream, grid, block, a);
    else launch_adjoint_x<6>(ctx->stream, grid, block, a);
    GF_LAUNCH_CHECK(ctx);
  }
  {
    ProfScope prof(ctx, "weights_adjoint_gather");
    hipLaunchKernelGGL(k_adjoint_gather, dim3(grid_for(p->n * kGT, kBlock)), dim3(kBlock), 0, ctx->stream,
                       nbr->grouped, nbr->grow_ptr, nbr->grev, a.dbar, p->n, xbar_3n);
    GF_LAUNCH_CHECK(ctx);
  }
  return GF_OK;
}
