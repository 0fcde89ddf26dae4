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
template <int M, unsigned SEL>
__device__ void adjoint_row(const AArgs &a, int32_t i, int64_t ob, int lane) {
  const int64_t b = a.row_ptr[i];
  const int n = (int)(a.row_ptr[i + 1] - b);
  RowGeom g;
  g.xi = a.x[i]; g.yi = a.y[i]; g.zi = a.z[i]; g.hi = a.h[i]; g.inv_h = 1.0 / g.hi;
  if constexpr (M == 6) tangent_frame(a.nx[i], a.ny[i], a.nz[i], g.t1, g.t2);
  // n < M (status 3) and rank-deficient rows (status 2) have constant zero stencils
  bool ok = n >= M && !(a.status && a.status[i] >= 2);
  constexpr int NP = npack(M);
  double G[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) G[p] = 0.0;
  if (ok) {
    for (int k = lane; k < n; k += kT) {
      const int32_t j = a.col[b + k];
      const double dx = a.x[j] - g.xi, dy = a.y[j] - g.yi, dz = a.z[j] - g.zi;
      const double w = support_weight<false>(dx * dx + dy * dy + dz * dz, 0.5 * (g.hi + a.h[j]), a.wf);
      double phi[M];
      monomials<M>(g, dx, dy, dz, phi);
      gram_add<M>(G, phi, w);
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) G[p] = team_sum(G[p], kT);
  }
  double dinv[M];
  if (ok) ok = ldlt<M>(G, dinv);
  if (!ok) {
    for (int k = lane; k < n; k += kT) {
      double *d = a.dbar + 3 * (ob + k);
      d[0] = 0.0; d[1] = 0.0; d[2] = 0.0;
    }
    return;
  }
  // lambda_s = G^{-1} d_s (dimensionless targets)
  double lam[4][M];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (!((SEL >> s) & 1u)) continue;
#pragma unroll
    for (int r = 0; r < M; ++r) lam[s][r] = 0.0;
    if constexpr (M == 10) {
      if (s < 3) lam[s][s + 1] = 1.0; else { lam[s][4] = 2.0; lam[s][5] = 2.0; lam[s][6] = 2.0; }
    } else {
      if (s < 2) lam[s][s + 1] = 1.0; else if (s == 3) { lam[s][3] = 2.0; lam[s][4] = 2.0; }
    }
    ldlt_solve<M>(G, dinv, lam[s]);
  }
  // ybar of this row, per stencil s (zero if not selected)
  double yb[4] = {0.0, 0.0, 0.0, 0.0};
  {
    int q = 0;
    for (int s = 0; s < 4; ++s)
      if (a.mask & (1u << s)) yb[s] = a.ybar[(int64_t)(q++) * a.n + i];
  }
  const double ui = a.u[i];
  const double ih = g.inv_h, ih2 = g.inv_h * g.inv_h;
  // chatbar_j for the dimensionless stencils of this particle
  auto chatbar = [&](int32_t j, double cb[4]) {
    const double du = (j != i) ? (a.u[j] - ui) : 0.0;
    if constexpr (M == 10) {
      cb[0] = yb[0] * du * ih; cb[1] = yb[1] * du * ih; cb[2] = yb[2] * du * ih;
    } else {
      const double gx = yb[0] * du * ih, gy = yb[1] * du * ih, gz = yb[2] * du * ih;
      cb[0] = g.t1[0] * gx + g.t1[1] * gy + g.t1[2] * gz;
      cb[1] = g.t2[0] * gx + g.t2[1] * gy + g.t2[2] * gz;
      cb[2] = 0.0;
    }
    cb[3] = yb[3] * du * ih2;
  };
  // lambdabar_s = sum_j chatbar_js w_j phi_j
  double mu[4][M];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int r = 0; r < M; ++r) mu[s][r] = 0.0;  // (entries outside SEL are never read)
  for (int k = lane; k < n; k += kT) {
    const int32_t j = a.col[b + k];
    const double dx = a.x[j] - g.xi, dy = a.y[j] - g.yi, dz = a.z[j] - g.zi;
    const double w = support_weight<false>(dx * dx + dy * dy + dz * dz, 0.5 * (g.hi + a.h[j]), a.wf);
    double phi[M], cb[4];
    monomials<M>(g, dx, dy, dz, phi);
    chatbar(j, cb);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (!((SEL >> s) & 1u)) continue;
#pragma unroll
      for (int r = 0; r < M; ++r) mu[s][r] += cb[s] * w * phi[r];
    }
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (!((SEL >> s) & 1u)) continue;
#pragma unroll
    for (int r = 0; r < M; ++r) mu[s][r] = team_sum(mu[s][r], kT);
    ldlt_solve<M>(G, dinv, mu[s]);
  }
  double own[3] = {0.0, 0.0, 0.0};  // this lane's share of sum_j dbar(i, j)
  for (int k = lane; k < n; k += kT) {
    const int32_t j = a.col[b + k];
    double *out = a.dbar + 3 * (ob + k);
    if (j == i) { out[0] = 0.0; out[1] = 0.0; out[2] = 0.0; continue; }
    const double dx = a.x[j] - g.xi, dy = a.y[j] - g.yi, dz = a.z[j] - g.zi;
    const double d2 = dx * dx + dy * dy + dz * dz;
    const double r = 0.5 * (g.hi + a.h[j]);
    const double w = support_weight<false>(d2, r, a.wf);
    double phi[M], cb[4];
    monomials<M>(g, dx, dy, dz, phi);
    chatbar(j, cb);
    double wb = 0.0, pb[M];
#pragma unroll
    for (int q = 0; q < M; ++q) pb[q] = 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (!((SEL >> s) & 1u)) continue;
      double pl = 0.0, mp = 0.0;
#pragma unroll
      for (int q = 0; q < M; ++q) { pl += phi[q] * lam[s][q]; mp += mu[s][q] * phi[q]; }
      wb += cb[s] * pl - mp * pl;
#pragma unroll
      for (int q = 0; q < M; ++q) pb[q] += cb[s] * w * lam[s][q] - w * (mu[s][q] * pl + lam[s][q] * mp);
    }
    double dd[3];
    monomials_grad_dot<M>(g, dx, dy, dz, pb, dd);
    const double f = wb * support_weight_dfac(d2, r, a.wf);
    out[0] = dd[0] + f * dx;
    out[1] = dd[1] + f * dy;
    out[2] = dd[2] + f * dz;
    own[0] += out[0];
    own[1] += out[1];
    own[2] += out[2];
  }
  // x_i loses every dbar(i, j), whether or not (j, i) is listed
#pragma unroll
  for (int c = 0; c < 3; ++c) own[c] = team_sum(own[c], kT);
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) a.xbar[3 * (int64_t)i + c] -= own[c];
  }
}

template <int M, unsigned SEL>
__global__ void __launch_bounds__(kBlock) k_adjoint_x(AArgs a) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t team = gt / kT;
  const int lane = (int)(gt % kT);
  if (team >= a.nrows) return;
  adjoint_row<M, SEL>(a, a.sched[team], a.gbase[team], lane);
}

template <int M>
void launch_adjoint_x(hipStream_t sm, dim3 grid, dim3 block, const AArgs &a) {
  if (a.mask == 8u) hipLaunchKernelGGL((k_adjoint_x<M, 8u>), grid, block, 0, sm, a);       // Laplacian
  else if (a.mask == 7u) hipLaunchKernelGGL((k_adjoint_x<M, 7u>), grid, block, 0, sm, a);  // gradient
  else hipLaunchKernelGGL((k_adjoint_x<M, 15u>), grid, block, 0, sm, a);
}

// xbar_j += sum over entries (j, i) of row j, i != j, of dbar(i, j) (x_j gains
// what row i differentiated with respect to it; the row's own entries were
// subtracted by the row kernel); rows in grouped order, a team of kT lanes
// per row; the twin dbar(i, j) sits at grev[g] (a Morton-near row).  An entry
// (j, i) without a twin (i a ghost particle whose row holds only itself)
// adds nothing.
__global__ void __launch_bounds__(kBlock) k_adjoint_gather(const int32_t *__restrict__ grouped,
                                                           const int64_t *__restrict__ grow_ptr,
                                                           const int32_t *__restrict__ grev,
                                                           const double *__restrict__ dbar, int64_t n,
                                                           double *__restrict__ xbar) {
  const int64_t gt = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t t = gt / kT;
  const int lane = (int)(gt % kT);
  if (t >= n) return;
  const int32_t j = grouped[t];
  const int64_t g0 = grow_ptr[t], g1 = grow_ptr[t + 1];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll 4
  for (int64_t gk = g0 + lane; gk < g1; gk += kT) {
    const int32_t tw = grev[gk];
    if (tw < 0) continue;
    s0 += dbar[3 * (int64_t)tw];
    s1 += dbar[3 * (int64_t)tw + 1];
    s2 += dbar[3 * (int64_t)tw + 2];
  }
  s0 = team_sum(s0, kT);
  s1 = team_sum(s1, kT);
  s2 = team_sum(s2, kT);
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
  if ((st = ensure_scratch(ctx, arena_bytes({sizeof(double) * 3 * (size_t)std::max<int64_t>(nbr->nnz, 1)}), &ar)))
    return st;
  AArgs a;
  a.x = p->x; a.y = p->y; a.z = p->z; a.h = p->h; a.nx = p->nx; a.ny = p->ny; a.nz = p->nz;
  a.row_ptr = nbr->row_ptr; a.col = nbr->col; a.n = p->n;
  a.wf = make_weight_fn(prm.alpha_w);
  a.mask = op_mask; a.u = u; a.ybar = ybar; a.status = status_n;
  a.dbar = ar.take<double>(3 * (size_t)std::max<int64_t>(nbr->nnz, 1));
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
    hipLaunchKernelGGL(k_adjoint_gather, dim3(grid_for(p->n * kT, kBlock)), dim3(kBlock), 0, ctx->stream,
                       nbr->grouped, nbr->grow_ptr, nbr->grev, a.dbar, p->n, xbar_3n);
    GF_LAUNCH_CHECK(ctx);
  }
  return GF_OK;
}
