// 3D -> 2D transition of flagged wall particles (Sec. 5.1, Alg. 3).
//
// Two gather passes over the (symmetric) same-model neighbourhoods, no
// atomics: (1) every interior / free-surface bulk particle b that has a
// flagged neighbour finds the nearest wall particle of S_b and is deleted if
// that wall particle is flagged; (2) every flagged particle i sums, in
// ascending index order, the particles b of S_i mapped to it (b is in S_i
// because neighbourhoods are symmetric).  Sums run in the same order as the
// definition reads, so the lumped masses are reproducible.
#include "internal.h"

namespace {
constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) k_owner(const double *__restrict__ x, const double *__restrict__ y,
                                                  const double *__restrict__ z, const int8_t *__restrict__ model,
                                                  const int8_t *__restrict__ kind, const int64_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ col, const uint8_t *__restrict__ flag,
                                                  int64_t n, uint8_t *__restrict__ keep, int32_t *__restrict__ owner) {
#pragma clang fp contract(off)
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  int32_t own = -1;
  if (model[b] == GF_MODEL_BULK && kind[b] != GF_KIND_WALL) {
    bool cand = false;
    for (int64_t k = row_ptr[b]; k < row_ptr[b + 1] && !cand; ++k) cand = flag[col[k]] == 1;
    if (cand) {
      int32_t best = -1;
      double bestd = INFINITY;
      const double xb = x[b], yb = y[b], zb = z[b];
      for (int64_t k = row_ptr[b]; k < row_ptr[b + 1]; ++k) {
        const int32_t j = col[k];
        if (kind[j] != GF_KIND_WALL || model[j] != GF_MODEL_BULK) continue;
        const double dx = x[j] - xb, dy = y[j] - yb, dz = z[j] - zb;
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        if (d2 < bestd) { bestd = d2; best = j; }  // ascending j: ties keep the smaller index
      }
      if (best >= 0 && flag[best] == 1) own = best;
    }
  }
  owner[b] = own;
  keep[b] = own < 0 ? 1 : 0;
}

__global__ void __launch_bounds__(kBlock) k_lump(const double *__restrict__ x, const double *__restrict__ y,
                                                 const double *__restrict__ z, const double *__restrict__ nx,
                                                 const double *__restrict__ ny, const double *__restrict__ nz,
                                                 const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                                 const uint8_t *__restrict__ flag, const int32_t *__restrict__ owner,
                                                 const uint8_t *__restrict__ keep, const double *__restrict__ mass,
                                                 const double *__restrict__ rho, const double *__restrict__ phi,
                                                 int64_t n, double *__restrict__ mass_out, double *__restrict__ rho_out,
                                                 double *__restrict__ phi_out, double *__restrict__ height_out,
                                                 double *__restrict__ diam_out) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (flag[i] != 1) {
    mass_out[i] = keep[i] ? mass[i] : 0.0;
    rho_out[i] = rho[i];
    phi_out[i] = phi[i];
    height_out[i] = 0.0;
    diam_out[i] = 0.0;
    return;
  }
  double m = mass[i], r = rho[i], p = phi[i], H = 0.0;
  int64_t cnt = 0;
  const double xi = x[i], yi = y[i], zi = z[i], a = nx[i], bb = ny[i], c = nz[i];
  for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
    const int32_t b = col[k];
    if (owner[b] != (int32_t)i) continue;
    m += mass[b];
    r += rho[b];
    p += phi[b];
    const double dn = fabs((x[b] - xi) * a + (y[b] - yi) * bb + (z[b] - zi) * c);
    H = fmax(H, dn);
    ++cnt;
  }
  mass_out[i] = m;
  rho_out[i] = r / (double)(1 + cnt);
  phi_out[i] = p / (double)(1 + cnt);
  height_out[i] = H;
  diam_out[i] = cbrt(6.0 * m / (3.14159265358979323846 * rho_out[i]));
}
}  // namespace

extern "C" gf_status gf_transition_3d_to_2d(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr, const uint8_t *flag,
                                            const double *mass, const double *rho, const double *phi,
                                            double *mass_out, double *rho_out, double *phi_out, double *height_out,
                                            double *diam_out, uint8_t *keep_out, int32_t *owner_out) {
  if (!ctx) return GF_EINVAL;
  gf_status st = check_particles(ctx, p, true, true);
  if (st) return st;
  if ((st = check_nbr(ctx, nbr, p->n))) return st;
  if (nbr->cross) return set_error(ctx, GF_EINVAL, "the transition uses same-model neighbourhoods");
  if (!flag || !mass || !rho || !phi || !mass_out || !rho_out || !phi_out || !height_out || !diam_out || !keep_out ||
      !owner_out)
    return set_error(ctx, GF_EINVAL, "all arrays are required");
  const dim3 grid(grid_for(p->n, kBlock)), block(kBlock);
  ProfScope prof(ctx, "transition_3d_to_2d");
  hipLaunchKernelGGL(k_owner, grid, block, 0, ctx->stream, p->x, p->y, p->z, p->model, p->kind, nbr->row_ptr, nbr->col,
                     flag, p->n, keep_out, owner_out);
  GF_LAUNCH_CHECK(ctx);
  hipLaunchKernelGGL(k_lump, grid, block, 0, ctx->stream, p->x, p->y, p->z, p->nx, p->ny, p->nz, nbr->row_ptr,
                     nbr->col, flag, owner_out, keep_out, mass, rho, phi, p->n, mass_out, rho_out, phi_out,
                     height_out, diam_out);
  GF_LAUNCH_CHECK(ctx);
  return GF_OK;
}
