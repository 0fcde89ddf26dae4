// 3D -> 2D transition of flagged wall particles (Sec. 5.1, Alg. 3), as
// per-particle outputs (gf_transition_3d_to_2d) or applied to the cloud
// (gf_transition_3d_to_2d_cloud: deleted particles compacted away, the
// transitioning ones turned into film particles, every field mapped).
//
// Two gather passes over the (symmetric) same-model neighbourhoods, no
// atomics: (1) every interior / free-surface bulk particle b that has a
// flagged neighbour finds the nearest wall particle of S_b and is deleted if
// that wall particle is flagged; (2) every flagged particle i sums, in
// ascending index order, the particles b of S_i mapped to it (b is in S_i
// because neighbourhoods are symmetric).  Sums run in the same order as the
// definition reads, so the lumped masses are reproducible.
//
// Each scan runs on a team of kTT lanes per particle (lane l takes the
// entries k0 + l, k0 + l + kTT, ...), so a particle waits for about
// |S|/kTT dependent loads instead of |S|; the owner search takes its
// entries four at a time per lane, every load of a step issued before the
// first is used.  The nearest wall particle is the
// team minimum of (distance, index), which keeps the smallest index among
// equal distances as an ascending scan does; the lumped sums walk each chunk
// of kTT entries lane by lane, i.e. in ascending entry order.
#include "internal.h"

namespace {
constexpr int kBlock = 256;
constexpr int kTT = 8;  // lanes per particle in the neighbourhood scans
static_assert(64 % kTT == 0, "a team lies within a wave");
constexpr int kTU = 4;  // entries per lane and step of the owner search

__global__ void __launch_bounds__(kBlock) k_owner(const double *__restrict__ x, const double *__restrict__ y,
                                                  const double *__restrict__ z, const int8_t *__restrict__ model,
                                                  const int8_t *__restrict__ kind, const int64_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ col, const uint8_t *__restrict__ flag,
                                                  int64_t n, uint8_t *__restrict__ keep, int32_t *__restrict__ owner) {
#pragma clang fp contract(off)
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t b = gt / kTT;
  const int lane = (int)(gt % kTT);
  if (b >= n) return;  // (the whole team)
  int32_t own = -1;
  if (model[b] == GF_MODEL_BULK && kind[b] != GF_KIND_WALL) {
    const int64_t k0 = row_ptr[b], k1 = row_ptr[b + 1];
    // entries past the row's end re-read its last entry (a step starts only at kb < k1), which
    // the OR sees twice and the nearest-wall search skips
    int cand = 0;
    for (int64_t kb = k0 + lane; kb < k1; kb += kTU * kTT) {
      int32_t j[kTU];
#pragma unroll
      for (int u = 0; u < kTU; ++u) j[u] = col[min(kb + u * kTT, k1 - 1)];
#pragma unroll
      for (int u = 0; u < kTU; ++u) cand |= flag[j[u]] == 1;
    }
    for (int o = kTT >> 1; o > 0; o >>= 1) cand |= __shfl_xor(cand, o, kTT);
    if (cand) {
      int32_t best = -1;
      double bestd = INFINITY;
      const double xb = x[b], yb = y[b], zb = z[b];
      for (int64_t kb = k0 + lane; kb < k1; kb += kTU * kTT) {
        int32_t j[kTU];
#pragma unroll
        for (int u = 0; u < kTU; ++u) j[u] = col[min(kb + u * kTT, k1 - 1)];
        bool wall[kTU];
        double d2[kTU];
#pragma unroll
        for (int u = 0; u < kTU; ++u) {
          wall[u] = kb + u * kTT < k1 && kind[j[u]] == GF_KIND_WALL && model[j[u]] == GF_MODEL_BULK;
          const double dx = x[j[u]] - xb, dy = y[j[u]] - yb, dz = z[j[u]] - zb;
          d2[u] = (dx * dx + dy * dy) + dz * dz;
        }
#pragma unroll
        for (int u = 0; u < kTU; ++u)  // ascending j: ties keep the smaller index
          if (wall[u] && d2[u] < bestd) { bestd = d2[u]; best = j[u]; }
      }
      for (int o = kTT >> 1; o > 0; o >>= 1) {
        const double od = __shfl_xor(bestd, o, kTT);
        const int32_t oj = __shfl_xor(best, o, kTT);
        if (oj >= 0 && (best < 0 || od < bestd || (od == bestd && oj < best))) {
          bestd = od;
          best = oj;
        }
      }
      if (best >= 0 && flag[best] == 1) own = best;
    }
  }
  if (lane == 0) {
    owner[b] = own;
    keep[b] = own < 0 ? 1 : 0;
  }
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
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = gt / kTT;
  const int lane = (int)(gt % kTT);
  if (i >= n) return;  // (the whole team)
  if (flag[i] != 1) {
    if (lane == 0) {
      mass_out[i] = keep[i] ? mass[i] : 0.0;
      rho_out[i] = rho[i];
      phi_out[i] = phi[i];
      height_out[i] = 0.0;
      diam_out[i] = 0.0;
    }
    return;
  }
  double m = mass[i], r = rho[i], p = phi[i], H = 0.0;
  int64_t cnt = 0;
  const double xi = x[i], yi = y[i], zi = z[i], a = nx[i], bb = ny[i], c = nz[i];
  const int64_t k0 = row_ptr[i], k1 = row_ptr[i + 1];
  for (int64_t kc = k0; kc < k1; kc += kTT) {
    const int64_t k = kc + lane;
    int hit = 0;
    double mb = 0.0, rb = 0.0, pb = 0.0, db = 0.0;
    if (k < k1) {
      const int32_t b = col[k];
      if (owner[b] == (int32_t)i) {
        hit = 1;
        mb = mass[b];
        rb = rho[b];
        pb = phi[b];
        db = fabs((x[b] - xi) * a + (y[b] - yi) * bb + (z[b] - zi) * c);
      }
    }
    for (int l = 0; l < kTT; ++l) {  // ascending entry order
      if (__shfl(hit, l, kTT)) {
        m += __shfl(mb, l, kTT);
        r += __shfl(rb, l, kTT);
        p += __shfl(pb, l, kTT);
        H = fmax(H, __shfl(db, l, kTT));
        ++cnt;
      }
    }
  }
  if (lane == 0) {
    mass_out[i] = m;
    rho_out[i] = r / (double)(1 + cnt);
    phi_out[i] = p / (double)(1 + cnt);
    height_out[i] = H;
    diam_out[i] = cbrt(6.0 * m / (3.14159265358979323846 * rho_out[i]));
  }
}

__global__ void __launch_bounds__(kBlock) k_keep32(const uint8_t *__restrict__ keep, int64_t n,
                                                   int32_t *__restrict__ k32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) k32[i] = keep[i];
}

struct CloudIn {
  const double *x, *y, *z, *nx, *ny, *nz, *h;
  const int8_t *model, *kind;
  const double *mass, *rho, *phi;
  int nphi;
  const double *film_height, *diam, *h_film;
  int64_t n;
};

// The new cloud: kept particles at pos[i].  k_cloud_copy copies every kept
// particle that is not flagged; k_cloud_lump (a team per particle) turns the
// flagged ones into film particles with the data of the particles mapped
// onto them (ascending index order, as in k_lump).
__global__ void __launch_bounds__(kBlock) k_cloud_copy(CloudIn c, const uint8_t *__restrict__ flag,
                                                       const uint8_t *__restrict__ keep,
                                                       const int64_t *__restrict__ pos, NewOut o) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= c.n || !keep[i] || flag[i] == 1) return;
  const int64_t t = pos[i];
  const bool film = c.model[i] == GF_MODEL_FILM;
  o.x[t] = c.x[i];
  o.y[t] = c.y[i];
  o.z[t] = c.z[i];
  o.nx[t] = c.nx[i];
  o.ny[t] = c.ny[i];
  o.nz[t] = c.nz[i];
  if (o.src) o.src[t] = (int32_t)i;
  o.h[t] = c.h[i];
  o.model[t] = c.model[i];
  o.kind[t] = c.kind[i];
  o.mass[t] = c.mass[i];
  o.rho[t] = c.rho[i];
  for (int f = 0; f < c.nphi; ++f) o.phi[(int64_t)f * o.cap + t] = c.phi[(int64_t)f * c.n + i];
  if (o.height) o.height[t] = (film && c.film_height) ? c.film_height[i] : 0.0;
  if (o.diam) o.diam[t] = (film && c.diam) ? c.diam[i] : 0.0;
}

__global__ void __launch_bounds__(kBlock) k_cloud_lump(CloudIn c, const int64_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ col,
                                                       const uint8_t *__restrict__ flag,
                                                       const int32_t *__restrict__ owner,
                                                       const uint8_t *__restrict__ keep,
                                                       const int64_t *__restrict__ pos, NewOut o) {
#pragma clang fp contract(off)
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = gt / kTT;
  const int lane = (int)(gt % kTT);
  if (i >= c.n || flag[i] != 1 || !keep[i]) return;  // (the whole team)
  const int64_t t = pos[i];
  double m = c.mass[i], r = c.rho[i], H = 0.0;
  int64_t cnt = 0;
  const double xi = c.x[i], yi = c.y[i], zi = c.z[i], a = c.nx[i], bb = c.ny[i], cc = c.nz[i];
  const int64_t k0 = row_ptr[i], k1 = row_ptr[i + 1];
  for (int64_t kc = k0; kc < k1; kc += kTT) {
    const int64_t k = kc + lane;
    int hit = 0;
    double mb = 0.0, rb = 0.0, db = 0.0;
    if (k < k1) {
      const int32_t b = col[k];
      if (owner[b] == (int32_t)i) {
        hit = 1;
        mb = c.mass[b];
        rb = c.rho[b];
        db = fabs((c.x[b] - xi) * a + (c.y[b] - yi) * bb + (c.z[b] - zi) * cc);
      }
    }
    for (int l = 0; l < kTT; ++l) {  // ascending entry order
      if (__shfl(hit, l, kTT)) {
        m += __shfl(mb, l, kTT);
        r += __shfl(rb, l, kTT);
        H = fmax(H, __shfl(db, l, kTT));
        ++cnt;
      }
    }
  }
  const double rho_new = r / (double)(1 + cnt);
  for (int f = 0; f < c.nphi; ++f) {
    const double *ph = c.phi + (int64_t)f * c.n;
    double acc = ph[i];
    for (int64_t kc = k0; kc < k1; kc += kTT) {
      const int64_t k = kc + lane;
      int hit = 0;
      double vb = 0.0;
      if (k < k1) {
        const int32_t b = col[k];
        if (owner[b] == (int32_t)i) {
          hit = 1;
          vb = ph[b];
        }
      }
      for (int l = 0; l < kTT; ++l)
        if (__shfl(hit, l, kTT)) acc += __shfl(vb, l, kTT);
    }
    if (lane == 0) o.phi[(int64_t)f * o.cap + t] = acc / (double)(1 + cnt);
  }
  if (lane != 0) return;
  o.x[t] = c.x[i];
  o.y[t] = c.y[i];
  o.z[t] = c.z[i];
  o.nx[t] = c.nx[i];
  o.ny[t] = c.ny[i];
  o.nz[t] = c.nz[i];
  if (o.src) o.src[t] = (int32_t)i;
  o.h[t] = c.h_film ? c.h_film[i] : c.h[i];
  o.model[t] = GF_MODEL_FILM;
  o.kind[t] = GF_KIND_WALL;
  o.mass[t] = m;
  o.rho[t] = rho_new;
  if (o.height) o.height[t] = H;
  if (o.diam) o.diam[t] = cbrt(6.0 * m / (3.14159265358979323846 * rho_new));
}
}  // namespace

extern "C" gf_status gf_transition_3d_to_2d_cloud(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr,
                                                  const uint8_t *flag, const double *mass, const double *rho,
                                                  const double *phi, int nphi, const double *film_height,
                                                  const double *diam, const double *h_film,
                                                  gf_new_particles *out, int64_t *count) {
  if (!ctx) return GF_EINVAL;
  gf_status st = check_particles(ctx, p, true, true);
  if (st) return st;
  if ((st = check_nbr(ctx, nbr, p->n))) return st;
  if (nbr->cross) return set_error(ctx, GF_EINVAL, "the transition uses same-model neighbourhoods");
  if (!flag || !mass || !rho) return set_error(ctx, GF_EINVAL, "flag, mass and rho are required");
  if (nphi < 0 || (nphi > 0 && !phi)) return set_error(ctx, GF_EINVAL, "nphi < 0 or phi missing");
  if ((st = check_out(ctx, out, nphi, count))) return st;
  *count = 0;
  const int64_t n = p->n;
  Arena ar;
  std::vector<size_t> sz = {sizeof(uint8_t) * n, sizeof(int32_t) * n, sizeof(int32_t) * n, sizeof(int64_t) * (n + 1),
                            sizeof(int64_t) * scan_tmp_elems(n + 1)};
  if ((st = ensure_scratch(ctx, arena_bytes(sz), &ar))) return st;
  uint8_t *keep = ar.take<uint8_t>(n);
  int32_t *owner = ar.take<int32_t>(n);
  int32_t *k32 = ar.take<int32_t>(n);
  int64_t *pos = ar.take<int64_t>(n + 1);
  int64_t *tmp = ar.take<int64_t>(scan_tmp_elems(n + 1));
  const dim3 grid(grid_for(n, kBlock)), tgrid(grid_for(n * kTT, kBlock)), block(kBlock);
  {
    ProfScope prof(ctx, "transition_cloud_owner");
    hipLaunchKernelGGL(k_owner, tgrid, block, 0, ctx->stream, p->x, p->y, p->z, p->model, p->kind, nbr->row_ptr,
                       nbr->col, flag, n, keep, owner);
    hipLaunchKernelGGL(k_keep32, grid, block, 0, ctx->stream, keep, n, k32);
    GF_LAUNCH_CHECK(ctx);
    if ((st = scan_i32_to_i64(ctx, k32, pos, n, tmp))) return st;
  }
  if ((st = ensure_host(ctx, 64))) return st;
  GF_HIP(ctx, hipMemcpyAsync(ctx->host_pinned, pos + n, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
  GF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const int64_t total = *(int64_t *)ctx->host_pinned;
  *count = total;
  if (total > out->cap)
    return set_error(ctx, GF_ECAPACITY, "%lld particles remain, capacity %lld", (long long)total, (long long)out->cap);
  CloudIn c{p->x, p->y, p->z, p->nx, p->ny, p->nz, p->h, p->model, p->kind, mass, rho, phi, nphi,
            film_height, diam, h_film, n};
  ProfScope prof(ctx, "transition_cloud_write");
  hipLaunchKernelGGL(k_cloud_copy, grid, block, 0, ctx->stream, c, flag, keep, pos, new_out(out));
  hipLaunchKernelGGL(k_cloud_lump, tgrid, block, 0, ctx->stream, c, nbr->row_ptr, nbr->col, flag, owner, keep, pos,
                     new_out(out));
  GF_LAUNCH_CHECK(ctx);
  return GF_OK;
}

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
  const dim3 tgrid(grid_for(p->n * kTT, kBlock)), block(kBlock);
  ProfScope prof(ctx, "transition_3d_to_2d");
  hipLaunchKernelGGL(k_owner, tgrid, block, 0, ctx->stream, p->x, p->y, p->z, p->model, p->kind, nbr->row_ptr, nbr->col,
                     flag, p->n, keep_out, owner_out);
  GF_LAUNCH_CHECK(ctx);
  hipLaunchKernelGGL(k_lump, tgrid, block, 0, ctx->stream, p->x, p->y, p->z, p->nx, p->ny, p->nz, nbr->row_ptr,
                     nbr->col, flag, owner_out, keep_out, mass, rho, phi, p->n, mass_out, rho_out, phi_out,
                     height_out, diam_out);
  GF_LAUNCH_CHECK(ctx);
  return GF_OK;
}
