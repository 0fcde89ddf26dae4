// Coupling layer of the two models: film height of the droplet model
// (Eq. Height), the 2D -> 3D transition (Sec. 5.2, Alg. 4) and the ghost
// particles of the buffer zone (Sec. 6.1, Alg. 5).
//
// The film height is a gather over the same-model lists, one team of lanes
// per particle in Morton order.  The transitions work on few particles (the
// flagged ones): per-particle counts, one device scan for the output offsets,
// a read-back of the total (the caller sizes its buffers), then one thread
// per source writes its new particles.  Sums over a neighbourhood run in
// ascending index order, so averaged and lumped values are reproducible.
#include "internal.h"

namespace {
constexpr int kBlock = 256;
constexpr int kHeightTeam = 8;
constexpr double kPi = 3.14159265358979323846;

__global__ void __launch_bounds__(kBlock) k_flag_rows(const int64_t *__restrict__ same_rp,
                                                      const int64_t *__restrict__ cross_rp, int64_t n,
                                                      uint8_t *__restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // S_i over both models holds S_i of i's own model plus the particles of
  // the other model within the support
  flag[i] = (cross_rp[i + 1] - cross_rp[i]) != (same_rp[i + 1] - same_rp[i]) ? 1 : 0;
}

// Eq. (Height): one team of kHeightTeam lanes per film particle, rows in
// grouped (Morton) order so that neighbouring teams share their neighbours'
// data; the launch covers the film rows of the grouped order only (a team per
// bulk row would find nothing to sum, and half the waves would do no work).
__global__ void __launch_bounds__(kBlock) k_film_height(const int32_t *__restrict__ grouped, int64_t n,
                                                        const double *__restrict__ x, const double *__restrict__ y,
                                                        const double *__restrict__ z, const double *__restrict__ h,
                                                        const int8_t *__restrict__ model,
                                                        const double *__restrict__ diam,
                                                        const int64_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col, double alpha,
                                                        double *__restrict__ height) {
  const int lane = threadIdx.x % kHeightTeam;
  const int64_t r = (int64_t)blockIdx.x * (kBlock / kHeightTeam) + threadIdx.x / kHeightTeam;
  if (r >= n) return;  // whole teams leave together
  const int32_t i = grouped[r];
  double acc = 0.0;
  if (model[i] == GF_MODEL_FILM) {
    const double xi = x[i], yi = y[i], zi = z[i];
    for (int64_t k = row_ptr[i] + lane; k < row_ptr[i + 1]; k += kHeightTeam) {
      const int32_t j = col[k];
      const double dx = x[j] - xi, dy = y[j] - yi, dz = z[j] - zi;
      const double r2 = (dx * dx + dy * dy) + dz * dz;
      const double hj2 = h[j] * h[j];
      const double d = diam[j];
      const double vol = kPi * d * d * d / 6.0;
      acc += alpha / (kPi * hj2) * exp(-alpha * r2 / hj2) * vol;
    }
#pragma unroll
    for (int o = kHeightTeam / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kHeightTeam);
  }
  if (lane == 0) height[i] = acc;
}

// the bulk rows' film height: zero
__global__ void __launch_bounds__(kBlock) k_zero_rows(const int32_t *__restrict__ grouped, int64_t n,
                                                      double *__restrict__ height) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) height[grouped[r]] = 0.0;
}

// gamma of Eq. (gamma) with psi~ of Eq. (psi~); false if it is not a valid
// count (psi~ <= 0, too many layers, not a number)
__device__ inline bool layers(double H, double h3, double r_min, double r_max, int64_t *gam) {
#pragma clang fp contract(off)
  const double psit = (r_min * h3 + r_max * h3) / 2.0;
  if (!(psit > 0.0)) return false;
  const double g = H > 0.0 ? ceil(H / psit) : 0.0;
  if (!(g >= 0.0 && g <= (double)GF_MAX_GAMMA)) return false;
  *gam = (int64_t)g;
  return true;
}

struct Src {
  const double *x, *y, *z, *nx, *ny, *nz;
  const int8_t *model, *kind;
  const double *mass, *rho, *phi;
  int nphi;
  int64_t n;
};

// the 1 + gamma 3D particles of film particle i, written from position t0
__device__ void expand_film(const Src &s, int64_t i, int64_t t0, int64_t gam, double H, double h3,
                            const NewOut &o) {
#pragma clang fp contract(off)
  const double psi = gam > 0 ? H / (double)gam : 0.0;
  const double xi = s.x[i], yi = s.y[i], zi = s.z[i], ax = s.nx[i], ay = s.ny[i], az = s.nz[i];
  const double m = s.mass[i] / (double)(1 + gam);
  for (int64_t k = 0; k <= gam; ++k) {
    const int64_t t = t0 + k;
    const double step = (double)k * psi;
    o.x[t] = xi + step * ax;
    o.y[t] = yi + step * ay;
    o.z[t] = zi + step * az;
    o.h[t] = h3;
    o.model[t] = GF_MODEL_BULK;
    o.kind[t] = k == 0 ? GF_KIND_WALL : (k == gam ? GF_KIND_FREE_SURFACE : GF_KIND_INTERIOR);
    o.nx[t] = ax;
    o.ny[t] = ay;
    o.nz[t] = az;
    o.mass[t] = m;
    o.rho[t] = s.rho[i];
    for (int f = 0; f < s.nphi; ++f) o.phi[(int64_t)f * o.cap + t] = s.phi[(int64_t)f * s.n + i];
    if (o.height) o.height[t] = 0.0;
    if (o.diam) o.diam[t] = 0.0;
    if (o.src) o.src[t] = (int32_t)i;
  }
}

// ---------------------------------------------------------------- 2D -> 3D
__global__ void __launch_bounds__(kBlock) k_count_2d3d(const int8_t *__restrict__ model,
                                                       const uint8_t *__restrict__ flag,
                                                       const double *__restrict__ H, const double *__restrict__ h3,
                                                       double r_min, double r_max, int64_t n,
                                                       int32_t *__restrict__ cnt, int32_t *__restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t c = 0;
  if (flag[i] == 2 && model[i] == GF_MODEL_FILM) {
    int64_t gam = 0;
    if (layers(H[i], h3[i], r_min, r_max, &gam)) c = (int32_t)(1 + gam);
    else atomicAdd(bad, 1);
  }
  cnt[i] = c;
}

__global__ void __launch_bounds__(kBlock) k_write_2d3d(Src s, const int64_t *__restrict__ off,
                                                       const double *__restrict__ H, const double *__restrict__ h3,
                                                       NewOut o) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n) return;
  const int64_t c = off[i + 1] - off[i];
  if (c == 0) return;
  expand_film(s, i, off[i], c - 1, H[i], h3[i], o);
}

// ---------------------------------------------------------------- buffer zone
// owner[b]: for a flagged interior / free-surface 3D particle, the nearest
// flagged wall particle of S_b (the wall ghost its ghost maps onto), else -1
// The nearest flagged wall particle of each flagged interior bulk particle b,
// over S_b.  Few particles are flagged, so a wave takes 64 particles, finds
// its flagged ones by a ballot and scans each of their rows with all 64
// lanes, each lane taking kOwnU entries per step with every load of the step
// issued before the first is used (entries past the row's end re-read its
// last entry and are skipped); the wave minimum of (distance, index) keeps
// the smallest index among equal distances, as an ascending scan does.
constexpr int kOwnU = 4;
__global__ void __launch_bounds__(kBlock) k_ghost_owner(const double *__restrict__ x, const double *__restrict__ y,
                                                        const double *__restrict__ z,
                                                        const int8_t *__restrict__ model,
                                                        const int8_t *__restrict__ kind,
                                                        const uint8_t *__restrict__ flag,
                                                        const int64_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ col, int64_t n,
                                                        int32_t *__restrict__ owner) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63;
  const int64_t b0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);  // the wave's first particle
  const int64_t bl = b0 + lane;
  const bool mine = bl < n && flag[bl] && model[bl] == GF_MODEL_BULK && kind[bl] != GF_KIND_WALL;
  if (bl < n && !mine) owner[bl] = -1;
  uint64_t todo = __ballot(mine);  // the same in every lane: the loop below is uniform
  while (todo) {
    const int src = __builtin_ctzll(todo);
    todo &= todo - 1;
    const int64_t b = b0 + src;
    const double xb = x[b], yb = y[b], zb = z[b];
    const int64_t k1 = row_ptr[b + 1];  // a step starts only at kb < k1: k1 - 1 is in the row
    int32_t best = -1;
    double bestd = INFINITY;
    for (int64_t kb = row_ptr[b] + lane; kb < k1; kb += kOwnU * 64) {
      int32_t j[kOwnU];
#pragma unroll
      for (int u = 0; u < kOwnU; ++u) j[u] = col[min(kb + u * 64, k1 - 1)];
      bool wall[kOwnU];
      double d2[kOwnU];
#pragma unroll
      for (int u = 0; u < kOwnU; ++u) {
        wall[u] = kb + u * 64 < k1 && flag[j[u]] && kind[j[u]] == GF_KIND_WALL;
        const double dx = x[j[u]] - xb, dy = y[j[u]] - yb, dz = z[j[u]] - zb;
        d2[u] = (dx * dx + dy * dy) + dz * dz;
      }
#pragma unroll
      for (int u = 0; u < kOwnU; ++u)  // ascending j: ties keep the smaller index
        if (wall[u] && d2[u] < bestd) { bestd = d2[u]; best = j[u]; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double od = __shfl_xor(bestd, o, 64);
      const int32_t oj = __shfl_xor(best, o, 64);
      if (oj >= 0 && (best < 0 || od < bestd || (od == bestd && oj < best))) {
        bestd = od;
        best = oj;
      }
    }
    if (lane == 0) owner[b] = best;
  }
}

__global__ void __launch_bounds__(kBlock) k_count_ghosts(const int8_t *__restrict__ model,
                                                         const int8_t *__restrict__ kind,
                                                         const uint8_t *__restrict__ flag,
                                                         const double *__restrict__ H,
                                                         const double *__restrict__ h3, double r_min,
                                                         double r_max, int64_t n, int32_t *__restrict__ cnt,
                                                         int32_t *__restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t c = 0;
  if (flag[i]) {
    if (model[i] == GF_MODEL_BULK) {
      c = kind[i] == GF_KIND_WALL ? 1 : 0;
    } else {
      int64_t gam = 0;
      if (layers(H[i], h3[i], r_min, r_max, &gam)) c = (int32_t)(1 + gam);
      else atomicAdd(bad, 1);
    }
  }
  cnt[i] = c;
}

__global__ void __launch_bounds__(kBlock) k_write_ghosts(Src s, const int64_t *__restrict__ off,
                                                         const uint8_t *__restrict__ flag,
                                                         const int32_t *__restrict__ owner,
                                                         const int64_t *__restrict__ row_ptr,
                                                         const int32_t *__restrict__ col,
                                                         const double *__restrict__ H,
                                                         const double *__restrict__ h_other, NewOut o) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n) return;
  const int64_t t = off[i];
  const int64_t c = off[i + 1] - t;
  if (c == 0) return;
  if (s.model[i] != GF_MODEL_BULK) {
    expand_film(s, i, t, c - 1, H[i], h_other[i], o);
    return;
  }
  // wall ghost i turns into a 2D ghost: data of the ghosts mapped onto it
  // (members of S_i, by symmetry of the neighbourhoods)
  const double xi = s.x[i], yi = s.y[i], zi = s.z[i], ax = s.nx[i], ay = s.ny[i], az = s.nz[i];
  double m = s.mass[i], r = s.rho[i], Hn = 0.0;
  int64_t cntT = 0;
  const int64_t k0 = row_ptr[i], k1 = row_ptr[i + 1];
  for (int64_t k = k0; k < k1; ++k) {
    const int32_t b = col[k];
    if (!flag[b] || owner[b] != (int32_t)i) continue;
    m += s.mass[b];
    r += s.rho[b];
    const double dn = fabs((s.x[b] - xi) * ax + (s.y[b] - yi) * ay + (s.z[b] - zi) * az);
    Hn = fmax(Hn, dn);
    ++cntT;
  }
  const double rho_new = r / (double)(1 + cntT);
  for (int f = 0; f < s.nphi; ++f) {
    const double *ph = s.phi + (int64_t)f * s.n;
    double acc = ph[i];
    for (int64_t k = k0; k < k1; ++k) {
      const int32_t b = col[k];
      if (flag[b] && owner[b] == (int32_t)i) acc += ph[b];
    }
    o.phi[(int64_t)f * o.cap + t] = acc / (double)(1 + cntT);
  }
  o.x[t] = xi;
  o.y[t] = yi;
  o.z[t] = zi;
  o.h[t] = h_other[i];
  o.model[t] = GF_MODEL_FILM;
  o.kind[t] = GF_KIND_WALL;
  o.nx[t] = ax;
  o.ny[t] = ay;
  o.nz[t] = az;
  o.mass[t] = m;
  o.rho[t] = rho_new;
  if (o.height) o.height[t] = Hn;
  if (o.diam) o.diam[t] = cbrt(6.0 * m / (kPi * rho_new));
  if (o.src) o.src[t] = (int32_t)i;
}

// counts -> offsets (device scan) -> total and error count read back
gf_status offsets(gf_ctx *ctx, const int32_t *cnt, int64_t *off, int64_t n, int64_t *tmp, const int32_t *bad,
                  int64_t *total, int32_t *nbad) {
  gf_status st = scan_i32_to_i64(ctx, cnt, off, n, tmp);
  if (st) return st;
  if ((st = ensure_host(ctx, 64))) return st;
  char *hp = (char *)ctx->host_pinned;
  GF_HIP(ctx, hipMemcpyAsync(hp, off + n, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
  GF_HIP(ctx, hipMemcpyAsync(hp + 8, bad, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
  GF_HIP(ctx, hipStreamSynchronize(ctx->stream));
  *total = *(int64_t *)hp;
  *nbad = *(int32_t *)(hp + 8);
  return GF_OK;
}
__global__ void __launch_bounds__(64) k_zero_bad(int32_t *bad) {
  if (threadIdx.x == 0) bad[0] = 0;
}
}  // namespace

gf_status check_out(gf_ctx *ctx, const gf_new_particles *o, int nphi, int64_t *count) {
  if (!o || !count) return set_error(ctx, GF_EINVAL, "out and count are required");
  if (o->cap < 0) return set_error(ctx, GF_EINVAL, "out->cap is negative");
  if (o->cap > 0 && (!o->x || !o->y || !o->z || !o->h || !o->model || !o->kind || !o->nx || !o->ny || !o->nz ||
                     !o->mass || !o->rho || (nphi > 0 && !o->phi)))
    return set_error(ctx, GF_EINVAL, "out is missing a required array");
  return GF_OK;
}

extern "C" gf_status gf_film_height(gf_ctx *ctx, const gf_particles *p, const gf_nbr *same, const double *diam,
                                    double alpha, double *height_out) {
  if (!ctx) return GF_EINVAL;
  gf_status st = check_particles(ctx, p, false, false);
  if (st) return st;
  if ((st = check_nbr(ctx, same, p->n))) return st;
  if (same->cross) return set_error(ctx, GF_EINVAL, "the film height uses same-model neighbourhoods");
  if (!diam || !height_out) return set_error(ctx, GF_EINVAL, "diam and height_out are required");
  if (!(alpha > 0.0) || !std::isfinite(alpha)) return set_error(ctx, GF_EINVAL, "alpha must be positive and finite");
  const int64_t rows_per_block = kBlock / kHeightTeam;
  // the grouped order holds the bulk rows, then the film rows
  const int64_t r0 = same->group_start[GF_NBAND], r1 = same->group_start[2 * GF_NBAND];
  ProfScope prof(ctx, "film_height");
  if (r0 > 0)
    hipLaunchKernelGGL(k_zero_rows, dim3(grid_for(r0, kBlock)), dim3(kBlock), 0, ctx->stream, same->grouped, r0,
                       height_out);
  if (r1 > r0)
    hipLaunchKernelGGL(k_film_height, dim3(grid_for((r1 - r0 + rows_per_block - 1) / rows_per_block, 1)), dim3(kBlock),
                       0, ctx->stream, same->grouped + r0, r1 - r0, p->x, p->y, p->z, p->h, p->model, diam,
                       same->row_ptr, same->col, alpha, height_out);
  GF_LAUNCH_CHECK(ctx);
  return GF_OK;
}

extern "C" gf_status gf_transition_2d_to_3d(gf_ctx *ctx, const gf_particles *p, const uint8_t *flag,
                                            const double *film_height, const double *h3d, double r_min,
                                            double r_max, const double *mass, const double *rho,
                                            const double *phi, int nphi, gf_new_particles *out,
                                            int64_t *count) {
  if (!ctx) return GF_EINVAL;
  gf_status st = check_particles(ctx, p, false, true);
  if (st) return st;
  if (!flag || !film_height || !h3d || !mass || !rho) return set_error(ctx, GF_EINVAL, "a required array is NULL");
  if (nphi < 0 || (nphi > 0 && !phi)) return set_error(ctx, GF_EINVAL, "nphi < 0 or phi missing");
  if (!(r_min > 0.0) || !(r_max >= r_min) || !std::isfinite(r_max))
    return set_error(ctx, GF_EINVAL, "need 0 < r_min <= r_max");
  if ((st = check_out(ctx, out, nphi, count))) return st;
  *count = 0;
  const int64_t n = p->n;
  Arena ar;
  std::vector<size_t> sz = {sizeof(int32_t) * n, sizeof(int64_t) * (n + 1), sizeof(int64_t) * scan_tmp_elems(n + 1),
                            64};
  if ((st = ensure_scratch(ctx, arena_bytes(sz), &ar))) return st;
  int32_t *cnt = ar.take<int32_t>(n);
  int64_t *off = ar.take<int64_t>(n + 1);
  int64_t *tmp = ar.take<int64_t>(scan_tmp_elems(n + 1));
  int32_t *bad = ar.take<int32_t>(16);
  const dim3 grid(grid_for(n, kBlock)), block(kBlock);
  int64_t total = 0;
  int32_t nbad = 0;
  {
    ProfScope prof(ctx, "transition_2d_to_3d_count");
    hipLaunchKernelGGL(k_zero_bad, dim3(1), dim3(64), 0, ctx->stream, bad);
    hipLaunchKernelGGL(k_count_2d3d, grid, block, 0, ctx->stream, p->model, flag, film_height, h3d, r_min, r_max, n,
                       cnt, bad);
    GF_LAUNCH_CHECK(ctx);
  }
  if ((st = offsets(ctx, cnt, off, n, tmp, bad, &total, &nbad))) return st;
  if (nbad) return set_error(ctx, GF_EINVAL, "%d film particles have no valid layer count (height, h3d)", nbad);
  *count = total;
  if (total > out->cap)
    return set_error(ctx, GF_ECAPACITY, "%lld new particles, capacity %lld", (long long)total, (long long)out->cap);
  if (total == 0) return GF_OK;
  Src s{p->x, p->y, p->z, p->nx, p->ny, p->nz, p->model, p->kind, mass, rho, phi, nphi, n};
  ProfScope prof(ctx, "transition_2d_to_3d_write");
  hipLaunchKernelGGL(k_write_2d3d, grid, block, 0, ctx->stream, s, off, film_height, h3d, new_out(out));
  GF_LAUNCH_CHECK(ctx);
  return GF_OK;
}

extern "C" gf_status gf_buffer_flags(gf_ctx *ctx, const gf_particles *p, const gf_nbr *same, const gf_nbr *cross,
                                     uint8_t *flag_out) {
  if (!ctx) return GF_EINVAL;
  gf_status st = check_particles(ctx, p, false, false);
  if (st) return st;
  if ((st = check_nbr(ctx, same, p->n)) || (st = check_nbr(ctx, cross, p->n))) return st;
  if (same->cross || !cross->cross)
    return set_error(ctx, GF_EINVAL, "need same-model and cross-model neighbourhoods, in that order");
  if (!flag_out) return set_error(ctx, GF_EINVAL, "flag_out is NULL");
  ProfScope prof(ctx, "buffer_flags");
  hipLaunchKernelGGL(k_flag_rows, dim3(grid_for(p->n, kBlock)), dim3(kBlock), 0, ctx->stream, same->row_ptr,
                     cross->row_ptr, p->n, flag_out);
  GF_LAUNCH_CHECK(ctx);
  return GF_OK;
}

extern "C" gf_status gf_buffer_zone(gf_ctx *ctx, const gf_particles *p, const gf_nbr *same, const gf_nbr *cross,
                                    const double *film_height, const double *h_other, double r_min, double r_max,
                                    const double *mass, const double *rho, const double *phi, int nphi,
                                    gf_new_particles *out, int64_t *count, uint8_t *flag_out) {
  if (!ctx) return GF_EINVAL;
  gf_status st = check_particles(ctx, p, true, true);
  if (st) return st;
  if ((st = check_nbr(ctx, same, p->n)) || (st = check_nbr(ctx, cross, p->n))) return st;
  if (same->cross || !cross->cross)
    return set_error(ctx, GF_EINVAL, "need same-model and cross-model neighbourhoods, in that order");
  if (!film_height || !h_other || !mass || !rho) return set_error(ctx, GF_EINVAL, "a required array is NULL");
  if (nphi < 0 || (nphi > 0 && !phi)) return set_error(ctx, GF_EINVAL, "nphi < 0 or phi missing");
  if (!(r_min > 0.0) || !(r_max >= r_min) || !std::isfinite(r_max))
    return set_error(ctx, GF_EINVAL, "need 0 < r_min <= r_max");
  if ((st = check_out(ctx, out, nphi, count))) return st;
  *count = 0;
  const int64_t n = p->n;
  Arena ar;
  std::vector<size_t> sz = {sizeof(uint8_t) * n, sizeof(int32_t) * n, sizeof(int32_t) * n, sizeof(int64_t) * (n + 1),
                            sizeof(int64_t) * scan_tmp_elems(n + 1), 64};
  if ((st = ensure_scratch(ctx, arena_bytes(sz), &ar))) return st;
  uint8_t *flag = ar.take<uint8_t>(n);
  int32_t *owner = ar.take<int32_t>(n);
  int32_t *cnt = ar.take<int32_t>(n);
  int64_t *off = ar.take<int64_t>(n + 1);
  int64_t *tmp = ar.take<int64_t>(scan_tmp_elems(n + 1));
  int32_t *bad = ar.take<int32_t>(16);
  if (flag_out) flag = flag_out;
  const dim3 grid(grid_for(n, kBlock)), block(kBlock);
  {
    ProfScope prof(ctx, "buffer_flags_owner");
    hipLaunchKernelGGL(k_zero_bad, dim3(1), dim3(64), 0, ctx->stream, bad);
    hipLaunchKernelGGL(k_flag_rows, grid, block, 0, ctx->stream, same->row_ptr, cross->row_ptr, n, flag);
    hipLaunchKernelGGL(k_ghost_owner, grid, block, 0, ctx->stream, p->x, p->y, p->z, p->model, p->kind, flag,
                       same->row_ptr, same->col, n, owner);
    hipLaunchKernelGGL(k_count_ghosts, grid, block, 0, ctx->stream, p->model, p->kind, flag, film_height, h_other,
                       r_min, r_max, n, cnt, bad);
    GF_LAUNCH_CHECK(ctx);
  }
  int64_t total = 0;
  int32_t nbad = 0;
  if ((st = offsets(ctx, cnt, off, n, tmp, bad, &total, &nbad))) return st;
  if (nbad) return set_error(ctx, GF_EINVAL, "%d film particles have no valid layer count (height, h_other)", nbad);
  *count = total;
  if (total > out->cap)
    return set_error(ctx, GF_ECAPACITY, "%lld ghost particles, capacity %lld", (long long)total, (long long)out->cap);
  if (total == 0) return GF_OK;
  Src s{p->x, p->y, p->z, p->nx, p->ny, p->nz, p->model, p->kind, mass, rho, phi, nphi, n};
  ProfScope prof(ctx, "buffer_write");
  hipLaunchKernelGGL(k_write_ghosts, grid, block, 0, ctx->stream, s, off, flag, owner, same->row_ptr, same->col,
                     film_height, h_other, new_out(out));
  GF_LAUNCH_CHECK(ctx);
  return GF_OK;
}
