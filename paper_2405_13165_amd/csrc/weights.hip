// Second-order GFDM stencils (Eq. GFDM_Definition) and their fused
// application.
//
// Batched path: particles are grouped by model (10 monomials in 3D, 6 on the
// film) and by neighbour-count band; inside a group they are taken in Morton
// order.  Each particle is handled by a team of T lanes of a wave: the lanes
// stride over the neighbours and accumulate the weighted moments of the
// offsets, from which the team assembles G = M^T W M, inverts it by
// Gauss-Jordan (exact 1-norm condition number of the Gram matrix of the
// offsets scaled by 1/h_i), and a second pass over the neighbours writes
// c_j = w_j phi_j^T lambda (and, fused, applies the stencils to a field).  Rows of the tiled bands are processed
// one neighbour tile per block: the tile's distinct neighbour positions are
// staged in LDS once and both passes read them there.  Particles whose
// condition number exceeds kappa_max, or whose pivots are not positive, are
// queued and re-solved by a Householder QR of sqrt(W) M (one wave per
// particle), which also decides rank deficiency.
//
// Plain path: one work-item per particle in the caller's order, an FP64 Gram
// matrix with LDL^T solves, FP64 output.
#include <algorithm>
#include <type_traits>
#include <mutex>

#include "stencil_common.h"

using namespace gfdm_dev;

namespace {
constexpr int kBlock = 256;
constexpr int kQrBlock = 64;
constexpr size_t kQrLdsMax = 48 * 1024;  // the QR panel goes to LDS up to this size
constexpr int kQrStride = 15;  // per neighbour: 10 columns, 4 targets, sqrt(w)

struct WArgs {
  const double *x, *y, *z, *h, *nx, *ny, *nz;
  const double4 *pos;  // (x, y, z, h) packed per particle for the batched kernels
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

// The stencils are written once and read by a later kernel, after this one has
// left L2.  NT: non-temporal stores, which keep them from evicting the
// neighbour positions and tile lists the kernel re-reads; they bypass the
// merging of partial lines in L2, so they pay only where each store
// instruction covers whole aligned lines (the team kernels' pass 2).  Scattered
// stores (one row per lane) go through L2.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <int OUT, bool NT = false>
__device__ inline void store_w(void *w, int64_t k, double c0, double c1, double c2, double c3) {
  if constexpr (OUT == GF_F32) {
    const f32x4 v = {(float)c0, (float)c1, (float)c2, (float)c3};
    f32x4 *p = reinterpret_cast<f32x4 *>(w) + k;
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
  } else {
    f64x2 *p = reinterpret_cast<f64x2 *>(w) + 2 * k;
    const f64x2 v0 = {c0, c1}, v1 = {c2, c3};
    if constexpr (NT) {
      __builtin_nontemporal_store(v0, p);
      __builtin_nontemporal_store(v1, p + 1);
    } else {
      p[0] = v0;
      p[1] = v1;
    }
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

// ------------------------------------------------------------------ batched
// Per-team LDS (doubles): one area that holds in turn the reduction buffer,
// the moments, the Gauss-Jordan pivot row, the target solutions and (tiled
// rows, teams of 8 or more lanes) the row's slots during pass 2 (an even
// count, so that every team area starts on a 16-byte boundary); then KC
// cached support weights per lane.
template <int M>
constexpr int team_lds_doubles(int T, int KC) {
  const int slots = T >= 8 ? (kTileBandRow / (2 * T) + 1) * T / 2 : 0;  // slot pairs, 4 bytes each
  return ((cmax(cmax(cmax(nmom<M>(), 4 * M), cmax(red_lanes(T) * red_lanes(T), M + 1)), slots) + 1) & ~1) + KC * T;
}

// Unnormalised support weight of a neighbour at offset d with support h_j.
// Equal supports (the common case; UNI: known for the whole tile, no test per
// neighbour): q^2 = |d|^2 / h_i^2.  Otherwise
// r_ij = (h_i + h_j) / 2 and q^2 = |d|^2 (2 / (h_i + h_j))^2, with the
// reciprocal taken from the hardware estimate and two Newton steps (each
// squares the relative error) instead of a full division.
template <bool FASTW, bool UNI>
__device__ inline double nbr_weight_raw(const WArgs &a, const RowGeom &g, double cs_row, double hj, double dx,
                                        double dy, double dz) {
  // cs: 1 / r_ij^2 times -a log2(e); cs_row = that of r_ij = h_i
  const double d2 = fma(dz, dz, fma(dy, dy, dx * dx));
  double cs;
  if (UNI || hj == g.hi) {
    cs = cs_row;
  } else {
    const double sh = g.hi + hj;
    double r = __builtin_amdgcn_rcp(sh);
    r = fma(r, fma(-sh, r, 1.0), r);
    r = fma(r, fma(-sh, r, 1.0), r);
    const double tr = 2.0 * r;
    cs = (tr * tr) * a.wf.nl2a;
  }
  return support_weight_raw<FASTW>(d2, cs, a.wf);
}

// Where a row finds the (x, y, z, h) of its neighbours.  idx(e) reads the
// handle of CSR entry e, get(handle) the position; `dummy` is a valid handle
// used for the loads issued past the end of a row.  kDeep: the position
// itself is also loaded one neighbour ahead (global gathers and LDS reads).
struct FetchGlobal {  // packed positions, gathered through col[]
  static constexpr bool kDeep = true;
  static constexpr bool kPairs = false;
  const double4 *pos;
  const int32_t *col;
  const double *u;     // field of the fused application
  int32_t dummy;
  __device__ int32_t idx(int64_t e) const { return col[e]; }
  __device__ double4 get(int32_t j) const { return pos[j]; }
  __device__ double field(int32_t j) const { return u[j]; }
};
// The tile's positions (and field) staged in LDS, addressed by slot[]: (x, y)
// and (z, h) in two arrays of 16-byte records, so that the two reads of a
// neighbour each start at one of 8 offsets in a 128-byte bank row (32-byte
// records start at one of 4, and the lanes of a read collide in the banks
// twice as often).
struct FetchTile {
  static constexpr bool kDeep = true;
  static constexpr bool kPairs = true;  // slots may be read in aligned pairs
  const double2 *sxy, *szh;
  const uint16_t *slot;
  const double *su;
  int32_t dummy;
  __device__ int32_t idx(int64_t e) const { return slot[e]; }
  __device__ double4 get(int32_t s) const {
    const double2 p = sxy[s], q = szh[s];
    return make_double4(p.x, p.y, q.x, q.y);
  }
  __device__ double field(int32_t s) const { return su[s]; }
};

// Pass 2 of the tiled rows of 8- or 16-lane teams: as FetchTile, with the
// row's slots copied into the team's LDS (entry e at sl[e - b2], b2 the even
// entry at or below the row's first), so that the loop issues no global loads
// (whose waits would also wait for the stencil stores in flight).
struct FetchTileL {
  static constexpr bool kDeep = true;
  static constexpr bool kPairs = false;
  const double2 *sxy, *szh;
  const uint16_t *sl;
  int64_t b2;
  const double *su;
  int32_t dummy;
  __device__ int32_t idx(int64_t e) const { return sl[e - b2]; }
  __device__ double4 get(int32_t s) const {
    const double2 p = sxy[s], q = szh[s];
    return make_double4(p.x, p.y, q.x, q.y);
  }
  __device__ double field(int32_t s) const { return su[s]; }
};

// Visit the neighbours k = k0, k0 + T, ... (k0 in (-T, T); negative k are
// skipped) of the row starting at CSR entry b, calling body(k, position,
// handle) with the loads software-pipelined (the handle two steps ahead is
// read on every step, past the row's end from its last entry: a valid handle,
// never used).
template <int T, class F, class Body>
__device__ inline void for_neighbours(const F &fetch, int64_t b, int n, int k0, Body &&body) {
  auto in = [n](int k) { return k >= 0 && k < n; };
  if constexpr (F::kDeep) {
    int32_t hc = in(k0) ? fetch.idx(b + k0) : fetch.dummy;
    int32_t hn = in(k0 + T) ? fetch.idx(b + k0 + T) : fetch.dummy;
    double4 pc = fetch.get(hc);
#pragma unroll 1
    for (int k = k0; k < n; k += T) {
      const double4 pj = pc;
      const int32_t h = hc;
      hc = hn;
      pc = fetch.get(hn);
      hn = fetch.idx(b + min(k + 2 * T, n - 1));
      if (k >= 0) body(k, pj, h);
    }
  } else {
    int32_t hc = in(k0) ? fetch.idx(b + k0) : fetch.dummy;
    int32_t hn = in(k0 + T) ? fetch.idx(b + k0 + T) : fetch.dummy;
#pragma unroll 1
    for (int k = k0; k < n; k += T) {
      const double4 pj = fetch.get(hc);
      const int32_t h = hc;
      hc = hn;
      hn = (k + 2 * T < n) ? fetch.idx(b + k + 2 * T) : fetch.dummy;
      if (k >= 0) body(k, pj, h);
    }
  }
}

// What a row reads before its neighbours: its extent, position, support,
// frame and field value, and (tiled rows) the slot groups of pass 1.  The tile
// kernel loads these before it stages the tile, so that their latency (three
// dependent reads: schedule, row extent, slots) overlaps the staging.
// Pass 1 of the tiled kernels reads its slots in aligned groups of G: pairs
// for teams of 8 or more lanes (a row of n entries takes ceil(n / 2T) steps of
// two slots instead of ceil(n / 4T) steps of four: fewer masked lanes at its
// end), quads for 4-lane teams (fewer registers, which hold that kernel at four
// waves per SIMD).
template <int T>
constexpr int slot_group() { return T >= 8 ? 2 : 4; }
template <int G>
using SlotVec = typename std::conditional<G == 2, ushort2, ushort4>::type;

template <int T, bool SLOTS>
struct RowPre {
  int32_t i;
  int64_t b;
  int n;
  RowGeom g;
  double ui;
  SlotVec<slot_group<T>()> ss[SLOTS ? kTileBandRow / (slot_group<T>() * T) + 1 : 1];
};

template <int M, int T, bool FUSED, bool SLOTS>
__device__ inline void row_pre(const WArgs &a, const uint16_t *slot, int32_t i, int lane, RowPre<T, SLOTS> &p) {
  p.i = i;
  p.b = a.row_ptr[i];
  p.n = (int)(a.row_ptr[i + 1] - p.b);
  row_geom<M>(a, i, p.g);
  p.ui = FUSED ? a.u[i] : 0.0;
  if constexpr (SLOTS) {
    // lane l takes the aligned groups of slots q0 + l, q0 + l + T, ...
    constexpr int G = slot_group<T>();
    constexpr int kQ1 = kTileBandRow / (G * T) + 1;
    const int64_t q0 = p.b / G + lane, e = p.b + p.n;
#pragma unroll
    for (int j = 0; j < kQ1; ++j) {
      const int64_t k = G * (q0 + j * T);
      if (k < e) p.ss[j] = *reinterpret_cast<const SlotVec<G> *>(slot + k);
    }
  }
}

// Moment-based team path.  Per particle, a team of T lanes of one wave:
//  pass 1  each lane accumulates the weighted moments sum w X^a Y^b Z^c
//          (a+b+c <= 4) of its neighbours' offsets (and caches its first KC
//          weights); the weights leave out their normalising factor, which
//          cancels from the stencils;
//  reduce  butterfly over the team; the moments are staged in LDS;
//  invert  the team assembles G from the moments (lane l owns rows
//          l, l+T, ...) and runs an in-place Gauss-Jordan inversion with the
//          pivot row broadcast through LDS (G is SPD: no pivoting); the
//          condition number is ||G_s||_1 ||G_s^-1||_1 of G_s, the Gram matrix
//          of the offsets scaled by 1/h_i; the target solutions lambda_s are
//          read off the rows of G^-1 and shared through LDS;
//  pass 2  each lane writes c_j = w_j phi_j . lambda_s for its neighbours.
// Neighbour loads are software-pipelined: the handle two neighbours ahead
// and the position one neighbour ahead are in flight during the arithmetic.
template <int M, int T, int OUT, bool FUSED, bool FASTW, int KC, bool UNI, class F, bool Q>
__device__ void weights_row_team(const WArgs &a, const RowPre<T, Q> &pre, int lane, double *sm, const F &fetch) {
  constexpr int NM = nmom<M>();
  constexpr int NL = NM > 4 * M ? NM : 4 * M;
  constexpr int R8 = red_lanes(T);
  constexpr int NA = cmax(NL, R8 * R8);
  double *s_red = sm;
  double *s_mom = sm;
  double *s_lam = sm;
  double *s_prow = sm;
  double *s_w = sm + (((cmax(NA, M + 1)) + 1) & ~1);
  const int32_t i = pre.i;
  const int64_t b = pre.b;
  const int n = pre.n;
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
  const RowGeom &g = pre.g;
  const double ih = g.inv_h, ih2 = ih * ih, cs_row = ih2 * a.wf.nl2a;
  // ---- pass 1: moments of the unscaled local coordinates
  double mom[NM];
#pragma unroll
  for (int p = 0; p < NM; ++p) mom[p] = 0.0;
  auto acc1 = [&](int k, const double4 &pj, int32_t) {
    const double dx = pj.x - g.xi, dy = pj.y - g.yi, dz = pj.z - g.zi;
    const double w = nbr_weight_raw<FASTW, UNI>(a, g, cs_row, pj.w, dx, dy, dz);
    if constexpr (KC > 0)
      if (k < KC * T) s_w[k] = w;
    double X, Y, Z;
    local_raw<M>(g, dx, dy, dz, X, Y, Z);
    moments_add_raw<M>(mom, w, X, Y, Z);
  };
  if constexpr (F::kPairs && KC == 0) {
    // tiled rows (at most kTileBandRow entries): lane l takes the aligned groups
    // of G slots q0 + l, q0 + l + T, ..., all loaded before the first is used
    // (with the row, by row_pre, where the team is at least 8 wide); a group may
    // reach up to G - 1 entries into the neighbouring rows (the slot array is
    // padded): those are skipped
    constexpr int G = slot_group<T>();
    constexpr int kQ1 = kTileBandRow / (G * T) + 1;
    const int64_t q0 = b / G + lane, e = b + n;
    SlotVec<G> ssl[Q ? 1 : kQ1];
    if constexpr (!Q) {
#pragma unroll
      for (int j = 0; j < kQ1; ++j) {
        const int64_t k = G * (q0 + j * T);
        if (k < e) ssl[j] = *reinterpret_cast<const SlotVec<G> *>(fetch.slot + k);
      }
    }
    const SlotVec<G> *ss = Q ? pre.ss : ssl;
#pragma unroll
    for (int j = 0; j < kQ1; ++j) {
      const int64_t k = G * (q0 + j * T);
      if (k < e) {
        // (k < e holds; k + G - 1 >= b, as groups are aligned)
        if constexpr (G == 4) {
          if (k >= b) acc1(0, fetch.get(ss[j].x), 0);
          if (k + 1 >= b && k + 1 < e) acc1(0, fetch.get(ss[j].y), 0);
          if (k + 2 >= b && k + 2 < e) acc1(0, fetch.get(ss[j].z), 0);
          if (k + 3 < e) acc1(0, fetch.get(ss[j].w), 0);
        } else {
          if (k >= b) acc1(0, fetch.get(ss[j].x), 0);
          if (k + 1 < e) acc1(0, fetch.get(ss[j].y), 0);
        }
      }
    }
  } else {
    for_neighbours<T>(fetch, b, n, lane, acc1);
  }
  // ---- team sum of the moments (left in s_mom)
  team_moment_sum<M, T>(mom, lane, s_red);
  // ---- Gauss-Jordan inversion of G; lane owns rows lane + q T (q < NR).
  // G is the Gram matrix of the unscaled monomials.  With D = diag(h_i^-deg a),
  // the matrix of the scaled coordinates d / h_i is D G D: its inverse gives the
  // same stencils (the powers of h_i cancel against the physical scaling of
  // the targets: column 1 of G^-1 is the x-derivative stencil's coefficient
  // vector as it stands), elimination without pivoting on an SPD matrix is
  // unaffected by the diagonal scaling, and only the condition number is taken
  // of D G D, whose row sums are d_r sum_c |G_rc| d_c (those of its inverse
  // sum_c |G^-1_rc| / (d_r d_c)).
  constexpr int NR = (M + T - 1) / T;
  constexpr int NLIN = M == 10 ? 3 : 2;  // monomials 1..NLIN are linear, the rest quadratic
  auto deg_rt = [](int r) { return (r == 0) ? 0 : (r <= NLIN ? 1 : 2); };
  double row[NR][M];
  double gsum = 0.0;
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int r = lane + q * T;
    const bool own = r < M;
    double sacc = 0.0;
#pragma unroll
    for (int c = 0; c < M; ++c) {
      const int mi = own ? (M == 10 ? kGram3.v[r][c] : kGram2.v[r][c]) : 0;
      row[q][c] = own ? s_mom[mi] : 0.0;
      const double dc = mono_deg<M>(c) == 0 ? 1.0 : (mono_deg<M>(c) == 1 ? ih : ih2);
      sacc = fma(fabs(row[q][c]), dc, sacc);
    }
    const int dg = deg_rt(r);
    gsum = fmax(gsum, sacc * (dg == 0 ? 1.0 : (dg == 1 ? ih : ih2)));
  }
  wave_sync();  // the pivot rows overwrite the moments
  const bool okp = team_gauss_jordan<M, T>(row, lane, s_prow);
  double isum = 0.0;
  {
    const double h = g.hi, h2 = h * h;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      double sacc = 0.0;
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const double hc = mono_deg<M>(c) == 0 ? 1.0 : (mono_deg<M>(c) == 1 ? h : h2);
        sacc = fma(fabs(row[q][c]), hc, sacc);
      }
      const int dg = deg_rt(lane + q * T);
      isum = fmax(isum, (lane + q * T < M) ? sacc * (dg == 0 ? 1.0 : (dg == 1 ? h : h2)) : 0.0);
    }
  }
  const double gnorm = team_max(gsum, T);
  const double inorm = team_max(isum, T);
  // a pivot that is not positive: G is not positive definite (rank deficient
  // or numerically so), reported as an infinite condition number
  const double kappa = okp ? gnorm * inorm : INFINITY;
  // lambda_s[r] from row r of G^{-1} (= column r): the coefficients of the
  // unscaled monomials in the stencils of the physical derivatives; on a film
  // s = 0, 1 are the two tangential derivatives (s = 2 unused), which pass 2
  // turns into the x, y, z components
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const int r = lane + q * T;
    if (r < M) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (M == 6 && s == 2) continue;
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
  wave_sync();
  if (lane == 0 && a.kappa_out) a.kappa_out[i] = (float)kappa;
  if (!okp || !(kappa <= a.kappa_max)) {
    if (lane == 0) {
      if (a.status) a.status[i] = 1;
      const int32_t q = atomicAdd(a.qcount, 1);
      a.queue[q] = i;
    }
    return;
  }
  // ---- pass 2: stencils (and their application)
  double lam[4 * M];
#pragma unroll
  for (int q = 0; q < 4 * M; ++q) lam[q] = s_lam[q];
  constexpr bool kSlotsLds = F::kPairs && Q && KC == 0;
  if constexpr (kSlotsLds) {
    // the target solutions are in registers: the team's area takes the row's
    // slot pairs (lane l's pair j is word l + j T)
    wave_sync();
    constexpr int kQ1 = kTileBandRow / (2 * T) + 1;
    const int64_t q0 = (b >> 1) + lane, e = b + n;
    uint32_t *s_sl = reinterpret_cast<uint32_t *>(sm);
#pragma unroll
    for (int j = 0; j < kQ1; ++j)
      if (2 * (q0 + j * T) < e) s_sl[lane + j * T] = __builtin_bit_cast(uint32_t, pre.ss[j]);
    wave_sync();
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const double ui = pre.ui;
  // the team's stores of one step cover whole aligned T-entry blocks
  const int k0 = a.w_out ? lane - (int)(b & (T - 1)) : lane;
  // Stores are issued one step late, at the start of the next step: a load
  // and a store in flight count against one counter, and the wait for the
  // next handle (right after the step) would otherwise wait for the store it
  // just issued.  (Two copies of the loop, with and without stores.)
  f32x4 vprev = {0.0f, 0.0f, 0.0f, 0.0f};
  int kprev = -1;
  auto body2 = [&](int k, const double4 &pj, int32_t h, auto store) {
    if constexpr (OUT == GF_F32 && decltype(store)::value)
      if (kprev >= 0) __builtin_nontemporal_store(vprev, reinterpret_cast<f32x4 *>(a.w_out) + (b + kprev));
    const double dx = pj.x - g.xi, dy = pj.y - g.yi, dz = pj.z - g.zi;
    double w;
    if constexpr (KC > 0)
      w = (k < KC * T) ? s_w[k] : nbr_weight_raw<FASTW, UNI>(a, g, cs_row, pj.w, dx, dy, dz);
    else
      w = nbr_weight_raw<FASTW, UNI>(a, g, cs_row, pj.w, dx, dy, dz);
    double X, Y, Z;
    local_raw<M>(g, dx, dy, dz, X, Y, Z);
    double c[4];
    if constexpr (M == 10) {
#pragma unroll
      for (int s = 0; s < 4; ++s) c[s] = w * poly_eval<M>(lam + s * M, X, Y, Z);
    } else {
      const double wu = w * poly_eval<M>(lam, X, Y, Z), wv = w * poly_eval<M>(lam + M, X, Y, Z);
#pragma unroll
      for (int s = 0; s < 3; ++s) c[s] = fma(g.t2[s], wv, g.t1[s] * wu);
      c[3] = w * poly_eval<M>(lam + 3 * M, X, Y, Z);
    }
    if constexpr (OUT == GF_F32) {
      // rounded once: the stored stencils are also the ones applied
      const f32x4 v = {(float)c[0], (float)c[1], (float)c[2], (float)c[3]};
      if constexpr (decltype(store)::value) {
        vprev = v;
        kprev = k;
      }
#pragma unroll
      for (int s = 0; s < 4; ++s) c[s] = (double)v[s];
    } else {
      if constexpr (decltype(store)::value) store_w<OUT, true>(a.w_out, b + k, c[0], c[1], c[2], c[3]);
    }
    if constexpr (FUSED) {
      // the diagonal entry contributes u_i - u_i = 0
      const double du = fetch.field(h) - ui;
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[s] = fma(c[s], du, acc[s]);
    }
  };
  auto pass2 = [&](const auto &f2) {
    if (a.w_out) {
      for_neighbours<T>(f2, b, n, k0, [&](int k, const double4 &pj, int32_t h) {
        body2(k, pj, h, std::true_type{});
      });
      if constexpr (OUT == GF_F32)
        if (kprev >= 0) __builtin_nontemporal_store(vprev, reinterpret_cast<f32x4 *>(a.w_out) + (b + kprev));
    } else {
      for_neighbours<T>(f2, b, n, k0, [&](int k, const double4 &pj, int32_t h) {
        body2(k, pj, h, std::false_type{});
      });
    }
  };
  if constexpr (kSlotsLds)
    pass2(FetchTileL{fetch.sxy, fetch.szh, reinterpret_cast<const uint16_t *>(sm), b & ~int64_t(1), fetch.su, 0});
  else
    pass2(fetch);
  if constexpr (FUSED) {
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[s] = team_sum(acc[s], T);
    if (lane == 0) store_fused(a, i, acc);
  }
  if (lane == 0 && a.status) a.status[i] = 0;
}

// Untiled batched kernel (rows with more than kTileBandRow neighbours):
// positions gathered from the packed array, weights of the first
// kCacheW x T neighbours cached in LDS between the passes.
constexpr int kCacheW = 8;

template <int M, int T, int OUT, bool FUSED, bool FASTW>
__global__ void __launch_bounds__(kBlock) k_weights_team(WArgs a) {
  __shared__ double smem[(kBlock / T) * team_lds_doubles<M>(T, kCacheW)];
  const int64_t gt = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t team = gt / T;
  const int lane = (int)(gt % T);
  if (team >= a.nrows) return;
  double *sm = smem + (threadIdx.x / T) * team_lds_doubles<M>(T, kCacheW);
  RowPre<T, false> pre;
  row_pre<M, T, FUSED, false>(a, nullptr, a.sched[team], lane, pre);
  weights_row_team<M, T, OUT, FUSED, FASTW, kCacheW, false>(a, pre, lane, sm, FetchGlobal{a.pos, a.col, a.u, pre.i});
}

// Tiled batched kernel: one block per neighbour tile (kTileRows rows, one
// team each).  The block stages the tile's distinct neighbour positions in
// LDS (at most cap of them; a larger tile reads them from global memory)
// and both passes address them through slot[].
struct TileArgs {
  const int64_t *off;  // tile list offsets (global tile ids)
  const int32_t *u;    // tile lists
  int64_t tile0;       // first tile of the group
  int cap;             // LDS capacity in positions
};

// LDS positions a tile block may stage (larger tiles read global memory)
constexpr int kTileCap = 1024;

// LDS of a tile block, in order: (x, y) records, (z, h) records, field values
// (fused), the team areas, one flag per wave.  The 3D kernels of 8 or more
// lanes (at most 3 blocks per CU, bound by registers) lay the arrays out for
// kTileCap positions whatever the tile holds: every offset is then a
// compile-time constant, and a neighbour's three reads share one address
// register.  The other kernels size them by the launch's largest tile, which
// keeps their LDS small enough for more blocks per CU.
template <int M, int T>
constexpr int tile_stride() { return (M == 10 && T >= 8) ? kTileCap : 0; }

template <int M, bool FUSED>
size_t tile_lds_bytes(int T, int cap) {
  const int st = (M == 10 && T >= 8) ? kTileCap : cap;  // = tile_stride<M, T>() or cap
  return sizeof(double4) * st + (FUSED ? sizeof(double) * ((st + 1) & ~1) : 0) +
         sizeof(double) * kTileRows * team_lds_doubles<M>(T, 0) + sizeof(int) * (kTileRows * T / 64);
}

template <int M, int T, int OUT, bool FUSED, bool FASTW>
__global__ void __launch_bounds__(kTileRows * T) __attribute__((amdgpu_waves_per_eu(T >= 8 ? 3 : 1)))
k_weights_tile(WArgs a, TileArgs ta, const uint16_t *__restrict__ slot) {
  extern __shared__ double4 s_dyn[];  // the kernel's only LDS: it starts at address 0
  constexpr int ZS = tile_stride<M, T>();
  const int st = ZS ? ZS : ta.cap;
  const int64_t tl = xcd_block(blockIdx.x, gridDim.x);
  const int64_t u0 = ta.off[ta.tile0 + tl];
  const int cnt = (int)(ta.off[ta.tile0 + tl + 1] - u0);
  const bool staged = cnt <= ta.cap;
  double2 *s_xy = reinterpret_cast<double2 *>(s_dyn), *s_zh = s_xy + st;   // positions
  double *s_u = reinterpret_cast<double *>(s_dyn + st);                    // fused field values
  double *s_team = s_u + (FUSED ? ((st + 1) & ~1) : 0);
  int *s_flag = reinterpret_cast<int *>(s_team + kTileRows * team_lds_doubles<M>(T, 0));
  const int team = threadIdx.x / T, lane = threadIdx.x % T;
  const int64_t r = tl * kTileRows + team;
  const bool live = r < a.nrows;
  // (4-lane teams would hold more slot groups per lane than their registers
  // allow: they load them in pass 1)
  RowPre<T, (T >= 8)> pre;
  if (live) row_pre<M, T, FUSED, (T >= 8)>(a, slot, a.sched[r], lane, pre);
  // uni: every staged support equals the first (then also each row's own, as
  // a row is its own neighbour), so no row needs the per-neighbour test
  int same = 1;
  if (staged) {
    const double h0 = a.h[ta.u[u0]];
    for (int s = threadIdx.x; s < cnt; s += blockDim.x) {
      const int32_t j = ta.u[u0 + s];
      const double hj = a.h[j];
      s_xy[s] = make_double2(a.x[j], a.y[j]);
      s_zh[s] = make_double2(a.z[j], hj);
      same &= hj == h0;
      if constexpr (FUSED) s_u[s] = a.u[j];
    }
  }
  // block-wide AND of `same`: a ballot per wave, one flag per wave, one barrier
  // (which also publishes the staged tile)
  constexpr int NW = kTileRows * T / 64;
  const bool wave_same = __ballot(!same) == 0;
  if ((threadIdx.x & 63) == 0) s_flag[threadIdx.x >> 6] = wave_same;
  __syncthreads();
  bool uni = true;
#pragma unroll
  for (int w = 0; w < NW; ++w) uni = uni && s_flag[w] != 0;
  if (!live) return;
  double *sm = s_team + team * team_lds_doubles<M>(T, 0);
  if (staged)
    if (uni)
      weights_row_team<M, T, OUT, FUSED, FASTW, 0, true>(a, pre, lane, sm, FetchTile{s_xy, s_zh, slot, s_u, 0});
    else
      weights_row_team<M, T, OUT, FUSED, FASTW, 0, false>(a, pre, lane, sm, FetchTile{s_xy, s_zh, slot, s_u, 0});
  else
    weights_row_team<M, T, OUT, FUSED, FASTW, 0, false>(a, pre, lane, sm, FetchGlobal{a.pos, a.col, a.u, pre.i});
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
// Columns (column-major, n rows) live in LDS where the longest row fits
// (LDSP: the reflections' dependent reads and updates stay on chip), else in
// a per-block slice of global scratch.
template <int OUT, bool FUSED, bool FASTW, bool LDSP>
__global__ void __launch_bounds__(kQrBlock) k_weights_qr(WArgs a, double *panels, int64_t slice) {
  extern __shared__ double s_panel[];
  const int lane = threadIdx.x;
  double *A = LDSP ? s_panel : panels + (int64_t)blockIdx.x * slice;
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

// profiling names: one per launch unit
const char *unit_kernel_name(const LaunchUnit &u, bool fused) {
  static const char *names[2][2][2] = {{{"weights_3d_tiles", "weights_3d_b3"}, {"weights_film_tiles", "weights_film_b3"}},
                                       {{"weights_apply_3d_tiles", "weights_apply_3d_b3"},
                                        {"weights_apply_film_tiles", "weights_apply_film_b3"}}};
  return names[fused ? 1 : 0][u.model][u.tiled ? 0 : 1];
}

template <int M, int OUT, bool FUSED, bool FASTW>
gf_status launch_team(gf_ctx *ctx, hipStream_t st, const WArgs &a, int T, const char *name) {
  ProfScope prof(ctx, name, st);
  const int64_t threads = a.nrows * (int64_t)T;
  const dim3 grid(grid_for(threads, kBlock)), block(kBlock);
  switch (T) {
    case 4: hipLaunchKernelGGL((k_weights_team<M, 4, OUT, FUSED, FASTW>), grid, block, 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_weights_team<M, 8, OUT, FUSED, FASTW>), grid, block, 0, st, a); break;
    case 16: hipLaunchKernelGGL((k_weights_team<M, 16, OUT, FUSED, FASTW>), grid, block, 0, st, a); break;
    default: return set_error(ctx, GF_EINVAL, "unsupported team size %d", T);
  }
  GF_LAUNCH_CHECK(ctx);
  return GF_OK;
}

template <int M, int OUT, bool FUSED, bool FASTW>
gf_status launch_tile(gf_ctx *ctx, hipStream_t st, const WArgs &a, const gf_nbr *nbr, const LaunchUnit &u, int T,
                      const char *name) {
  ProfScope prof(ctx, name, st);
  TileArgs ta;
  ta.off = nbr->tile_off;
  ta.u = nbr->tile_u;
  ta.tile0 = u.tile0;
  ta.cap = std::min(u.tile_max, tile_capacity(ctx, kTileCap));
  const size_t lds = tile_lds_bytes<M, FUSED>(T, ta.cap);
  const dim3 grid(grid_for(u.ntiles, 1)), block(kTileRows * T);
  switch (T) {
    case 4: hipLaunchKernelGGL((k_weights_tile<M, 4, OUT, FUSED, FASTW>), grid, block, lds, st, a, ta, nbr->slot); break;
    case 8: hipLaunchKernelGGL((k_weights_tile<M, 8, OUT, FUSED, FASTW>), grid, block, lds, st, a, ta, nbr->slot); break;
    case 16: hipLaunchKernelGGL((k_weights_tile<M, 16, OUT, FUSED, FASTW>), grid, block, lds, st, a, ta, nbr->slot); break;
    default: return set_error(ctx, GF_EINVAL, "unsupported team size %d", T);
  }
  GF_LAUNCH_CHECK(ctx);
  return GF_OK;
}

// One launch per launch unit; only_unit >= 0 restricts the launches to that
// unit and team_override > 0 replaces its team size (used by the autotuner).
template <int OUT, bool FUSED, bool FASTW>
gf_status launch_batched(gf_ctx *ctx, const gf_nbr *nbr, WArgs a, int only_unit = -1, int team_override = 0) {
  LaunchUnit units[2 * GF_NBAND];
  const int nu = launch_units(nbr, units);
  for (int q = 0; q < nu; ++q) {
    if (only_unit >= 0 && q != only_unit) continue;
    const LaunchUnit &u = units[q];
    a.sched = nbr->grouped + u.row0;
    a.nrows = u.nrows;
    const int T = team_override > 0 ? team_override : (FUSED ? ctx->fteam : ctx->wteam)[u.model][u.band];
    const char *name = unit_kernel_name(u, FUSED);
    gf_status st;
    if (u.tiled)
      st = (u.model == 0) ? launch_tile<10, OUT, FUSED, FASTW>(ctx, ctx->stream, a, nbr, u, T, name)
                          : launch_tile<6, OUT, FUSED, FASTW>(ctx, ctx->stream, a, nbr, u, T, name);
    else
      st = (u.model == 0) ? launch_team<10, OUT, FUSED, FASTW>(ctx, ctx->stream, a, T, name)
                          : launch_team<6, OUT, FUSED, FASTW>(ctx, ctx->stream, a, T, name);
    if (st) return st;
  }
  return GF_OK;
}

// whether any batched launch reads the packed positions (untiled units and
// tiles whose list exceeds the LDS capacity gather them from global memory)
bool needs_packed_positions(const gf_ctx *ctx, const gf_nbr *nbr) {
  LaunchUnit units[2 * GF_NBAND];
  const int nu = launch_units(nbr, units);
  for (int q = 0; q < nu; ++q)
    if (!units[q].tiled || units[q].tile_max > tile_capacity(ctx, kTileCap)) return true;
  return false;
}

// The fixed workspace of gf_gfdm_weights_apply_noalloc: a device array of
// the library (one copy per device, held until the process ends).  Host code
// never uses its name as an address: gf_create looks up its device address
// once per device (fixed_scratch_init) and kernels receive that address.
constexpr size_t kFixedScratchBytes = size_t(128) << 20;
constexpr int kFixedQrBlocks = 256;  // blocks of the QR fallback in that mode (the grid strides over the queue)

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

// fixed: carve the scratch from the library's fixed workspace (no
// allocation; GF_ECAPACITY if it does not fit) instead of the context arena.
gf_status weights_common(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr, gf_prec prec,
                         const gf_ls_params *params, gf_dtype wtype, void *w_out, int8_t *status_n, float *kappa_n,
                         gf_ls_stats *stats, bool fused, unsigned op_mask, const double *u, double *out,
                         bool fixed = false) {
  gf_status st = check_particles(ctx, p, false, false);
  if (st) return st;
  if ((st = check_nbr(ctx, nbr, p->n))) return st;
  if (nbr->cross) return set_error(ctx, GF_EINVAL, "stencils need same-model neighbourhoods");
  if (prec != GF_PLAIN_F64 && prec != GF_BATCHED) return set_error(ctx, GF_EINVAL, "unknown precision mode %d", (int)prec);
  if (wtype != GF_F64 && wtype != GF_F32) return set_error(ctx, GF_EINVAL, "unknown weight type %d", (int)wtype);
  if (prec == GF_PLAIN_F64 && wtype != GF_F64) return set_error(ctx, GF_EINVAL, "GF_PLAIN_F64 writes FP64 weights");
  if (!w_out && !fused) return set_error(ctx, GF_EINVAL, "w_out is NULL");
  if (reinterpret_cast<uintptr_t>(w_out) & 15) return set_error(ctx, GF_EINVAL, "w_out must be 16-byte aligned");
  if (fused && (!u || !out || (op_mask & 0xF) == 0 || (op_mask & ~0xFu)))
    return set_error(ctx, GF_EINVAL, "fused application needs u, out and a non-empty op mask");
  gf_ls_params prm;
  gf_ls_params_default(&prm);
  if (params) prm = *params;
  if (!(prm.alpha_w > 0.0) || !(prm.kappa_max > 0.0)) return set_error(ctx, GF_EINVAL, "alpha_w and kappa_max must be positive");
  bool has_film = nbr->group_start[2 * GF_NBAND] > nbr->group_start[GF_NBAND];
  if (has_film && (!p->nx || !p->ny || !p->nz)) return set_error(ctx, GF_EINVAL, "film particles need normals");
  const int64_t n = p->n;
  const int qr_blocks = (int)std::min<int64_t>(fixed ? kFixedQrBlocks : 1024, n);
  const int64_t slice = (int64_t)kQrStride * std::max(nbr->max_row, 1);
  const bool packed = prec == GF_BATCHED && needs_packed_positions(ctx, nbr);
  Arena ar;
  WeightsScratch ws;
  double4 *pos = nullptr;
  if (fixed) {
    // only what the fused call uses: queue, counter, QR panels, packed positions
    const size_t need = arena_bytes({sizeof(int32_t) * n, 64, sizeof(double) * slice * qr_blocks,
                                     packed ? sizeof(double4) * n : 0});
    if (need > kFixedScratchBytes)
      return set_error(ctx, GF_ECAPACITY, "the workspace of this call needs %zu bytes, the fixed workspace holds %zu "
                       "(%lld particles, longest row %d)", need, kFixedScratchBytes, (long long)n, (int)nbr->max_row);
    if (!ctx->fixed_scratch) return set_error(ctx, GF_EHIP, "fixed workspace address unknown");
    ar.base = (char *)ctx->fixed_scratch;
    ar.off = 0;
    ws.queue = ar.take<int32_t>(n);
    ws.qcount = ar.take<int32_t>(16);
    ws.qr = ar.take<double>(slice * qr_blocks);
    if (packed) pos = ar.take<double4>(n);
    ws.status = nullptr; ws.kappa = nullptr; ws.counts = nullptr; ws.kmax = nullptr;
  } else {
    if ((st = ensure_scratch(ctx, arena_bytes({sizeof(int32_t) * n, 64, sizeof(double) * slice * qr_blocks, (size_t)n,
                                               sizeof(float) * n, 64, 64, sizeof(double4) * n}),
                             &ar)))
      return st;
    ws.queue = ar.take<int32_t>(n);
    ws.qcount = ar.take<int32_t>(16);
    ws.qr = ar.take<double>(slice * qr_blocks);
    ws.status = ar.take<int8_t>(n);
    ws.kappa = ar.take<float>(n);
    ws.counts = ar.take<long long>(4);
    ws.kmax = ar.take<double>(1);
    pos = ar.take<double4>(n);
  }
  WArgs a;
  a.x = p->x; a.y = p->y; a.z = p->z; a.h = p->h; a.nx = p->nx; a.ny = p->ny; a.nz = p->nz; a.model = p->model;
  a.pos = pos;
  if (packed) {
    ProfScope prof(ctx, "pack_positions");
    hipLaunchKernelGGL(k_pack_pos, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, p->x, p->y, p->z, p->h, n, pos);
    GF_LAUNCH_CHECK(ctx);
  }
  a.row_ptr = nbr->row_ptr; a.col = nbr->col; a.sched = nullptr; a.nrows = n; a.n = n;
  a.wf = make_weight_fn(prm.alpha_w);
  a.kappa_max = prm.kappa_max;
  a.w_out = w_out;
  a.status = status_n ? status_n : ((stats && !fixed) ? ws.status : nullptr);
  a.kappa_out = kappa_n ? kappa_n : ((stats && !fixed) ? ws.kappa : nullptr);
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
  {
    const size_t lds = sizeof(double) * (size_t)slice;
    const bool ldsp = lds <= kQrLdsMax;
    const dim3 qg(qr_blocks), qb(kQrBlock);
    const size_t ql = ldsp ? lds : 0;
    if (!fused) {
      if (f32) {
        if (ldsp) hipLaunchKernelGGL((k_weights_qr<GF_F32, false, true, true>), qg, qb, ql, ctx->stream, a, ws.qr, slice);
        else hipLaunchKernelGGL((k_weights_qr<GF_F32, false, true, false>), qg, qb, ql, ctx->stream, a, ws.qr, slice);
      } else {
        if (ldsp) hipLaunchKernelGGL((k_weights_qr<GF_F64, false, false, true>), qg, qb, ql, ctx->stream, a, ws.qr, slice);
        else hipLaunchKernelGGL((k_weights_qr<GF_F64, false, false, false>), qg, qb, ql, ctx->stream, a, ws.qr, slice);
      }
    } else {
      if (f32) {
        if (ldsp) hipLaunchKernelGGL((k_weights_qr<GF_F32, true, true, true>), qg, qb, ql, ctx->stream, a, ws.qr, slice);
        else hipLaunchKernelGGL((k_weights_qr<GF_F32, true, true, false>), qg, qb, ql, ctx->stream, a, ws.qr, slice);
      } else {
        if (ldsp) hipLaunchKernelGGL((k_weights_qr<GF_F64, true, false, true>), qg, qb, ql, ctx->stream, a, ws.qr, slice);
        else hipLaunchKernelGGL((k_weights_qr<GF_F64, true, false, false>), qg, qb, ql, ctx->stream, a, ws.qr, slice);
      }
    }
  }
  GF_LAUNCH_CHECK(ctx);
  if (stats && !fixed) {
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

// ------------------------------------------------------------------ fixed workspace
static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_fixed_mutex;
void *g_fixed_ptr[kMaxDevices] = {nullptr};
}  // namespace

gf_status fixed_scratch_init(gf_ctx *ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return set_error(ctx, GF_ECAPACITY, "device index %d beyond %d", ctx->device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_fixed_mutex);
  if (!g_fixed_ptr[ctx->device]) {
    GF_HIP(ctx, hipSetDevice(ctx->device));
    void *ptr = nullptr;
    GF_HIP(ctx, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return set_error(ctx, GF_EHIP, "hipGetSymbolAddress returned no address for the fixed workspace");
    g_fixed_ptr[ctx->device] = ptr;
  }
  ctx->fixed_scratch = g_fixed_ptr[ctx->device];
  return GF_OK;
}

extern "C" gf_status gf_gfdm_weights_apply_noalloc(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr,
                                                   const gf_ls_params *params, gf_dtype wtype, void *w_out,
                                                   unsigned op_mask, const double *u, double *out,
                                                   int8_t *status_n) {
  if (!ctx) return GF_EINVAL;
  return weights_common(ctx, p, nbr, GF_BATCHED, params, wtype, w_out, status_n, nullptr, nullptr, true, op_mask, u,
                        out, true);
}

extern "C" size_t gf_noalloc_workspace_bytes(void) { return kFixedScratchBytes; }

// ------------------------------------------------------------------ autotuner
// Times every launch unit of the batched stencil kernel with teams of 4, 8
// and 16 lanes (median of three launches after a warm-up) and keeps the
// fastest; then the fused stencil + application kernel (more registers, so
// its best team size may differ), then the application kernel.
extern "C" gf_status gf_autotune(gf_ctx *ctx, const gf_particles *p, const gf_nbr *nbr, gf_dtype wtype,
                                 int *team_out) {
  if (!ctx) return GF_EINVAL;
  gf_status st = check_particles(ctx, p, false, false);
  if (st) return st;
  if ((st = check_nbr(ctx, nbr, p->n))) return st;
  if (nbr->cross) return set_error(ctx, GF_EINVAL, "stencils need same-model neighbourhoods");
  if (wtype != GF_F64 && wtype != GF_F32) return set_error(ctx, GF_EINVAL, "unknown weight type %d", (int)wtype);
  const bool has_film = nbr->group_start[2 * GF_NBAND] > nbr->group_start[GF_NBAND];
  if (has_film && (!p->nx || !p->ny || !p->nz)) return set_error(ctx, GF_EINVAL, "film particles need normals");
  const int64_t n = p->n;
  const size_t wbytes = (size_t)std::max<int64_t>(nbr->nnz, 1) * 4 * (wtype == GF_F32 ? sizeof(float) : sizeof(double));
  void *wbuf = nullptr;
  if (hipMalloc(&wbuf, wbytes) != hipSuccess) return set_error(ctx, GF_ENOMEM, "autotune buffer allocation failed");
  Arena ar;
  if ((st = ensure_scratch(ctx, arena_bytes({sizeof(int32_t) * n, 64, sizeof(double4) * n, sizeof(double) * n,
                                             sizeof(double) * 4 * n}), &ar))) {
    (void)hipFree(wbuf);
    return st;
  }
  WArgs a;
  a.x = p->x; a.y = p->y; a.z = p->z; a.h = p->h; a.nx = p->nx; a.ny = p->ny; a.nz = p->nz; a.model = p->model;
  a.row_ptr = nbr->row_ptr; a.col = nbr->col; a.sched = nullptr; a.nrows = n; a.n = n;
  gf_ls_params prm;
  gf_ls_params_default(&prm);
  a.wf = make_weight_fn(prm.alpha_w);
  a.kappa_max = prm.kappa_max;
  a.w_out = wbuf; a.status = nullptr; a.kappa_out = nullptr;
  a.queue = ar.take<int32_t>(n);
  a.qcount = ar.take<int32_t>(16);
  a.u = nullptr; a.y_out = nullptr; a.mask = 0;
  double4 *pos = ar.take<double4>(n);
  a.pos = pos;
  hipLaunchKernelGGL(k_pack_pos, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, ctx->stream, p->x, p->y, p->z, p->h, n, pos);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipFree(wbuf);
    return set_error(ctx, GF_EHIP, "event creation failed");
  }
  double *tu_field = ar.take<double>(n);
  double *tu_out = ar.take<double>(4 * n);
  (void)hipMemsetAsync(tu_field, 0, sizeof(double) * n, ctx->stream);
  const int sizes[3] = {4, 8, 16};
  const int saved_profile = ctx->profile;
  ctx->profile = 0;
  LaunchUnit units[2 * GF_NBAND];
  const int nu = launch_units(nbr, units);
  const bool f32 = wtype == GF_F32;
  // the team size of each unit: 8 lanes unless 4 or 16 is faster by more than
  // 3%.  The trials run back to back, where caches are warm; 3D rows do not
  // try 4 lanes (the kernel then holds one wave per SIMD and cannot hide the
  // memory latency of a cold cache, however it fares warm), and close calls
  // go to 8.
  auto tune = [&](int (*team)[4], bool fused) {
    for (int q = 0; q < nu && !st; ++q) {
      float med[3] = {INFINITY, INFINITY, INFINITY};
      for (int t = 0; t < 3 && !st; ++t) {
        if (units[q].model == 0 && sizes[t] == 4) continue;
        float times[3];
        for (int rep = -1; rep < 3 && !st; ++rep) {
          hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, ctx->stream, a.qcount, 16);
          if (rep >= 0) (void)hipEventRecord(e0, ctx->stream);
          if (fused)
            st = f32 ? launch_batched<GF_F32, true, true>(ctx, nbr, a, q, sizes[t])
                     : launch_batched<GF_F64, true, false>(ctx, nbr, a, q, sizes[t]);
          else
            st = f32 ? launch_batched<GF_F32, false, true>(ctx, nbr, a, q, sizes[t])
                     : launch_batched<GF_F64, false, false>(ctx, nbr, a, q, sizes[t]);
          if (rep >= 0) {
            (void)hipEventRecord(e1, ctx->stream);
            (void)hipEventSynchronize(e1);
            (void)hipEventElapsedTime(&times[rep], e0, e1);
          }
        }
        if (st) break;
        std::sort(times, times + 3);
        med[t] = times[1];
      }
      int bestT = 8;
      float best = med[1];
      for (int t = 0; t < 3; ++t)
        if (t != 1 && med[t] < 0.97f * med[1] && med[t] < best) { best = med[t]; bestT = sizes[t]; }
      if (!st) team[units[q].model][units[q].band] = bestT;
    }
  };
  tune(ctx->wteam, false);
  a.u = tu_field; a.y_out = tu_out; a.mask = 0xF;
  tune(ctx->fteam, true);
  a.u = nullptr; a.y_out = nullptr; a.mask = 0;
  // complete the stencils with the tuned configuration, then tune the application
  if (!st) {
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, ctx->stream, a.qcount, 16);
    st = (wtype == GF_F32) ? launch_batched<GF_F32, false, true>(ctx, nbr, a) : launch_batched<GF_F64, false, false>(ctx, nbr, a);
  }
  if (!st) st = tune_apply(ctx, nbr, wbuf, wtype);
  ctx->profile = saved_profile;
  (void)hipStreamSynchronize(ctx->stream);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(wbuf);
  if (st) return st;
  if (team_out) {
    for (int g = 0; g < 2 * GF_NBAND; ++g) {
      team_out[g] = ctx->wteam[g / GF_NBAND][g % GF_NBAND];
      team_out[2 * GF_NBAND + g] = ctx->ateam[g / GF_NBAND][g % GF_NBAND];
      team_out[4 * GF_NBAND + g] = ctx->fteam[g / GF_NBAND][g % GF_NBAND];
    }
  }
  return GF_OK;
}
