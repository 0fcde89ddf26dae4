// Device helpers shared by the stencil kernels (weights, fused application,
// position adjoint): local monomial bases, the support weight, packed
// symmetric Gram matrices and their LDL^T factorisation.
#pragma once

#include "internal.h"

namespace gfdm_dev {

// number of monomials of the second-order basis: 10 in 3D, 6 on a film
__host__ __device__ constexpr int npack(int M) { return M * (M + 1) / 2; }
// packed upper-triangular index of (a, c), a <= c
__host__ __device__ constexpr int pidx(int a, int c, int M) { return a * M - (a * (a - 1)) / 2 + (c - a); }

struct RowGeom {
  double xi, yi, zi, hi, inv_h;
  double t1[3], t2[3];  // film tangent frame
};

// Tangent frame of a film particle from its unit normal: t1 is the axis least
// aligned with n projected onto the tangent plane, t2 = n x t1.
__device__ inline void tangent_frame(double nx, double ny, double nz, double t1[3], double t2[3]) {
  const double an[3] = {fabs(nx), fabs(ny), fabs(nz)};
  int a = 0;
  if (an[1] < an[a]) a = 1;
  if (an[2] < an[a]) a = 2;
  const double n[3] = {nx, ny, nz};
  double e[3] = {0.0, 0.0, 0.0};
  e[a] = 1.0;
  const double en = n[a];
  double t[3] = {e[0] - en * n[0], e[1] - en * n[1], e[2] - en * n[2]};
  const double l = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  t1[0] = t[0] / l; t1[1] = t[1] / l; t1[2] = t[2] / l;
  t2[0] = n[1] * t1[2] - n[2] * t1[1];
  t2[1] = n[2] * t1[0] - n[0] * t1[2];
  t2[2] = n[0] * t1[1] - n[1] * t1[0];
}

// monomials of the scaled local coordinates
template <int M>
__device__ inline void monomials(const RowGeom &g, double dx, double dy, double dz, double phi[M]) {
  if constexpr (M == 10) {
    const double X = dx * g.inv_h, Y = dy * g.inv_h, Z = dz * g.inv_h;
    phi[0] = 1.0; phi[1] = X; phi[2] = Y; phi[3] = Z;
    phi[4] = X * X; phi[5] = Y * Y; phi[6] = Z * Z;
    phi[7] = X * Y; phi[8] = X * Z; phi[9] = Y * Z;
  } else {
    const double U = (dx * g.t1[0] + dy * g.t1[1] + dz * g.t1[2]) * g.inv_h;
    const double V = (dx * g.t2[0] + dy * g.t2[1] + dz * g.t2[2]) * g.inv_h;
    phi[0] = 1.0; phi[1] = U; phi[2] = V;
    phi[3] = U * U; phi[4] = V * V; phi[5] = U * V;
  }
}

// derivative of the monomials with respect to the offset d = x_j - x_i,
// contracted with a coefficient vector: returns sum_a pb[a] d(phi_a)/dd
template <int M>
__device__ inline void monomials_grad_dot(const RowGeom &g, double dx, double dy, double dz, const double pb[M],
                                          double out[3]) {
  if constexpr (M == 10) {
    const double X = dx * g.inv_h, Y = dy * g.inv_h, Z = dz * g.inv_h;
    const double gX = pb[1] + 2.0 * X * pb[4] + Y * pb[7] + Z * pb[8];
    const double gY = pb[2] + 2.0 * Y * pb[5] + X * pb[7] + Z * pb[9];
    const double gZ = pb[3] + 2.0 * Z * pb[6] + X * pb[8] + Y * pb[9];
    out[0] = gX * g.inv_h; out[1] = gY * g.inv_h; out[2] = gZ * g.inv_h;
  } else {
    const double U = (dx * g.t1[0] + dy * g.t1[1] + dz * g.t1[2]) * g.inv_h;
    const double V = (dx * g.t2[0] + dy * g.t2[1] + dz * g.t2[2]) * g.inv_h;
    const double gU = pb[1] + 2.0 * U * pb[3] + V * pb[5];
    const double gV = pb[2] + 2.0 * V * pb[4] + U * pb[5];
    for (int c = 0; c < 3; ++c) out[c] = (gU * g.t1[c] + gV * g.t2[c]) * g.inv_h;
  }
}

// support weight w(q) = (e^{-a q^2} - e^{-a}) / (1 - e^{-a}) of q^2.
// FASTW: e^x = 2^k 2^f with t = x log2(e) split in FP64 (k integer,
// |f| <= 1/2), so only 2^f is evaluated in FP32 (hardware exp2, ~1 ulp):
// relative error ~1e-7 independent of the size of x.  Every pass of a kernel
// evaluates the same expression.
template <bool FASTW>
__device__ inline double support_weight_q2(double q2, const WeightFn &wf) {
  if constexpr (FASTW) {
    const double t = -wf.alpha * q2 * 1.4426950408889634;
    const double k = rint(t);
    const float e = __builtin_amdgcn_exp2f((float)(t - k));
    return (ldexp((double)e, (int)k) - wf.ea) * wf.inv_den;
  } else {
    return (exp(-wf.alpha * q2) - wf.ea) * wf.inv_den;
  }
}
// e^{-a q^2} - e^{-a}: the support weight without its normalising factor
// 1 / (1 - e^{-a}).  A common factor of all weights of a row cancels from the
// stencils (G scales by it, the target solutions by its inverse), so the
// batched kernels leave it out.  Given q^2 = d2 s as d2 and cs = s (-a log2 e),
// t = d2 cs is the base-2 exponent; FASTW evaluates it as above.
template <bool FASTW>
__device__ inline double support_weight_raw(double d2, double cs, const WeightFn &wf) {
  if constexpr (FASTW) {
    const double t = d2 * cs;
    const double k = rint(t);
    const float e = __builtin_amdgcn_exp2f((float)fma(d2, cs, -k));
    return ldexp((double)e, (int)k) - wf.ea;
  } else {
    return exp2(d2 * cs) - wf.ea;
  }
}
// the same with q^2 = d2 / r^2
template <bool FASTW>
__device__ inline double support_weight(double d2, double r, const WeightFn &wf) {
  return support_weight_q2<FASTW>(d2 / (r * r), wf);
}
// dw/dd = -2 a e^{-a q^2} / (1 - e^{-a}) * d / r^2 ; returns the scalar factor
__device__ inline double support_weight_dfac(double d2, double r, const WeightFn &wf) {
  const double q2 = d2 / (r * r);
  return -2.0 * wf.alpha * exp(-wf.alpha * q2) * wf.inv_den / (r * r);
}

template <int M>
__device__ inline void gram_add(double G[npack(M)], const double phi[M], double w) {
  double wp[M];
#pragma unroll
  for (int a = 0; a < M; ++a) wp[a] = w * phi[a];
#pragma unroll
  for (int a = 0; a < M; ++a)
#pragma unroll
    for (int c = a; c < M; ++c) G[pidx(a, c, M)] += wp[a] * phi[c];
}

template <int M>
__device__ inline double gram_norm1(const double G[npack(M)]) {
  double best = 0.0;
#pragma unroll
  for (int c = 0; c < M; ++c) {
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < M; ++r) s += fabs(G[r <= c ? pidx(r, c, M) : pidx(c, r, M)]);
    best = fmax(best, s);
  }
  return best;
}

// In-place LDL^T of a packed SPD matrix: afterwards G[pidx(t, r)] (t < r)
// holds L[r][t] and dinv[k] = 1 / D[k].  Returns false if a pivot is not
// positive (or not finite).
template <int M>
__device__ inline bool ldlt(double G[npack(M)], double dinv[M]) {
  double d[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    double s = G[pidx(k, k, M)];
#pragma unroll
    for (int t = 0; t < k; ++t) s -= G[pidx(t, k, M)] * G[pidx(t, k, M)] * d[t];
    d[k] = s;
    if (!(s > 0.0) || !isfinite(s)) return false;
    const double inv = 1.0 / s;
    dinv[k] = inv;
#pragma unroll
    for (int r = k + 1; r < M; ++r) {
      double v = G[pidx(k, r, M)];
#pragma unroll
      for (int t = 0; t < k; ++t) v -= G[pidx(t, r, M)] * G[pidx(t, k, M)] * d[t];
      G[pidx(k, r, M)] = v * inv;
    }
  }
  return true;
}

template <int M>
__device__ inline void ldlt_solve(const double G[npack(M)], const double dinv[M], double x[M]) {
#pragma unroll
  for (int r = 1; r < M; ++r)
#pragma unroll
    for (int t = 0; t < r; ++t) x[r] -= G[pidx(t, r, M)] * x[t];
#pragma unroll
  for (int r = 0; r < M; ++r) x[r] *= dinv[r];
#pragma unroll
  for (int r = M - 2; r >= 0; --r)
#pragma unroll
    for (int t = r + 1; t < M; ++t) x[r] -= G[pidx(r, t, M)] * x[t];
}

// targets of the stencils as combinations of columns of G^{-1}:
// 3D: d/dX -> col 1, d/dY -> col 2, d/dZ -> col 3, Laplacian -> 2 (col 4 + 5 + 6)
// film: d/dU -> col 1, d/dV -> col 2, surface Laplacian -> 2 (col 3 + 4)
template <int M>
__device__ inline double target_coef(int s, int c) {
  if constexpr (M == 10) {
    if (s < 3) return (c == s + 1) ? 1.0 : 0.0;
    return (c >= 4 && c <= 6) ? 2.0 : 0.0;
  } else {
    if (s < 2) return (c == s + 1) ? 1.0 : 0.0;
    if (s == 2) return 0.0;
    return (c == 3 || c == 4) ? 2.0 : 0.0;
  }
}

// ---------------------------------------------------------------- moments
// G_rc = sum_j w_j phi_r phi_c depends only on the moments
// sum_j w_j X^a Y^b Z^c with a+b+c <= 4 (35 in 3D, 15 on the film), so the
// batched kernels accumulate those instead of the 55 (21) Gram entries.
struct MomTable3 {
  int idx[5][5][5];
  constexpr MomTable3() : idx{} {
    int k = 0;
    for (int a = 0; a <= 4; ++a)
      for (int b = 0; a + b <= 4; ++b)
        for (int c = 0; a + b + c <= 4; ++c) idx[a][b][c] = k++;
  }
};
struct MomTable2 {
  int idx[5][5];
  constexpr MomTable2() : idx{} {
    int k = 0;
    for (int a = 0; a <= 4; ++a)
      for (int b = 0; a + b <= 4; ++b) idx[a][b] = k++;
  }
};
constexpr MomTable3 kMom3{};
constexpr MomTable2 kMom2{};
template <int M>
__host__ __device__ constexpr int nmom() { return M == 10 ? 35 : 15; }
// exponents of the monomials [1 X Y Z X^2 Y^2 Z^2 XY XZ YZ] and [1 U V U^2 V^2 UV]
constexpr int kExp3[10][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0},
                              {0, 2, 0}, {0, 0, 2}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
constexpr int kExp2[6][2] = {{0, 0}, {1, 0}, {0, 1}, {2, 0}, {0, 2}, {1, 1}};
// moment index of G_rc
template <int M>
__host__ __device__ constexpr int gram_moment(int r, int c) {
  if constexpr (M == 10)
    return kMom3.idx[kExp3[r][0] + kExp3[c][0]][kExp3[r][1] + kExp3[c][1]][kExp3[r][2] + kExp3[c][2]];
  else
    return kMom2.idx[kExp2[r][0] + kExp2[c][0]][kExp2[r][1] + kExp2[c][1]];
}

// degree of monomial a of the basis
template <int M>
__host__ __device__ constexpr int mono_deg(int a) {
  return M == 10 ? kExp3[a][0] + kExp3[a][1] + kExp3[a][2] : kExp2[a][0] + kExp2[a][1];
}

// Unscaled local coordinates of a neighbour: (dx, dy, dz) in 3D, the offset
// projected on the tangent frame (U, V, 0) on a film.  The batched kernels
// work in these and move the powers of 1/h_i onto the per-row quantities (the
// moments when G is assembled, the target solutions before pass 2), where
// they cost a few operations per row instead of per neighbour.
template <int M>
__device__ inline void local_raw(const RowGeom &g, double dx, double dy, double dz, double &X, double &Y,
                                 double &Z) {
  if constexpr (M == 10) {
    X = dx; Y = dy; Z = dz;
  } else {
    X = fma(dz, g.t1[2], fma(dy, g.t1[1], dx * g.t1[0]));
    Y = fma(dz, g.t2[2], fma(dy, g.t2[1], dx * g.t2[0]));
    Z = 0.0;
  }
}

// mom += w X^a Y^b Z^c for every a + b + c <= 4.  Every monomial of degree 3
// or 4 is (w times a monomial of degree 2) times a monomial of degree 1 or 2,
// so 15 products (6 on a film) feed the 35 (15) accumulations.
template <int M>
__device__ inline void moments_add_raw(double mom[nmom<M>()], double w, double X, double Y, double Z) {
  if constexpr (M == 10) {
    constexpr auto I = [](int a, int b, int c) { return kMom3.idx[a][b][c]; };
    const double wx = w * X, wy = w * Y, wz = w * Z;
    const double xx = X * X, yy = Y * Y, zz = Z * Z, xy = X * Y, xz = X * Z, yz = Y * Z;
    const double wxx = wx * X, wyy = wy * Y, wzz = wz * Z, wxy = wx * Y, wxz = wx * Z, wyz = wy * Z;
    mom[I(0, 0, 0)] += w;
    mom[I(1, 0, 0)] += wx; mom[I(0, 1, 0)] += wy; mom[I(0, 0, 1)] += wz;
    mom[I(2, 0, 0)] += wxx; mom[I(0, 2, 0)] += wyy; mom[I(0, 0, 2)] += wzz;
    mom[I(1, 1, 0)] += wxy; mom[I(1, 0, 1)] += wxz; mom[I(0, 1, 1)] += wyz;
    mom[I(3, 0, 0)] = fma(wxx, X, mom[I(3, 0, 0)]);
    mom[I(2, 1, 0)] = fma(wxx, Y, mom[I(2, 1, 0)]);
    mom[I(2, 0, 1)] = fma(wxx, Z, mom[I(2, 0, 1)]);
    mom[I(1, 2, 0)] = fma(wyy, X, mom[I(1, 2, 0)]);
    mom[I(0, 3, 0)] = fma(wyy, Y, mom[I(0, 3, 0)]);
    mom[I(0, 2, 1)] = fma(wyy, Z, mom[I(0, 2, 1)]);
    mom[I(1, 0, 2)] = fma(wzz, X, mom[I(1, 0, 2)]);
    mom[I(0, 1, 2)] = fma(wzz, Y, mom[I(0, 1, 2)]);
    mom[I(0, 0, 3)] = fma(wzz, Z, mom[I(0, 0, 3)]);
    mom[I(1, 1, 1)] = fma(wxy, Z, mom[I(1, 1, 1)]);
    mom[I(4, 0, 0)] = fma(wxx, xx, mom[I(4, 0, 0)]);
    mom[I(3, 1, 0)] = fma(wxx, xy, mom[I(3, 1, 0)]);
    mom[I(3, 0, 1)] = fma(wxx, xz, mom[I(3, 0, 1)]);
    mom[I(2, 2, 0)] = fma(wxx, yy, mom[I(2, 2, 0)]);
    mom[I(2, 1, 1)] = fma(wxx, yz, mom[I(2, 1, 1)]);
    mom[I(2, 0, 2)] = fma(wxx, zz, mom[I(2, 0, 2)]);
    mom[I(1, 3, 0)] = fma(wyy, xy, mom[I(1, 3, 0)]);
    mom[I(0, 4, 0)] = fma(wyy, yy, mom[I(0, 4, 0)]);
    mom[I(1, 2, 1)] = fma(wyy, xz, mom[I(1, 2, 1)]);
    mom[I(0, 3, 1)] = fma(wyy, yz, mom[I(0, 3, 1)]);
    mom[I(0, 2, 2)] = fma(wyy, zz, mom[I(0, 2, 2)]);
    mom[I(1, 0, 3)] = fma(wzz, xz, mom[I(1, 0, 3)]);
    mom[I(0, 1, 3)] = fma(wzz, yz, mom[I(0, 1, 3)]);
    mom[I(0, 0, 4)] = fma(wzz, zz, mom[I(0, 0, 4)]);
    mom[I(1, 1, 2)] = fma(wzz, xy, mom[I(1, 1, 2)]);
  } else {
    constexpr auto I = [](int a, int b) { return kMom2.idx[a][b]; };
    const double wu = w * X, wv = w * Y;
    const double uu = X * X, vv = Y * Y, uv = X * Y;
    const double wuu = wu * X, wvv = wv * Y, wuv = wu * Y;
    mom[I(0, 0)] += w;
    mom[I(1, 0)] += wu; mom[I(0, 1)] += wv;
    mom[I(2, 0)] += wuu; mom[I(0, 2)] += wvv; mom[I(1, 1)] += wuv;
    mom[I(3, 0)] = fma(wuu, X, mom[I(3, 0)]);
    mom[I(2, 1)] = fma(wuu, Y, mom[I(2, 1)]);
    mom[I(1, 2)] = fma(wvv, X, mom[I(1, 2)]);
    mom[I(0, 3)] = fma(wvv, Y, mom[I(0, 3)]);
    mom[I(4, 0)] = fma(wuu, uu, mom[I(4, 0)]);
    mom[I(3, 1)] = fma(wuu, uv, mom[I(3, 1)]);
    mom[I(2, 2)] = fma(wuu, vv, mom[I(2, 2)]);
    mom[I(1, 3)] = fma(wvv, uv, mom[I(1, 3)]);
    mom[I(0, 4)] = fma(wvv, vv, mom[I(0, 4)]);
  }
}

// sum_a l[a] phi_a(X, Y, Z) over the quadratic basis, in nested (Horner) form:
// l0 + X (l1 + l4 X + l7 Y + l8 Z) + Y (l2 + l5 Y + l9 Z) + Z (l3 + l6 Z)
// (film: l0 + U (l1 + l3 U + l5 V) + V (l2 + l4 V)); 9 (5) fused multiply-adds
template <int M>
__device__ inline double poly_eval(const double *l, double X, double Y, double Z) {
  if constexpr (M == 10) {
    const double ax = fma(l[8], Z, fma(l[7], Y, fma(l[4], X, l[1])));
    const double ay = fma(l[9], Z, fma(l[5], Y, l[2]));
    const double az = fma(l[6], Z, l[3]);
    return fma(Z, az, fma(Y, ay, fma(X, ax, l[0])));
  } else {
    const double au = fma(l[5], Y, fma(l[3], X, l[1]));
    const double av = fma(l[4], Y, l[2]);
    return fma(Y, av, fma(X, au, l[0]));
  }
}

// ---------------------------------------------------------------- team solve
// The batched stencil kernels give each particle a team of T lanes of one
// wave.  Entry (r, c) of the Gram matrix is the moment kGram[r][c].
template <int M>
struct GramTable {
  unsigned char v[M][M];
  constexpr GramTable() : v{} {
    for (int r = 0; r < M; ++r)
      for (int c = 0; c < M; ++c) v[r][c] = (unsigned char)gram_moment<M>(r, c);
  }
};
static __constant__ GramTable<10> kGram3 = GramTable<10>();
static __constant__ GramTable<6> kGram2 = GramTable<6>();

// lanes of a team that take part in the moment transpose-reduction (the
// team's partial sums are first folded down to this many lanes)
__host__ __device__ constexpr int red_lanes(int T) { return T < 4 ? T : 4; }

__host__ __device__ constexpr int cmax(int a, int b) { return a > b ? a : b; }

// orders the LDS traffic of the lanes of one wave around a hand-off
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Team sum of the moments, left in s[0 .. nmom): butterflies down to R8
// lanes, then a transpose through LDS in chunks of R8 moments (lane m of the
// chunk adds the R8 partials of moment c R8 + m in lane order).  s holds at
// least max(nmom, R8 R8) doubles of the team's LDS.
template <int M, int T>
__device__ inline void team_moment_sum(double (&mom)[nmom<M>()], int lane, double *s) {
  constexpr int NM = nmom<M>();
  constexpr int R8 = red_lanes(T);
#pragma unroll
  for (int o = T / 2; o >= R8; o >>= 1)
#pragma unroll
    for (int p = 0; p < NM; ++p) mom[p] += __shfl_xor(mom[p], o, T);
  constexpr int NC = (NM + R8 - 1) / R8;
  const int l8 = lane % R8;
  double res[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
#pragma unroll
    for (int m = 0; m < R8; ++m)
      if (c * R8 + m < NM) s[m * R8 + l8] = mom[c * R8 + m];
    wave_sync();
    double t = s[l8 * R8];
#pragma unroll
    for (int q = 1; q < R8; ++q) t += s[l8 * R8 + q];
    res[c] = t;
    wave_sync();
  }
  // the buffer is free again: the moments take its place
#pragma unroll
  for (int c = 0; c < NC; ++c)
    if (c * R8 + l8 < NM) s[c * R8 + l8] = res[c];
  wave_sync();
}

// In-place Gauss-Jordan inversion of the team's SPD matrix (no pivoting):
// lane owns rows lane + q T (q < NR), the pivot row goes to the other lanes
// through s_prow (M + 1 doubles of the team's LDS).  Afterwards row[q][:] is
// row lane + q T of the inverse.  Returns false if a pivot is not positive
// (or not finite): the matrix is not positive definite.
template <int M, int T>
__device__ inline bool team_gauss_jordan(double (&row)[(M + T - 1) / T][M], int lane, double *s_prow) {
  constexpr int NR = (M + T - 1) / T;
  bool okp = true;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const int kq = k / T;
    if (lane == k % T) {
      const double piv = row[kq][k];
      // 1 / piv from the hardware estimate and two Newton steps
      double ip = __builtin_amdgcn_rcp(piv);
      ip = fma(ip, fma(-piv, ip, 1.0), ip);
      ip = fma(ip, fma(-piv, ip, 1.0), ip);
      row[kq][k] = 1.0;
#pragma unroll
      for (int c = 0; c < M; ++c) row[kq][c] *= ip;
#pragma unroll
      for (int c = 0; c < M; ++c) s_prow[c] = row[kq][c];
      s_prow[M] = piv;
    }
    wave_sync();
    double pr[M];
#pragma unroll
    for (int c = 0; c < M; ++c) pr[c] = s_prow[c];
    const double piv = s_prow[M];
    okp = okp && (piv > 0.0) && isfinite(piv);
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int r = lane + q * T;
      if (r < M && r != k) {
        const double f = row[q][k];
        row[q][k] = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) row[q][c] -= f * pr[c];
      }
    }
    wave_sync();
  }
  return okp;
}

// (x, y, z, h) of every particle packed into one 32-byte record: kernels that
// gather neighbour positions through the column lists read one record per
// neighbour instead of four scattered values
static __global__ void __launch_bounds__(256) k_pack_pos(const double *__restrict__ x, const double *__restrict__ y,
                                                         const double *__restrict__ z, const double *__restrict__ h,
                                                         int64_t n, double4 *__restrict__ pos) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pos[i] = make_double4(x[i], y[i], z[i], h[i]);
}

// Consecutive workgroups are dispatched round-robin over the 8 XCDs of the
// chip, each with its own L2.  Remap so that XCD k processes the k-th
// contiguous slice of the (Morton-ordered) work: neighbouring particles then
// share an L2.  Bijective for any grid size.
__device__ inline unsigned xcd_block(unsigned bid, unsigned nblocks) {
  constexpr unsigned kXcd = 8;
  const unsigned q = nblocks / kXcd, r = nblocks % kXcd;
  const unsigned xcd = bid % kXcd, idx = bid / kXcd;
  return (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

template <typename T>
__device__ inline T team_sum(T v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
  return v;
}
__device__ inline double team_max(double v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, width));
  return v;
}

// Solve the team's Gram system: factor, estimate the 1-norm condition number
// exactly from the columns of G^{-1} (spread over the T lanes of the team),
// and return lam[s][:] = G^{-1} d_s for the four targets on every lane.
// All lanes of a team hold identical G on entry (butterfly sums are
// symmetric), so every decision below is uniform across the team.
template <int M, int T>
__device__ inline bool team_solve(double G[npack(M)], int lane, double lam[4][M], double *kappa) {
  const double gn = gram_norm1<M>(G);
  double dinv[M];
  if (!ldlt<M>(G, dinv)) {
    *kappa = INFINITY;
    return false;
  }
  if constexpr (T == 1) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int r = 0; r < M; ++r) lam[s][r] = 0.0;
    // one lane: columns one at a time, folded into kappa and the targets
    double colmax = 0.0;
    for (int c = 0; c < M; ++c) {
      double x[M];
#pragma unroll
      for (int r = 0; r < M; ++r) x[r] = (r == c) ? 1.0 : 0.0;
      ldlt_solve<M>(G, dinv, x);
      double sacc = 0.0;
#pragma unroll
      for (int r = 0; r < M; ++r) sacc += fabs(x[r]);
      colmax = fmax(colmax, sacc);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const double cf = target_coef<M>(s, c);
        if (cf != 0.0) {
#pragma unroll
          for (int r = 0; r < M; ++r) lam[s][r] += cf * x[r];
        }
      }
    }
    *kappa = gn * colmax;
  } else {
    constexpr int NC = (M + T - 1) / T;
    double cols[NC][M];
    double colmax = 0.0;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const int c = lane + q * T;
#pragma unroll
      for (int r = 0; r < M; ++r) cols[q][r] = (r == c) ? 1.0 : 0.0;
      if (c < M) {
        ldlt_solve<M>(G, dinv, cols[q]);
        double sacc = 0.0;
#pragma unroll
        for (int r = 0; r < M; ++r) sacc += fabs(cols[q][r]);
        colmax = fmax(colmax, sacc);
      }
    }
    colmax = team_max(colmax, T);
    *kappa = gn * colmax;
    // G and its factors are dead here; assemble the targets from the columns
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int r = 0; r < M; ++r) lam[s][r] = 0.0;
#pragma unroll
    for (int c = 1; c < M; ++c) {
      bool used = false;
#pragma unroll
      for (int s = 0; s < 4; ++s) used |= target_coef<M>(s, c) != 0.0;
      if (!used) continue;
#pragma unroll
      for (int r = 0; r < M; ++r) {
        const double v = __shfl(cols[c / T][r], c % T, T);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const double cf = target_coef<M>(s, c);
          if (cf != 0.0) lam[s][r] += cf * v;
        }
      }
    }
  }
  return isfinite(*kappa);
}

}  // namespace gfdm_dev
