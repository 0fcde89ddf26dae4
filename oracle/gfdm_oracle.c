/*
 * FP64 CPU oracle for the GFDM hot path of "Adaptive coupling of 3D and 2D
 * fluid flow models" (Suchde).  TEST INFRASTRUCTURE ONLY: it is used by the
 * test-suite, the smoke check and the CPU baseline of the benchmark, never by
 * the product path.  It shares no code, header or table with the GPU library.
 *
 * Everything here is written for clarity, not speed: plain loops over
 * particles (OpenMP over the outer particle loop only), FP64 throughout,
 * compiled with -ffp-contract=off so that every expression rounds as written.
 *
 * Contents (paper sections / equations):
 *   - neighbourhoods S_i, Eq. (Nbd) in Sec. 2.2; same-model sets, Sec. 6.2
 *   - local PCA covariance and eigenpairs, Sec. 4.1.2 / 4.1.3
 *   - 3D->2D detection (Alg. 2), 2D->3D detection Eq. (2Dto3Dcond), and the
 *     space/time smoothing rules of Sec. 4.3
 *   - GFDM stencils of Eq. (GFDM_Definition), second order (Sec. 2.3), via
 *     Householder QR of the weighted monomial matrix; a long-double normal-
 *     equations form of the same stencil for cross-checking
 *   - stencil application, pressure-system assembly (PDE + zeta*BC, Sec. 7.2)
 *   - 3D->2D transition with averaging, mass lumping and film height (Sec. 5.1,
 *     Alg. 3)
 *   - adjoints of stencil application and of the stencil weights with respect
 *     to particle positions
 *   - film height of the droplet model, Eq. (Height) in Sec. 2.4
 *   - 2D->3D transition with particle addition and mass splitting (Sec. 5.2,
 *     Eq. (psi~), Eq. (gamma), Alg. 4)
 *   - the first loop of the ghost-particle procedure (Sec. 6.1, Alg. 5)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define KIND_INTERIOR 0
#define KIND_FREE_SURFACE 1
#define KIND_WALL 2

/* ------------------------------------------------------------------------- */
/* Neighbourhoods, Eq. (Nbd): j in S_i  iff  |x_j - x_i| <= (h_i + h_j) / 2,  */
/* evaluated as d2 = (dx*dx + dy*dy) + dz*dz <= r*r with r = 0.5*(h_i+h_j).   */
/* S_i holds only particles of the same model as i (Sec. 6.2) unless the      */
/* cross-model variant is requested.  i is always in S_i.                      */
/* ------------------------------------------------------------------------- */
static int in_support(int64_t i, int64_t j, const double *x, const double *y,
                      const double *z, const double *h) {
  double dx = x[j] - x[i];
  double dy = y[j] - y[i];
  double dz = z[j] - z[i];
  double d2 = (dx * dx + dy * dy) + dz * dz;
  double r = 0.5 * (h[i] + h[j]);
  return d2 <= r * r;
}

/* Brute force O(N^2).  col == NULL: fill row_ptr, return nnz.  Otherwise fill
 * col (rows come out ascending because j runs ascending). */
int64_t orc_nbr_brute(int64_t n, const double *x, const double *y, const double *z,
                      const double *h, const int8_t *model, int cross,
                      int64_t *row_ptr, int32_t *col) {
  if (col == NULL) {
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
      int64_t c = 0;
      for (int64_t j = 0; j < n; ++j) {
        if (!cross && model[j] != model[i]) continue;
        if (j == i || in_support(i, j, x, y, z, h)) ++c;
      }
      row_ptr[i + 1] = row_ptr[i] + c;
    }
    return row_ptr[n];
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    int64_t p = row_ptr[i];
    for (int64_t j = 0; j < n; ++j) {
      if (!cross && model[j] != model[i]) continue;
      if (j == i || in_support(i, j, x, y, z, h)) col[p++] = (int32_t)j;
    }
  }
  return row_ptr[n];
}

/* Uniform-grid search: cell edge = max h, so every member of S_i lies in the
 * 27 cells around the cell of i.  Rows are sorted ascending afterwards. */
typedef struct {
  double lo[3], edge;
  int64_t dim[3];
  int64_t *start; /* ncell + 1 */
  int64_t *items; /* particle ids grouped by cell */
} grid_t;

static int64_t cell_coord(double v, double lo, double edge, int64_t dim) {
  int64_t c = (int64_t)floor((v - lo) / edge);
  if (c < 0) c = 0;
  if (c >= dim) c = dim - 1;
  return c;
}

static void grid_build(grid_t *g, int64_t n, const double *x, const double *y,
                       const double *z, const double *h) {
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double hmax = 0.0;
  const double *p[3] = {x, y, z};
  for (int64_t i = 0; i < n; ++i) {
    for (int d = 0; d < 3; ++d) {
      if (p[d][i] < lo[d]) lo[d] = p[d][i];
      if (p[d][i] > hi[d]) hi[d] = p[d][i];
    }
    if (h[i] > hmax) hmax = h[i];
  }
  double edge = hmax > 0 ? hmax : 1.0;
  /* keep the cell count bounded for very sparse clouds */
  for (;;) {
    int64_t total = 1;
    for (int d = 0; d < 3; ++d) total *= (int64_t)floor((hi[d] - lo[d]) / edge) + 1;
    if (total <= 4 * n + 64) break;
    edge *= 1.5;
  }
  g->edge = edge;
  int64_t ncell = 1;
  for (int d = 0; d < 3; ++d) {
    g->lo[d] = lo[d];
    g->dim[d] = (int64_t)floor((hi[d] - lo[d]) / edge) + 1;
    ncell *= g->dim[d];
  }
  g->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
  g->items = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t *cid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) {
    int64_t c0 = cell_coord(x[i], lo[0], edge, g->dim[0]);
    int64_t c1 = cell_coord(y[i], lo[1], edge, g->dim[1]);
    int64_t c2 = cell_coord(z[i], lo[2], edge, g->dim[2]);
    cid[i] = c0 + g->dim[0] * (c1 + g->dim[1] * c2);
    g->start[cid[i] + 1]++;
  }
  for (int64_t c = 0; c < ncell; ++c) g->start[c + 1] += g->start[c];
  int64_t *fillp = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
  memcpy(fillp, g->start, sizeof(int64_t) * (size_t)ncell);
  for (int64_t i = 0; i < n; ++i) g->items[fillp[cid[i]]++] = i;
  free(fillp);
  free(cid);
}

static int cmp_i32(const void *a, const void *b) {
  int32_t u = *(const int32_t *)a, v = *(const int32_t *)b;
  return (u > v) - (u < v);
}

/* visit S_i through the grid; col == NULL counts only */
static int64_t grid_row(const grid_t *g, int64_t i, const double *x, const double *y,
                        const double *z, const double *h, const int8_t *model, int cross,
                        int32_t *out) {
  int64_t c[3] = {cell_coord(x[i], g->lo[0], g->edge, g->dim[0]),
                  cell_coord(y[i], g->lo[1], g->edge, g->dim[1]),
                  cell_coord(z[i], g->lo[2], g->edge, g->dim[2])};
  int64_t cnt = 0;
  for (int64_t a = c[2] - 1; a <= c[2] + 1; ++a) {
    if (a < 0 || a >= g->dim[2]) continue;
    for (int64_t b = c[1] - 1; b <= c[1] + 1; ++b) {
      if (b < 0 || b >= g->dim[1]) continue;
      for (int64_t e = c[0] - 1; e <= c[0] + 1; ++e) {
        if (e < 0 || e >= g->dim[0]) continue;
        int64_t cell = e + g->dim[0] * (b + g->dim[1] * a);
        for (int64_t k = g->start[cell]; k < g->start[cell + 1]; ++k) {
          int64_t j = g->items[k];
          if (!cross && model[j] != model[i]) continue;
          if (j == i || in_support(i, j, x, y, z, h)) {
            if (out) out[cnt] = (int32_t)j;
            ++cnt;
          }
        }
      }
    }
  }
  if (out) qsort(out, (size_t)cnt, sizeof(int32_t), cmp_i32);
  return cnt;
}

int64_t orc_nbr_grid(int64_t n, const double *x, const double *y, const double *z,
                     const double *h, const int8_t *model, int cross, int64_t *row_ptr,
                     int32_t *col) {
  grid_t g;
  grid_build(&g, n, x, y, z, h);
  if (col == NULL) {
    row_ptr[0] = 0;
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) cnt[i] = grid_row(&g, i, x, y, z, h, model, cross, NULL);
    for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[i];
    free(cnt);
  } else {
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) grid_row(&g, i, x, y, z, h, model, cross, col + row_ptr[i]);
  }
  free(g.start);
  free(g.items);
  return row_ptr[n];
}

/* ------------------------------------------------------------------------- */
/* Local PCA, Sec. 4.1.2: P_i = sum_j (x_j - x_c)(x_j - x_c)^T over S_i, with  */
/* x_c the centroid.  Coordinates are taken relative to x_i first (P is       */
/* translation invariant); this keeps exactly coplanar neighbourhoods exactly  */
/* coplanar.  Eigenpairs by the cyclic Jacobi method.                          */
/* ------------------------------------------------------------------------- */

/* Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations.  On return
 * lam[k] are eigenvalues and V[:,k] (column k, V[r*3+k]) unit eigenvectors. */
static void jacobi3(const double A0[9], double lam[3], double V[9]) {
  double A[9];
  memcpy(A, A0, sizeof(A));
  for (int r = 0; r < 9; ++r) V[r] = (r % 4 == 0) ? 1.0 : 0.0;
  double fro = 0.0;
  for (int r = 0; r < 9; ++r) fro += A[r] * A[r];
  fro = sqrt(fro);
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = sqrt(2.0 * (A[1] * A[1] + A[2] * A[2] + A[5] * A[5]));
    if (off <= 1e-15 * fro || off == 0.0) break;
    static const int PQ[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int t = 0; t < 3; ++t) {
      int p = PQ[t][0], q = PQ[t][1];
      double apq = A[p * 3 + q];
      if (apq == 0.0) continue;
      /* rotation angle that annihilates A[p][q]: cot(2 phi) = (a_qq - a_pp)/(2 a_pq) */
      double theta = (A[q * 3 + q] - A[p * 3 + p]) / (2.0 * apq);
      double tn = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      double c = 1.0 / sqrt(tn * tn + 1.0), s = tn * c;
      /* A <- J^T A J with J the rotation in the (p,q) plane */
      for (int k = 0; k < 3; ++k) { /* columns p and q */
        double akp = A[k * 3 + p], akq = A[k * 3 + q];
        A[k * 3 + p] = c * akp - s * akq;
        A[k * 3 + q] = s * akp + c * akq;
      }
      for (int k = 0; k < 3; ++k) { /* rows p and q */
        double apk = A[p * 3 + k], aqk = A[q * 3 + k];
        A[p * 3 + k] = c * apk - s * aqk;
        A[q * 3 + k] = s * apk + c * aqk;
      }
      A[p * 3 + q] = 0.0;
      A[q * 3 + p] = 0.0;
      for (int k = 0; k < 3; ++k) {
        double vkp = V[k * 3 + p], vkq = V[k * 3 + q];
        V[k * 3 + p] = c * vkp - s * vkq;
        V[k * 3 + q] = s * vkp + c * vkq;
      }
    }
  }
  for (int k = 0; k < 3; ++k) lam[k] = A[k * 3 + k];
}

/* lam3n: lambda_1 >= lambda_2 >= lambda_3 per particle; w3_3n: unit eigenvector
 * of lambda_3, sign chosen so that its largest-magnitude component is
 * positive; eps_n: epsilon_lambda = 2 lambda_3 / (lambda_1 + lambda_2)
 * (Sec. 4.1.2), +inf when lambda_1 + lambda_2 == 0. */
void orc_pca(int64_t n, const double *x, const double *y, const double *z,
             const int64_t *row_ptr, const int32_t *col, double *lam3n, double *w3_3n,
             double *eps_n) {
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n; ++i) {
    int64_t b = row_ptr[i], e = row_ptr[i + 1];
    double cnt = (double)(e - b);
    double mx = 0, my = 0, mz = 0;
    for (int64_t k = b; k < e; ++k) {
      int64_t j = col[k];
      mx += x[j] - x[i];
      my += y[j] - y[i];
      mz += z[j] - z[i];
    }
    mx /= cnt; my /= cnt; mz /= cnt;
    double P[9] = {0};
    for (int64_t k = b; k < e; ++k) {
      int64_t j = col[k];
      double d[3] = {(x[j] - x[i]) - mx, (y[j] - y[i]) - my, (z[j] - z[i]) - mz};
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) P[r * 3 + c] += d[r] * d[c];
    }
    double lam[3], V[9];
    jacobi3(P, lam, V);
    int ord[3] = {0, 1, 2};
    /* descending by eigenvalue, ties keep the original order */
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 2 - a; ++c)
        if (lam[ord[c]] < lam[ord[c + 1]]) { int t = ord[c]; ord[c] = ord[c + 1]; ord[c + 1] = t; }
    for (int k = 0; k < 3; ++k) lam3n[3 * i + k] = lam[ord[k]];
    double w[3] = {V[0 * 3 + ord[2]], V[1 * 3 + ord[2]], V[2 * 3 + ord[2]]};
    double nw = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    int big = 0;
    for (int r = 1; r < 3; ++r) if (fabs(w[r]) > fabs(w[big])) big = r;
    double sg = (w[big] < 0) ? -1.0 : 1.0;
    for (int r = 0; r < 3; ++r) w3_3n[3 * i + r] = sg * w[r] / nw;
    double den = lam3n[3 * i] + lam3n[3 * i + 1];
    eps_n[i] = (den == 0.0) ? INFINITY : 2.0 * lam3n[3 * i + 2] / den;
  }
}

/* ------------------------------------------------------------------------- */
/* Transition detection.  flag: 0 none, 1 bulk->film, 2 film->bulk.            */
/*  3D wall particles (Alg. 2): by the kinds of S_i \ {i}:                      */
/*    some free-surface neighbour -> flag iff (eigenvalue AND eigenvector test) */
/*                                   or user criterion                          */
/*    else some interior neighbour -> no flag                                   */
/*    else (walls only, or none)   -> flag without PCA                          */
/*  eigenvalue test: eps_lambda < eps_max (Eq. EigenvalueLimit);                */
/*  eigenvector test: |n.w3| >= cos(theta*) (w3 along the depth direction);     */
/*  literal_rule=1 uses the inequality exactly as printed, |n.w3| < cos(theta*).*/
/*  Film particles: flag 2 iff H_film >= h_3D (Eq. 2Dto3Dcond) or user flag.    */
/*  Smoothing (Sec. 4.3): rule 2 first -- no flag if the particle transitioned  */
/*  in the previous step; then rule 1 -- a flag survives only if some other     */
/*  particle of its cross-model neighbourhood is of the target model or carries */
/*  the same flag.                                                              */
/* ------------------------------------------------------------------------- */
void orc_classify(int64_t n, const int8_t *model, const int8_t *kind, const double *nx,
                  const double *ny, const double *nz, const int64_t *row_ptr,
                  const int32_t *col, const int64_t *xrow_ptr, const int32_t *xcol,
                  const double *eps_n, const double *w3_3n, const double *film_height,
                  const double *h3d, const uint8_t *prev_transitioned,
                  const uint8_t *user_flag, double eps_max, double theta_star,
                  int literal_rule, uint8_t *flag_out) {
  uint8_t *raw = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
  double cos_t = cos(theta_star);
  for (int64_t i = 0; i < n; ++i) {
    uint8_t f = 0;
    int user = user_flag ? (user_flag[i] != 0) : 0;
    if (model[i] == 0 && kind[i] == KIND_WALL) {
      int64_t n_int = 0, n_fs = 0;
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        int64_t j = col[k];
        if (j == i) continue;
        if (kind[j] == KIND_INTERIOR) ++n_int;
        if (kind[j] == KIND_FREE_SURFACE) ++n_fs;
      }
      if (n_fs > 0) {
        double nd = fabs(nx[i] * w3_3n[3 * i] + ny[i] * w3_3n[3 * i + 1] + nz[i] * w3_3n[3 * i + 2]);
        int eig_ok = eps_n[i] < eps_max;
        int vec_ok = literal_rule ? (nd < cos_t) : (nd >= cos_t);
        if ((eig_ok && vec_ok) || user) f = 1;
      } else if (n_int == 0) {
        f = 1;
      }
    } else if (model[i] == 1) {
      int hcrit = (film_height && h3d) ? (film_height[i] >= h3d[i]) : 0;
      if (hcrit || user) f = 2;
    }
    if (prev_transitioned && prev_transitioned[i]) f = 0;
    raw[i] = f;
  }
  for (int64_t i = 0; i < n; ++i) {
    uint8_t f = raw[i];
    if (f != 0 && xrow_ptr != NULL) {
      int target = (f == 1) ? 1 : 0;
      int ok = 0;
      for (int64_t k = xrow_ptr[i]; k < xrow_ptr[i + 1]; ++k) {
        int64_t j = xcol[k];
        if (j == i) continue;
        if (model[j] == target || raw[j] == f) { ok = 1; break; }
      }
      if (!ok) f = 0;
    }
    flag_out[i] = f;
  }
  free(raw);
}

/* ------------------------------------------------------------------------- */
/* GFDM stencils, Eq. (GFDM_Definition), order 2 (Sec. 2.3).                   */
/* For particle i with neighbours j in S_i (including i):                       */
/*   scaled offsets X = (x_j - x_i)/h_i (3D) or tangent coordinates U, V of     */
/*   x_j - x_i scaled by h_i (film, flat surface GFDM of Sec. 2.4);             */
/*   monomials 3D  phi = [1, X, Y, Z, X^2, Y^2, Z^2, XY, XZ, YZ]  (m = 10)      */
/*             film phi = [1, U, V, U^2, V^2, UV]                 (m = 6)       */
/*   weight w_j = (exp(-a q^2) - exp(-a)) / (1 - exp(-a)), q = |x_j-x_i|/r_ij,  */
/*   r_ij = (h_i+h_j)/2 (a Gaussian that vanishes on the support boundary).     */
/* The stencil c (scaled) is the minimiser of sum_j c_j^2 / w_j subject to the  */
/* exactness conditions sum_j c_j phi_k(X_j) = d_k for every monomial, i.e.     */
/* monomials up to order 2 are differentiated exactly.  With A = sqrt(W) M and  */
/* A = QR:  c = sqrt(W) Q R^{-T} d.                                             */
/* Targets d: d/dX -> e_1, d/dY -> e_2, d/dZ -> e_3, Laplacian -> 2 at X^2, Y^2,*/
/* Z^2 (film: d/dU, d/dV, surface Laplacian 2 at U^2, V^2).  Physical weights:  */
/* first derivatives / h_i, Laplacian / h_i^2.  Film gradient weights are       */
/* returned as global x, y, z components t1*c_U + t2*c_V.                       */
/* Output w[(row_ptr[i]+k)*4 + s], s = 0 d/dx, 1 d/dy, 2 d/dz, 3 Laplacian.     */
/* status: 0 ok, 2 rank deficient (min|R_kk| <= 1e-12 max|R_kk|), 3 n_i < m;    */
/* weights are zero for status 2 and 3.  kappa: ||R||_1 ||R^-1||_1.             */
/* ------------------------------------------------------------------------- */
static double support_weight(double q, double a) {
  return (exp(-a * q * q) - exp(-a)) / (1.0 - exp(-a));
}

/* tangent frame of a film particle from its unit normal */
static void tangent_frame(const double nrm[3], double t1[3], double t2[3]) {
  int a = 0;
  for (int r = 1; r < 3; ++r) if (fabs(nrm[r]) < fabs(nrm[a])) a = r;
  double e[3] = {0, 0, 0};
  e[a] = 1.0;
  double en = e[0] * nrm[0] + e[1] * nrm[1] + e[2] * nrm[2];
  for (int r = 0; r < 3; ++r) t1[r] = e[r] - en * nrm[r];
  double l = sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
  for (int r = 0; r < 3; ++r) t1[r] /= l;
  t2[0] = nrm[1] * t1[2] - nrm[2] * t1[1];
  t2[1] = nrm[2] * t1[0] - nrm[0] * t1[2];
  t2[2] = nrm[0] * t1[1] - nrm[1] * t1[0];
}

/* monomials and their first derivatives in the scaled local coordinates */
static int monomials(int film, const double X[3], double *phi, double dphi[][3]) {
  if (!film) {
    double v[10] = {1, X[0], X[1], X[2], X[0] * X[0], X[1] * X[1], X[2] * X[2],
                    X[0] * X[1], X[0] * X[2], X[1] * X[2]};
    memcpy(phi, v, sizeof(v));
    if (dphi) {
      double g[10][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
                         {2 * X[0], 0, 0}, {0, 2 * X[1], 0}, {0, 0, 2 * X[2]},
                         {X[1], X[0], 0}, {X[2], 0, X[0]}, {0, X[2], X[1]}};
      memcpy(dphi, g, sizeof(g));
    }
    return 10;
  }
  double v[6] = {1, X[0], X[1], X[0] * X[0], X[1] * X[1], X[0] * X[1]};
  memcpy(phi, v, sizeof(v));
  if (dphi) {
    double g[6][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {2 * X[0], 0, 0}, {0, 2 * X[1], 0},
                      {X[1], X[0], 0}};
    memcpy(dphi, g, sizeof(g));
  }
  return 6;
}

/* target vectors d for the three (film: two) first derivatives and the Laplacian */
static void targets(int film, double d[4][10]) {
  memset(d, 0, sizeof(double) * 40);
  if (!film) {
    d[0][1] = 1; d[1][2] = 1; d[2][3] = 1;
    d[3][4] = 2; d[3][5] = 2; d[3][6] = 2;
  } else {
    d[0][1] = 1; d[1][2] = 1;
    d[3][3] = 2; d[3][4] = 2;
  }
}

/* local scaled coordinates of neighbour j of i */
static void local_coords(int film, const double dvec[3], double hi, const double t1[3],
                         const double t2[3], double X[3]) {
  if (!film) {
    X[0] = dvec[0] / hi; X[1] = dvec[1] / hi; X[2] = dvec[2] / hi;
  } else {
    X[0] = (dvec[0] * t1[0] + dvec[1] * t1[1] + dvec[2] * t1[2]) / hi;
    X[1] = (dvec[0] * t2[0] + dvec[1] * t2[1] + dvec[2] * t2[2]) / hi;
    X[2] = 0.0;
  }
}

typedef struct {
  int64_t ni;
  int m, film;
  double t1[3], t2[3];
  double *A;    /* ni x m, row-major, overwritten by the Householder vectors */
  double *V;    /* Householder vectors, ni x m (column k in V[:,k], rows >= k) */
  double *sw;   /* sqrt(w_j) */
  double *w;    /* w_j */
  double *X;    /* ni x 3 scaled coordinates */
  double R[100];
  int status;
  double kappa;
} ls_t;

/* Build the weighted monomial matrix of particle i and factor it, A = QR. */
static void ls_factor(ls_t *L, int64_t i, const double *x, const double *y, const double *z,
                      const double *h, const int8_t *model, const double *nx, const double *ny,
                      const double *nz, const int64_t *row_ptr, const int32_t *col, double a) {
  int64_t b = row_ptr[i];
  int64_t ni = row_ptr[i + 1] - b;
  L->ni = ni;
  L->film = model[i] == 1;
  L->m = L->film ? 6 : 10;
  int m = L->m;
  if (L->film) {
    double nrm[3] = {nx[i], ny[i], nz[i]};
    tangent_frame(nrm, L->t1, L->t2);
  }
  L->A = (double *)calloc((size_t)(ni * m + 1), sizeof(double));
  L->V = (double *)calloc((size_t)(ni * m + 1), sizeof(double));
  L->sw = (double *)malloc(sizeof(double) * (size_t)(ni + 1));
  L->w = (double *)malloc(sizeof(double) * (size_t)(ni + 1));
  L->X = (double *)malloc(sizeof(double) * (size_t)(3 * ni + 1));
  for (int64_t k = 0; k < ni; ++k) {
    int64_t j = col[b + k];
    double dv[3] = {x[j] - x[i], y[j] - y[i], z[j] - z[i]};
    double dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    double r = 0.5 * (h[i] + h[j]);
    double wk = support_weight(dist / r, a);
    L->w[k] = wk;
    L->sw[k] = sqrt(wk);
    local_coords(L->film, dv, h[i], L->t1, L->t2, &L->X[3 * k]);
    double phi[10];
    monomials(L->film, &L->X[3 * k], phi, NULL);
    for (int c = 0; c < m; ++c) L->A[k * m + c] = L->sw[k] * phi[c];
  }
  L->status = 0;
  L->kappa = 0;
  if (ni < m) { L->status = 3; return; }
  /* Householder QR: for each column k, reflect A[k:,k] onto a multiple of e_k. */
  double *A = L->A;
  for (int k = 0; k < m; ++k) {
    double nrm2 = 0;
    for (int64_t r = k; r < ni; ++r) nrm2 += A[r * m + k] * A[r * m + k];
    double nrm = sqrt(nrm2);
    double alpha = (A[k * m + k] > 0) ? -nrm : nrm;
    for (int64_t r = 0; r < ni; ++r) L->V[r * m + k] = (r >= k) ? A[r * m + k] : 0.0;
    L->V[k * m + k] -= alpha;
    double vtv = 0;
    for (int64_t r = k; r < ni; ++r) vtv += L->V[r * m + k] * L->V[r * m + k];
    if (vtv > 0) {
      for (int c = k; c < m; ++c) {
        double s = 0;
        for (int64_t r = k; r < ni; ++r) s += L->V[r * m + k] * A[r * m + c];
        s = 2.0 * s / vtv;
        for (int64_t r = k; r < ni; ++r) A[r * m + c] -= s * L->V[r * m + k];
      }
    }
  }
  double rmax = 0, rmin = INFINITY;
  for (int r = 0; r < m; ++r) {
    for (int c = 0; c < m; ++c) L->R[r * 10 + c] = (c >= r) ? A[r * m + c] : 0.0;
    double d = fabs(L->R[r * 10 + r]);
    if (d > rmax) rmax = d;
    if (d < rmin) rmin = d;
  }
  if (!(rmin > 1e-12 * rmax)) { L->status = 2; return; }
  /* kappa_1(R) = ||R||_1 ||R^{-1}||_1 with R^{-1} by back substitution */
  double Rinv[100] = {0};
  for (int c = 0; c < m; ++c) {
    for (int r = m - 1; r >= 0; --r) {
      double s = (r == c) ? 1.0 : 0.0;
      for (int t = r + 1; t < m; ++t) s -= L->R[r * 10 + t] * Rinv[t * 10 + c];
      Rinv[r * 10 + c] = s / L->R[r * 10 + r];
    }
  }
  double n1 = 0, n1i = 0;
  for (int c = 0; c < m; ++c) {
    double s = 0, si = 0;
    for (int r = 0; r < m; ++r) { s += fabs(L->R[r * 10 + c]); si += fabs(Rinv[r * 10 + c]); }
    if (s > n1) n1 = s;
    if (si > n1i) n1i = si;
  }
  L->kappa = n1 * n1i;
}

static void ls_free(ls_t *L) {
  free(L->A); free(L->V); free(L->sw); free(L->w); free(L->X);
}

/* y = Q [z; 0]  with Q = H_0 H_1 ... H_{m-1} */
static void apply_q(const ls_t *L, const double *zt, double *yv) {
  int m = L->m;
  for (int64_t r = 0; r < L->ni; ++r) yv[r] = (r < m) ? zt[r] : 0.0;
  for (int k = m - 1; k >= 0; --k) {
    double vtv = 0, s = 0;
    for (int64_t r = k; r < L->ni; ++r) {
      vtv += L->V[r * m + k] * L->V[r * m + k];
      s += L->V[r * m + k] * yv[r];
    }
    if (vtv == 0) continue;
    s = 2.0 * s / vtv;
    for (int64_t r = k; r < L->ni; ++r) yv[r] -= s * L->V[r * m + k];
  }
}

/* lambda = G^{-1} d with G = R^T R */
static void gram_solve(const ls_t *L, const double *d, double *lam) {
  int m = L->m;
  double zt[10];
  for (int r = 0; r < m; ++r) { /* R^T zt = d */
    double s = d[r];
    for (int t = 0; t < r; ++t) s -= L->R[t * 10 + r] * zt[t];
    zt[r] = s / L->R[r * 10 + r];
  }
  for (int r = m - 1; r >= 0; --r) { /* R lam = zt */
    double s = zt[r];
    for (int t = r + 1; t < m; ++t) s -= L->R[r * 10 + t] * lam[t];
    lam[r] = s / L->R[r * 10 + r];
  }
}

void orc_gfdm_weights(int64_t n, const double *x, const double *y, const double *z,
                      const double *h, const int8_t *model, const double *nx, const double *ny,
                      const double *nz, const int64_t *row_ptr, const int32_t *col,
                      double alpha_w, const int64_t *rows, int64_t nrows, double *w_out,
                      int8_t *status, double *kappa) {
  /* rows == NULL: every particle.  Otherwise only the listed rows are computed. */
  int64_t cnt = rows ? nrows : n;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t t = 0; t < cnt; ++t) {
    int64_t i = rows ? rows[t] : t;
    ls_t L;
    ls_factor(&L, i, x, y, z, h, model, nx, ny, nz, row_ptr, col, alpha_w);
    int64_t b = row_ptr[i];
    double *wi = w_out + 4 * b;
    memset(wi, 0, sizeof(double) * 4 * (size_t)L.ni);
    if (status) status[i] = (int8_t)L.status;
    if (kappa) kappa[i] = L.kappa;
    if (L.status == 0) {
      int m = L.m;
      double d[4][10];
      targets(L.film, d);
      double *yv = (double *)malloc(sizeof(double) * (size_t)L.ni);
      double *chat = (double *)malloc(sizeof(double) * 4 * (size_t)L.ni);
      for (int s = 0; s < 4; ++s) {
        if (L.film && s == 2) { for (int64_t k = 0; k < L.ni; ++k) chat[4 * k + s] = 0; continue; }
        double zt[10];
        for (int r = 0; r < m; ++r) { /* R^T zt = d */
          double acc = d[s][r];
          for (int q = 0; q < r; ++q) acc -= L.R[q * 10 + r] * zt[q];
          zt[r] = acc / L.R[r * 10 + r];
        }
        apply_q(&L, zt, yv);
        for (int64_t k = 0; k < L.ni; ++k) chat[4 * k + s] = L.sw[k] * yv[k];
      }
      double hi = h[i];
      for (int64_t k = 0; k < L.ni; ++k) {
        if (!L.film) {
          for (int s = 0; s < 3; ++s) wi[4 * k + s] = chat[4 * k + s] / hi;
        } else {
          double cu = chat[4 * k + 0] / hi, cv = chat[4 * k + 1] / hi;
          for (int s = 0; s < 3; ++s) wi[4 * k + s] = L.t1[s] * cu + L.t2[s] * cv;
        }
        wi[4 * k + 3] = chat[4 * k + 3] / (hi * hi);
      }
      free(yv);
      free(chat);
    }
    ls_free(&L);
  }
}

/* Condition number of the least-squares Gram matrix G = M^T W M = R^T R of
 * particle i in the scaled local coordinates of Eq. (GFDM_Definition):
 * kappa_1(G) = ||G||_1 ||G^{-1}||_1 with G^{-1} = R^{-1} R^{-T}.  This is the
 * per-particle condition estimate that decides whether a particle's stencil
 * must be recomputed by the FP64 Householder form (spec precision
 * scheme; the paper itself solves every local problem the same way).
 * 0 for status 3 (n_i < m), +inf for status 2 (rank deficient). */
void orc_gram_kappa(int64_t n, const double *x, const double *y, const double *z,
                    const double *h, const int8_t *model, const double *nx, const double *ny,
                    const double *nz, const int64_t *row_ptr, const int32_t *col, double alpha_w,
                    double *kappa_gram) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    ls_t L;
    ls_factor(&L, i, x, y, z, h, model, nx, ny, nz, row_ptr, col, alpha_w);
    if (L.status == 3) { kappa_gram[i] = 0.0; ls_free(&L); continue; }
    if (L.status == 2) { kappa_gram[i] = INFINITY; ls_free(&L); continue; }
    int m = L.m;
    double G[100] = {0}, Rinv[100] = {0}, Ginv[100] = {0};
    for (int r = 0; r < m; ++r)          /* G = R^T R */
      for (int c = 0; c < m; ++c) {
        double acc = 0;
        for (int t = 0; t < m; ++t) acc += L.R[t * 10 + r] * L.R[t * 10 + c];
        G[r * 10 + c] = acc;
      }
    for (int c = 0; c < m; ++c)          /* R^{-1} by back substitution */
      for (int r = m - 1; r >= 0; --r) {
        double acc = (r == c) ? 1.0 : 0.0;
        for (int t = r + 1; t < m; ++t) acc -= L.R[r * 10 + t] * Rinv[t * 10 + c];
        Rinv[r * 10 + c] = acc / L.R[r * 10 + r];
      }
    for (int r = 0; r < m; ++r)          /* G^{-1} = R^{-1} R^{-T} */
      for (int c = 0; c < m; ++c) {
        double acc = 0;
        for (int t = 0; t < m; ++t) acc += Rinv[r * 10 + t] * Rinv[c * 10 + t];
        Ginv[r * 10 + c] = acc;
      }
    double n1 = 0, n1i = 0;
    for (int c = 0; c < m; ++c) {
      double sg = 0, si = 0;
      for (int r = 0; r < m; ++r) { sg += fabs(G[r * 10 + c]); si += fabs(Ginv[r * 10 + c]); }
      if (sg > n1) n1 = sg;
      if (si > n1i) n1i = si;
    }
    kappa_gram[i] = n1 * n1i;
    ls_free(&L);
  }
}

/* The same stencil from the normal equations G lambda = d, G = M^T W M,
 * c_j = w_j phi_j^T lambda, in long double with a Cholesky solve.  Used only
 * to cross-check the Householder form (the two are algebraically equal). */
void orc_gfdm_weights_normal_ld(int64_t n, const double *x, const double *y, const double *z,
                                const double *h, const int8_t *model, const double *nx,
                                const double *ny, const double *nz, const int64_t *row_ptr,
                                const int32_t *col, double alpha_w, double *w_out) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    int64_t b = row_ptr[i], ni = row_ptr[i + 1] - b;
    int film = model[i] == 1;
    int m = film ? 6 : 10;
    double t1[3] = {0}, t2[3] = {0};
    if (film) { double nrm[3] = {nx[i], ny[i], nz[i]}; tangent_frame(nrm, t1, t2); }
    memset(w_out + 4 * b, 0, sizeof(double) * 4 * (size_t)ni);
    if (ni < m) continue;
    long double G[10][10] = {{0}};
    for (int64_t k = 0; k < ni; ++k) {
      int64_t j = col[b + k];
      double dv[3] = {x[j] - x[i], y[j] - y[i], z[j] - z[i]};
      double dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
      long double wk = support_weight(dist / (0.5 * (h[i] + h[j])), alpha_w);
      double X[3], phi[10];
      local_coords(film, dv, h[i], t1, t2, X);
      monomials(film, X, phi, NULL);
      for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) G[r][c] += wk * (long double)phi[r] * (long double)phi[c];
    }
    long double Lc[10][10] = {{0}};
    int ok = 1;
    for (int c = 0; c < m && ok; ++c) {
      long double s = G[c][c];
      for (int k = 0; k < c; ++k) s -= Lc[c][k] * Lc[c][k];
      if (!(s > 0)) { ok = 0; break; }
      Lc[c][c] = sqrtl(s);
      for (int r = c + 1; r < m; ++r) {
        long double t = G[r][c];
        for (int k = 0; k < c; ++k) t -= Lc[r][k] * Lc[c][k];
        Lc[r][c] = t / Lc[c][c];
      }
    }
    if (!ok) continue;
    double d[4][10];
    targets(film, d);
    long double lam[4][10];
    for (int s = 0; s < 4; ++s) {
      long double zt[10];
      for (int r = 0; r < m; ++r) {
        long double acc = d[s][r];
        for (int k = 0; k < r; ++k) acc -= Lc[r][k] * zt[k];
        zt[r] = acc / Lc[r][r];
      }
      for (int r = m - 1; r >= 0; --r) {
        long double acc = zt[r];
        for (int k = r + 1; k < m; ++k) acc -= Lc[k][r] * lam[s][k];
        lam[s][r] = acc / Lc[r][r];
      }
    }
    for (int64_t k = 0; k < ni; ++k) {
      int64_t j = col[b + k];
      double dv[3] = {x[j] - x[i], y[j] - y[i], z[j] - z[i]};
      double dist = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
      long double wk = support_weight(dist / (0.5 * (h[i] + h[j])), alpha_w);
      double X[3], phi[10];
      local_coords(film, dv, h[i], t1, t2, X);
      monomials(film, X, phi, NULL);
      long double c[4];
      for (int s = 0; s < 4; ++s) {
        long double acc = 0;
        for (int r = 0; r < m; ++r) acc += (long double)phi[r] * lam[s][r];
        c[s] = wk * acc;
      }
      double *wk4 = w_out + 4 * (b + k);
      if (!film) {
        for (int s = 0; s < 3; ++s) wk4[s] = (double)(c[s] / h[i]);
      } else {
        for (int s = 0; s < 3; ++s) wk4[s] = (double)((t1[s] * c[0] + t2[s] * c[1]) / h[i]);
      }
      wk4[3] = (double)(c[3] / ((long double)h[i] * h[i]));
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Stencil application, Eq. (GFDM_Definition) in differenced form:             */
/*   y_i^s = sum_{j in S_i, j != i} c_ij^s (u_j - u_i)                          */
/* which equals sum_j c_ij^s u_j because the stencil annihilates constants.     */
/* op_mask bit s selects stencil s; outputs are stacked [K][n] in bit order.    */
/* ------------------------------------------------------------------------- */
void orc_apply(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *w,
               unsigned op_mask, const double *u, double *out) {
  int sel[4], K = 0;
  for (int s = 0; s < 4; ++s) if (op_mask & (1u << s)) sel[K++] = s;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    for (int q = 0; q < K; ++q) {
      double acc = 0;
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        int64_t j = col[k];
        if (j == i) continue;
        acc += w[4 * k + sel[q]] * (u[j] - u[i]);
      }
      out[(int64_t)q * n + i] = acc;
    }
  }
}

/* Transpose of the map u -> y above: ubar_j = sum_i sum_s dy_i^s/du_j ybar_i^s. */
void orc_apply_adjoint(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *w,
                       unsigned op_mask, const double *ybar, double *ubar) {
  int sel[4], K = 0;
  for (int s = 0; s < 4; ++s) if (op_mask & (1u << s)) sel[K++] = s;
  for (int64_t j = 0; j < n; ++j) ubar[j] = 0;
  for (int64_t i = 0; i < n; ++i) {
    for (int q = 0; q < K; ++q) {
      double yb = ybar[(int64_t)q * n + i];
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        int64_t j = col[k];
        if (j == i) continue;
        double c = w[4 * k + sel[q]];
        ubar[j] += c * yb;
        ubar[i] -= c * yb;
      }
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Pressure-system rows (implicit pressure Poisson of the projection scheme,    */
/* Sec. 2.3; PDE + zeta*BC rows of Sec. 7.2):                                   */
/*   0 interior        : A_ij = c_ij^Lap                                        */
/*   1 Dirichlet       : A_ij = delta_ij                                        */
/*   2 combined Neumann: A_ij = c_ij^Lap + (zeta/h_i) n_i . c_ij^grad           */
/*   3 plain Neumann   : A_ij = n_i . c_ij^grad                                 */
/* ------------------------------------------------------------------------- */
void orc_poisson_assemble(int64_t n, const double *h, const double *nx, const double *ny,
                          const double *nz, const int8_t *row_type, const int64_t *row_ptr,
                          const int32_t *col, const double *w, double zeta, double *val) {
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      const double *c = w + 4 * k;
      double ngrad = nx[i] * c[0] + ny[i] * c[1] + nz[i] * c[2];
      switch (row_type[i]) {
        case 0: val[k] = c[3]; break;
        case 1: val[k] = (col[k] == i) ? 1.0 : 0.0; break;
        case 2: val[k] = c[3] + (zeta / h[i]) * ngrad; break;
        default: val[k] = ngrad; break;
      }
    }
  }
}

/* ------------------------------------------------------------------------- */
/* 3D -> 2D transition, Sec. 5.1 / Alg. 3, for particles with flag == 1.        */
/*  candidates: interior / free-surface 3D neighbours of flagged particles;     */
/*  owner(b): the wall particle of S_b nearest to b (smaller index on ties);    */
/*  b is deleted and mapped to owner(b) iff owner(b) is flagged;                */
/*  for flagged i with T_i = {b : owner(b) = i}:                                */
/*    phi_new = (phi_i + sum_T phi_b) / (1 + n(T_i))   (also rho)               */
/*    m_new   = m_i + sum_T m_b                                                 */
/*    H_i     = max_T |(x_b - x_i) . n_i|   (0 if T_i is empty)                 */
/*    d_i     = (6 m_new / (pi rho_new))^(1/3)                                  */
/* Unflagged kept particles keep m, phi, rho; deleted ones get m_out = 0.       */
/* ------------------------------------------------------------------------- */
void orc_transition_3d_to_2d(int64_t n, const double *x, const double *y, const double *z,
                             const int8_t *model, const int8_t *kind, const double *nx,
                             const double *ny, const double *nz, const int64_t *row_ptr,
                             const int32_t *col, const uint8_t *flag, const double *mass,
                             const double *rho, const double *phi, double *mass_out,
                             double *rho_out, double *phi_out, double *height_out,
                             double *diam_out, uint8_t *keep, int32_t *owner) {
  for (int64_t b = 0; b < n; ++b) {
    owner[b] = -1;
    keep[b] = 1;
    if (model[b] != 0 || kind[b] == KIND_WALL) continue;
    int cand = 0;
    for (int64_t k = row_ptr[b]; k < row_ptr[b + 1]; ++k)
      if (flag[col[k]] == 1) { cand = 1; break; }
    if (!cand) continue;
    int64_t best = -1;
    double bestd = INFINITY;
    for (int64_t k = row_ptr[b]; k < row_ptr[b + 1]; ++k) {
      int64_t j = col[k];
      if (kind[j] != KIND_WALL || model[j] != 0) continue;
      double dx = x[j] - x[b], dy = y[j] - y[b], dz = z[j] - z[b];
      double d2 = (dx * dx + dy * dy) + dz * dz;
      if (d2 < bestd) { bestd = d2; best = j; }
    }
    if (best >= 0 && flag[best] == 1) { owner[b] = (int32_t)best; keep[b] = 0; }
  }
  for (int64_t i = 0; i < n; ++i) {
    mass_out[i] = keep[i] ? mass[i] : 0.0;
    rho_out[i] = rho[i];
    phi_out[i] = phi[i];
    height_out[i] = 0.0;
    diam_out[i] = 0.0;
    if (flag[i] != 1) continue;
    double m = mass[i], r = rho[i], p = phi[i], H = 0.0;
    int64_t cnt = 0;
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      int64_t b = col[k];
      if (owner[b] != i) continue;
      m += mass[b];
      r += rho[b];
      p += phi[b];
      double dn = fabs((x[b] - x[i]) * nx[i] + (y[b] - y[i]) * ny[i] + (z[b] - z[i]) * nz[i]);
      if (dn > H) H = dn;
      ++cnt;
    }
    mass_out[i] = m;
    rho_out[i] = r / (double)(1 + cnt);
    phi_out[i] = p / (double)(1 + cnt);
    height_out[i] = H;
    diam_out[i] = cbrt(6.0 * m / (M_PI * rho_out[i]));
  }
}

/* ------------------------------------------------------------------------- */
/* Film height of the droplet model, Eq. (Height), Sec. 2.4: for a film        */
/* particle i                                                                  */
/*   H_i = sum_{j in S_i} alpha / (pi h_j^2) exp(-alpha |x_j - x_i|^2 / h_j^2) V_j */
/* with the droplet volume V_j = pi d_j^3 / 6.  S_i is the same-model          */
/* neighbourhood (it contains i).  3D particles get 0.                         */
/* ------------------------------------------------------------------------- */
void orc_film_height(int64_t n, const double *x, const double *y, const double *z,
                     const double *h, const int8_t *model, const int64_t *row_ptr,
                     const int32_t *col, const double *diam, double alpha, double *height) {
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < n; ++i) {
    double H = 0.0;
    if (model[i] == 1) {
      for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
        int64_t j = col[k];
        double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
        double r2 = (dx * dx + dy * dy) + dz * dz;
        double hj2 = h[j] * h[j];
        double vol = M_PI * diam[j] * diam[j] * diam[j] / 6.0;
        H += alpha / (M_PI * hj2) * exp(-alpha * r2 / hj2) * vol;
      }
    }
    height[i] = H;
  }
}

/* ------------------------------------------------------------------------- */
/* 2D -> 3D transition, Sec. 5.2 and Alg. 4, of the film particles sel[0..ns) */
/* (ascending).  For each source s with film height H, inward unit normal n   */
/* and 3D resolution h3 at its location:                                      */
/*   psi~ = (r_min h3 + r_max h3) / 2        Eq. (psi~)                        */
/*   gamma = ceil(H / psi~)                  Eq. (gamma)   (0 if not H > 0)    */
/*   psi = H / gamma                                                          */
/* The source itself turns into a 3D wall particle and gamma particles are   */
/* added at x + (k psi) n, k = 1..gamma; the one at k = gamma is a free-      */
/* surface particle, the others interior.  Density and the nphi fields (each  */
/* a column of length n) are copied; the mass is split evenly over the        */
/* 1 + gamma particles; every new particle gets h = h3.  The particles of     */
/* source s are written at off[s] .. off[s+1]-1 in the order k = 0..gamma.    */
/* With ox == NULL only off[] is filled.  Returns the total count, or -1 if   */
/* some gamma exceeds max_gamma.                                              */
/* ------------------------------------------------------------------------- */
int64_t orc_transition_2d_to_3d(int64_t ns, const int64_t *sel, const double *x, const double *y,
                                const double *z, const double *nx, const double *ny,
                                const double *nz, const double *H, const double *h3,
                                double r_min, double r_max, const double *mass,
                                const double *rho, const double *phi, int nphi, int64_t n,
                                int64_t max_gamma, int64_t *off, double *ox, double *oy,
                                double *oz, double *oh, int8_t *omodel, int8_t *okind,
                                double *onx, double *ony, double *onz, double *omass,
                                double *orho, double *ophi, int64_t cap, int32_t *osrc) {
  off[0] = 0;
  for (int64_t s = 0; s < ns; ++s) {
    int64_t i = sel[s];
    double psit = (r_min * h3[i] + r_max * h3[i]) / 2.0;
    double g = H[i] > 0.0 ? ceil(H[i] / psit) : 0.0;
    if (!(g <= (double)max_gamma)) return -1;
    off[s + 1] = off[s] + 1 + (int64_t)g;
  }
  if (ox == NULL) return off[ns];
  for (int64_t s = 0; s < ns; ++s) {
    int64_t i = sel[s];
    int64_t gam = off[s + 1] - off[s] - 1;
    double psi = gam > 0 ? H[i] / (double)gam : 0.0;
    for (int64_t k = 0; k <= gam; ++k) {
      int64_t t = off[s] + k;
      double step = (double)k * psi;
      ox[t] = x[i] + step * nx[i];
      oy[t] = y[i] + step * ny[i];
      oz[t] = z[i] + step * nz[i];
      oh[t] = h3[i];
      omodel[t] = 0;
      okind[t] = k == 0 ? KIND_WALL : (k == gam ? KIND_FREE_SURFACE : KIND_INTERIOR);
      onx[t] = nx[i];
      ony[t] = ny[i];
      onz[t] = nz[i];
      omass[t] = mass[i] / (double)(1 + gam);
      orho[t] = rho[i];
      for (int f = 0; f < nphi; ++f) ophi[(int64_t)f * cap + t] = phi[(int64_t)f * n + i];
      osrc[t] = (int32_t)i;
    }
  }
  return off[ns];
}

/* ------------------------------------------------------------------------- */
/* Ghost particles, Sec. 6.1, first loop of Alg. 5: every particle i flags     */
/* itself and each particle j of the other model within its support (the      */
/* cross-model neighbourhood of Eq. (Nbd)).                                   */
/* ------------------------------------------------------------------------- */
void orc_buffer_flags(int64_t n, const int8_t *model, const int64_t *row_ptr, const int32_t *col,
                      uint8_t *flag) {
  for (int64_t i = 0; i < n; ++i) flag[i] = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
      int64_t j = col[k];
      if (model[j] != model[i]) {
        flag[i] = 1;
        flag[j] = 1;
      }
    }
}

/* ------------------------------------------------------------------------- */
/* Adjoint of the stencil weights with respect to particle positions.          */
/* For a loss L(y) with y_i^s = sum_{j!=i} c_ij^s (u_j - u_i), given ybar:      */
/*   cbar_ij^s = ybar_i^s (u_j - u_i)  (physical), scaled back to the           */
/*   dimensionless stencil of particle i.  With lambda_s = G^{-1} d_s,          */
/*   chat_j = w_j phi_j^T lambda_s, the chain rule through G = sum w phi phi^T  */
/*   gives mu_s = G^{-1} sum_j chatbar_j w_j phi_j and                          */
/*     wbar_j   = sum_s chatbar_js (phi_j.lambda_s) - (mu_s.phi_j)(phi_j.lambda_s)*/
/*     phibar_j = sum_s chatbar_js w_j lambda_s - w_j (mu_s (phi_j.lambda_s)    */
/*                                                    + lambda_s (mu_s.phi_j))  */
/*   then dbar_j = J_phi^T phibar_j / h_i + wbar_j dw/dd, with d = x_j - x_i;   */
/*   xbar_j += dbar_j, xbar_i -= dbar_j.  xbar is accumulated (+=).             */
/* ------------------------------------------------------------------------- */
void orc_weights_adjoint_x(int64_t n, const double *x, const double *y, const double *z,
                           const double *h, const int8_t *model, const double *nx,
                           const double *ny, const double *nz, const int64_t *row_ptr,
                           const int32_t *col, double alpha_w, unsigned op_mask,
                           const double *u, const double *ybar, double *xbar3n) {
  int sel[4], K = 0;
  for (int s = 0; s < 4; ++s) if (op_mask & (1u << s)) sel[K++] = s;
  double ea = exp(-alpha_w);
  for (int64_t i = 0; i < n; ++i) {
    ls_t L;
    ls_factor(&L, i, x, y, z, h, model, nx, ny, nz, row_ptr, col, alpha_w);
    if (L.status != 0) { ls_free(&L); continue; }
    int m = L.m;
    int64_t b = row_ptr[i], ni = L.ni;
    double hi = h[i];
    /* gradient w.r.t. the dimensionless stencils: rows k, scaled stencil s */
    double *cb = (double *)calloc((size_t)(4 * ni), sizeof(double));
    for (int q = 0; q < K; ++q) {
      int s = sel[q];
      double yb = ybar[(int64_t)q * n + i];
      for (int64_t k = 0; k < ni; ++k) {
        int64_t j = col[b + k];
        if (j == i) continue;
        double g = yb * (u[j] - u[i]);
        if (s == 3) {
          cb[4 * k + 3] += g / (hi * hi);
        } else if (!L.film) {
          cb[4 * k + s] += g / hi;
        } else {
          cb[4 * k + 0] += L.t1[s] * g / hi;
          cb[4 * k + 1] += L.t2[s] * g / hi;
        }
      }
    }
    double d[4][10];
    targets(L.film, d);
    double lam[4][10], mu[4][10];
    for (int s = 0; s < 4; ++s) {
      gram_solve(&L, d[s], lam[s]);
      double lb[10] = {0};
      for (int64_t k = 0; k < ni; ++k) {
        double phi[10];
        monomials(L.film, &L.X[3 * k], phi, NULL);
        for (int r = 0; r < m; ++r) lb[r] += cb[4 * k + s] * L.w[k] * phi[r];
      }
      gram_solve(&L, lb, mu[s]);
    }
    for (int64_t k = 0; k < ni; ++k) {
      int64_t j = col[b + k];
      if (j == i) continue;
      double phi[10], dphi[10][3];
      monomials(L.film, &L.X[3 * k], phi, dphi);
      double wb = 0, pb[10] = {0};
      for (int s = 0; s < 4; ++s) {
        double pl = 0, mp = 0;
        for (int r = 0; r < m; ++r) { pl += phi[r] * lam[s][r]; mp += mu[s][r] * phi[r]; }
        wb += cb[4 * k + s] * pl - mp * pl;
        for (int r = 0; r < m; ++r)
          pb[r] += cb[4 * k + s] * L.w[k] * lam[s][r] - L.w[k] * (mu[s][r] * pl + lam[s][r] * mp);
      }
      /* dphi/dX (local scaled coordinates) -> d/dd */
      double gX[3] = {0, 0, 0};
      for (int r = 0; r < m; ++r)
        for (int c = 0; c < 3; ++c) gX[c] += dphi[r][c] * pb[r];
      double dd[3];
      if (!L.film) {
        for (int c = 0; c < 3; ++c) dd[c] = gX[c] / hi;
      } else {
        for (int c = 0; c < 3; ++c) dd[c] = (gX[0] * L.t1[c] + gX[1] * L.t2[c]) / hi;
      }
      double dv[3] = {x[j] - x[i], y[j] - y[i], z[j] - z[i]};
      double r = 0.5 * (hi + h[j]);
      double q2 = (dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]) / (r * r);
      /* dw/dd = -2 a exp(-a q^2) / (1 - exp(-a)) * d / r^2 */
      double dwf = -2.0 * alpha_w * exp(-alpha_w * q2) / (1.0 - ea) / (r * r);
      for (int c = 0; c < 3; ++c) dd[c] += wb * dwf * dv[c];
      for (int c = 0; c < 3; ++c) {
        xbar3n[3 * j + c] += dd[c];
        xbar3n[3 * i + c] -= dd[c];
      }
    }
    free(cb);
    ls_free(&L);
  }
}
