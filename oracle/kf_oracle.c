/*
 * kf_oracle.c -- plain FP64 CPU oracle for Kalman-filter track fitting and
 * combinatorial track building.
 *
 * TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
 * CPU-baseline timing are its only users.  It is deliberately slow and
 * literal: full 6x6 matrices, explicit products J C J^T, the textbook
 * K = C H^T (H C H^T + V)^-1 gain and C - K H C covariance update, one track
 * at a time.  It shares no code, header or constant table with the GPU
 * library.
 *
 * What the paper fixes (Cerati et al., "Parallelized Kalman-Filter-Based
 * Reconstruction of Particle Tracks on Many-Core Processors and GPUs"):
 *  - Sec. 2: tracking = seeding, building, fitting; the fit repeats the Kalman
 *    filter over the hits assigned to a track, without branching.
 *  - Sec. 2.1: track state is a 6-vector with 6x6 covariance and hits are 3-D
 *    with 3x3 covariance, both in global coordinates.
 *  - Sec. 3: building partitions each layer's hits into directionally
 *    projective (eta) bins for look-up; "best hit" keeps the hit with the
 *    smallest chi2 increment; the combinatorial variant keeps several
 *    candidates per seed.
 *  - Sec. 3.1: the clone engine ranks a list of all compatible hits and copies
 *    only the best N candidates per seed; it reaches the same candidates as
 *    copying one candidate per compatible hit and then keeping the best N.
 *  - Sec. 4.3: candidates are ranked by number of hits, then by chi2.
 * The helix propagation, the Jacobian, material effects and the update are
 * not written out in the paper; they follow the standard global-coordinate
 * Kalman filter (Fruhwirth 1987, the paper's KF reference), and every
 * reading where the paper is silent is listed in the design notes
 * (propagation to the first crossing within half a turn, surface-constrained
 * Jacobian, Highland multiple scattering with mean energy loss applied after
 * the update on a layer, hole children, tie-breaks of the ranking).
 */
#include "kf_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define CLIGHT 0.299792458e-2 /* GeV / (T cm) */

static int finite_n(const double* v, int n) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(v[i])) return 0;
  return 1;
}

/* C[n][k] = A[n][m] * B[m][k] */
static void mat_mul(int n, int m, int k, const double* A, const double* B, double* C) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < k; ++j) {
      double acc = 0.0;
      for (int l = 0; l < m; ++l) acc += A[i * m + l] * B[l * k + j];
      C[i * k + j] = acc;
    }
}

static void mat_transpose6(const double* A, double* T) {
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) T[j * 6 + i] = A[i * 6 + j];
}

static void symmetrize6(double* C) {
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < i; ++j) {
      double m = 0.5 * (C[i * 6 + j] + C[j * 6 + i]);
      C[i * 6 + j] = m;
      C[j * 6 + i] = m;
    }
}

/* ------------------------------------------------------------------------
 * Helix in B = (0,0,bz).  With a = -q c bz, the transverse momentum turns by
 * phi = a t / pT after transverse path t (counter-clockwise for phi > 0):
 *   x(t)  = x + [px sin(phi) - py (1 - cos(phi))] / a
 *   y(t)  = y + [py sin(phi) + px (1 - cos(phi))] / a
 *   z(t)  = z + pz t / pT
 *   px(t) = px cos(phi) - py sin(phi),  py(t) = py cos(phi) + px sin(phi)
 * ---------------------------------------------------------------------- */
static void helix_step(const double* s, double a, double t, double* o) {
  double pt = hypot(s[3], s[4]);
  double phi = a * t / pt;
  double sn = sin(phi), cs = cos(phi);
  double sa, ca; /* sin(phi)/a and (1-cos(phi))/a */
  if (a != 0.0) {
    double h = sin(0.5 * phi);
    sa = sn / a;
    ca = 2.0 * h * h / a;
  } else {
    sa = t / pt;
    ca = 0.0;
  }
  o[0] = s[0] + s[3] * sa - s[4] * ca;
  o[1] = s[1] + s[4] * sa + s[3] * ca;
  o[2] = s[2] + s[5] * t / pt;
  o[3] = s[3] * cs - s[4] * sn;
  o[4] = s[4] * cs + s[3] * sn;
  o[5] = s[5];
}

/* Smallest transverse path t > 0, within less than half a turn, at which the
 * helix reaches |(x,y)| = R.  Closed form, then Newton polish.  *margin gets
 * the relative distance of the existence test from its threshold. */
static int32_t solve_path(const double* s, double a, double R, double* t_out, double* margin) {
  double pt = hypot(s[3], s[4]);
  if (!(pt > 0.0)) return OR_NO_CROSSING;
  double ux = s[3] / pt, uy = s[4] / pt;
  double au = s[0] * ux + s[1] * uy;  /* P0 . u */
  double an = -s[0] * uy + s[1] * ux; /* P0 . n, n = (-uy, ux) */
  double D = R * R - (s[0] * s[0] + s[1] * s[1]);
  double kappa = a / pt;
  double best = INFINITY;
  if (kappa == 0.0) {
    /* straight line: t^2 + 2 au t - D = 0 */
    double disc = au * au + D;
    *margin = fabs(disc) / (au * au + fabs(D) + 1e-300);
    if (disc < 0.0) return OR_NO_CROSSING;
    double sq = sqrt(disc);
    double r1 = -au + sq, r2 = -au - sq;
    if (r1 > 0.0 && r1 < best) best = r1;
    if (r2 > 0.0 && r2 < best) best = r2;
  } else {
    /* |P(t)|^2 = R^2  <=>  alpha sin(phi) + beta cos(phi) = gamma */
    double alpha = kappa * au;
    double beta = -(kappa * an + 1.0);
    double gamma = 0.5 * kappa * kappa * D - (kappa * an + 1.0);
    double M = hypot(alpha, beta);
    /* decision margin from the equivalent quadratic in w = tan(phi/2)/kappa:
     * A w^2 + 2 au w - D/2 = 0 with A = 2 (1 + kappa an) - kappa^2 D / 2 */
    double A = 2.0 * (1.0 + kappa * an) - 0.5 * kappa * kappa * D;
    *margin = fabs(au * au + 0.5 * A * D) / (au * au + fabs(0.5 * A * D) + 1e-300);
    if (fabs(gamma) > M) return OR_NO_CROSSING;
    double psi = atan2(alpha, beta);
    double dl = acos(gamma / M);
    for (int k = 0; k < 2; ++k) {
      double phi = psi + (k ? -dl : dl);
      while (phi > M_PI) phi -= 2.0 * M_PI;
      while (phi <= -M_PI) phi += 2.0 * M_PI;
      double t = phi / kappa;
      if (t > 0.0 && t < best) best = t;
    }
  }
  if (!isfinite(best)) return OR_NO_CROSSING;
  for (int it = 0; it < 4; ++it) {
    double o[6];
    helix_step(s, a, best, o);
    double f = o[0] * o[0] + o[1] * o[1] - R * R;
    double fp = 2.0 * (o[0] * o[3] + o[1] * o[4]) / pt;
    if (fp == 0.0) break;
    double tn = best - f / fp;
    if (!(tn > 0.0)) break;
    best = tn;
  }
  *t_out = best;
  return 0;
}

/* Jacobian of the state at the crossing with respect to the start state,
 * with the path length itself a function of the start state (the crossing
 * stays on the cylinder):  J = (I - v w^T) Jt, where Jt is the derivative at
 * fixed t, v = d(state)/dt and w^T = (x', y', 0, 0, 0, 0) / (x' ux' + y' uy'). */
static void surface_jacobian(const double* s, const double* o, double a, double t, double* J) {
  double px = s[3], py = s[4], pz = s[5];
  double pt = hypot(px, py);
  double pt2 = pt * pt, pt3 = pt2 * pt;
  double phi = a * t / pt;
  double sn = sin(phi), cs = cos(phi);
  double sa, ca;
  if (a != 0.0) {
    double h = sin(0.5 * phi);
    sa = sn / a;
    ca = 2.0 * h * h / a;
  } else {
    sa = t / pt;
    ca = 0.0;
  }
  double pxp = o[3], pyp = o[4];
  double Jt[36];
  memset(Jt, 0, sizeof Jt);
  Jt[0 * 6 + 0] = 1.0;
  Jt[1 * 6 + 1] = 1.0;
  Jt[2 * 6 + 2] = 1.0;
  Jt[5 * 6 + 5] = 1.0;
  /* d phi / d px = -phi px / pT^2, and (d phi / d px) / a = -t px / pT^3 */
  Jt[0 * 6 + 3] = sa - pxp * t * px / pt3;
  Jt[0 * 6 + 4] = -ca - pxp * t * py / pt3;
  Jt[1 * 6 + 3] = ca - pyp * t * px / pt3;
  Jt[1 * 6 + 4] = sa - pyp * t * py / pt3;
  Jt[2 * 6 + 3] = -pz * t * px / pt3;
  Jt[2 * 6 + 4] = -pz * t * py / pt3;
  Jt[2 * 6 + 5] = t / pt;
  Jt[3 * 6 + 3] = cs + pyp * phi * px / pt2;
  Jt[3 * 6 + 4] = -sn + pyp * phi * py / pt2;
  Jt[4 * 6 + 3] = sn - pxp * phi * px / pt2;
  Jt[4 * 6 + 4] = cs - pxp * phi * py / pt2;
  double kap = a / pt;
  double v[6] = {pxp / pt, pyp / pt, pz / pt, -kap * pyp, kap * pxp, 0.0};
  double den = (o[0] * pxp + o[1] * pyp) / pt;
  double w[6] = {o[0] / den, o[1] / den, 0.0, 0.0, 0.0, 0.0};
  double P[36];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) P[i * 6 + j] = (i == j ? 1.0 : 0.0) - v[i] * w[j];
  mat_mul(6, 6, 6, P, Jt, J);
}

static int32_t propagate_impl(const or_geometry* g, double* s, double* C, int32_t q, double R, double z_half,
                              double* J_out, double* path, double* margin) {
  double mg = INFINITY;
  if (!finite_n(s, 6) || !finite_n(C, 36)) return OR_NONFINITE;
  double a = -(double)q * CLIGHT * g->bz;
  double t;
  double m1 = INFINITY;
  int32_t st = solve_path(s, a, R, &t, &m1);
  if (m1 < mg) mg = m1;
  if (st) {
    if (margin) *margin = mg;
    return st;
  }
  double o[6], J[36], T[36], JT[36], Cn[36];
  helix_step(s, a, t, o);
  if (!finite_n(o, 6)) return OR_NONFINITE;
  if (z_half > 0.0) {
    double mz = fabs(fabs(o[2]) - z_half) / z_half;
    if (mz < mg) mg = mz;
    if (fabs(o[2]) > z_half) {
      if (margin) *margin = mg;
      return OR_OUT_OF_Z;
    }
  }
  surface_jacobian(s, o, a, t, J);
  mat_mul(6, 6, 6, J, C, T);
  mat_transpose6(J, JT);
  mat_mul(6, 6, 6, T, JT, Cn);
  symmetrize6(Cn);
  if (!finite_n(Cn, 36)) return OR_NONFINITE;
  memcpy(s, o, sizeof o);
  memcpy(C, Cn, sizeof Cn);
  if (J_out) memcpy(J_out, J, sizeof J);
  if (path) *path = t;
  if (margin) *margin = mg;
  return 0;
}

int32_t or_propagate_one(const or_geometry* g, double* s, double* C, int32_t q, double R, double z_half, double* J,
                         double* path) {
  return propagate_impl(g, s, C, q, R, z_half, J, path, NULL);
}

/* Thin scatterer on layer `layer`: path thickness x/X0 = x_over_x0 / |cos psi|
 * (psi = angle between momentum and the layer normal), Highland width
 * theta0 = 0.0136/(beta p) sqrt(x/X0) (1 + 0.038 ln(x/(X0 beta^2))), mean
 * energy loss eloss_per_x0 * x/X0.  Momentum scaled by f = p'/p (rows and
 * columns of the covariance likewise), then p'^2 theta0^2 (I - u u^T) added to
 * the momentum block.  theta0 and the loss use the incoming momentum. */
static int32_t material_impl(const or_geometry* g, int32_t layer, double* s, double* C, double* margin) {
  double xx0 = g->x_over_x0[layer];
  if (!(xx0 > 0.0)) return 0;
  double p = sqrt(s[3] * s[3] + s[4] * s[4] + s[5] * s[5]);
  double u[3] = {s[3] / p, s[4] / p, s[5] / p};
  double r = hypot(s[0], s[1]);
  double cospsi = fabs((u[0] * s[0] + u[1] * s[1]) / r);
  double tt = xx0 / cospsi;
  double m = g->mass;
  double E = sqrt(p * p + m * m);
  double beta = p / E;
  double th0 = 0.0136 / (beta * p) * sqrt(tt) * (1.0 + 0.038 * log(tt / (beta * beta)));
  double E2 = E - g->eloss_per_x0 * tt;
  if (margin) *margin = fabs(E2 - m) / m;
  if (!(E2 > m)) return OR_STOPPED;
  double p2 = sqrt(E2 * E2 - m * m);
  double f = p2 / p;
  for (int i = 3; i < 6; ++i) s[i] *= f;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      int mi = i >= 3, mj = j >= 3;
      if (mi && mj)
        C[i * 6 + j] *= f * f;
      else if (mi || mj)
        C[i * 6 + j] *= f;
    }
  double k = p2 * p2 * th0 * th0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[(i + 3) * 6 + (j + 3)] += k * ((i == j ? 1.0 : 0.0) - u[i] * u[j]);
  if (!finite_n(s, 6) || !finite_n(C, 36)) return OR_NONFINITE;
  return 0;
}

int32_t or_material_one(const or_geometry* g, int32_t layer, double* s, double* C) {
  return material_impl(g, layer, s, C, NULL);
}

/* 3x3 inverse by cofactors; returns 0 if the matrix is not positive definite. */
/* Cholesky factor R = L L^T of a symmetric 3x3 matrix (lower triangle read);
 * 0 unless R is positive definite.  A backward-stable factorisation: the
 * residual covariance of a crossing near the tangent point has a condition
 * number near 1e7, where an explicit cofactor inverse loses the gain. */
static int chol3(const double* R, double* L) {
  double d0 = R[0];
  if (!(d0 > 0.0)) return 0;
  double l00 = sqrt(d0);
  double l10 = R[3] / l00, l20 = R[6] / l00;
  double d1 = R[4] - l10 * l10;
  if (!(d1 > 0.0)) return 0;
  double l11 = sqrt(d1);
  double l21 = (R[7] - l20 * l10) / l11;
  double d2 = R[8] - l20 * l20 - l21 * l21;
  if (!(d2 > 0.0)) return 0;
  L[0] = l00; L[1] = 0.0; L[2] = 0.0;
  L[3] = l10; L[4] = l11; L[5] = 0.0;
  L[6] = l20; L[7] = l21; L[8] = sqrt(d2);
  return 1;
}

/* x = (L L^T)^-1 b */
static void chol3_solve(const double* L, const double* b, double* x) {
  double y0 = b[0] / L[0];
  double y1 = (b[1] - L[3] * y0) / L[4];
  double y2 = (b[2] - L[6] * y0 - L[7] * y1) / L[8];
  x[2] = y2 / L[8];
  x[1] = (y1 - L[7] * x[2]) / L[4];
  x[0] = (y0 - L[3] * x[1] - L[6] * x[2]) / L[0];
}

/* Measurement model H = [I3 0]: residual r = m - H x, R = H C H^T + V,
 * chi2 = r^T R^-1 r, gain K = C H^T R^-1, x += K r, C -= K H C; R^-1 applied
 * through its Cholesky factor. */
int32_t or_update_one(double* s, double* C, const double* m, const double* V, double* chi2, int32_t chi2_only) {
  double R[9], L[9];
  if (!finite_n(s, 6) || !finite_n(C, 36)) return OR_NONFINITE;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R[i * 3 + j] = C[i * 6 + j] + V[i * 3 + j];
  if (!chol3(R, L)) return OR_NOT_PD;
  double r[3] = {m[0] - s[0], m[1] - s[1], m[2] - s[2]};
  double Rir[3];
  chol3_solve(L, r, Rir);
  *chi2 = r[0] * Rir[0] + r[1] * Rir[1] + r[2] * Rir[2];
  if (chi2_only) return 0;
  /* K^T = R^-1 H C: column i of H C is (C[0][i], C[1][i], C[2][i]) */
  double K[18], HC[18], KHC[36];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 6; ++j) HC[i * 6 + j] = C[i * 6 + j];
  for (int i = 0; i < 6; ++i) {
    double col[3] = {C[0 * 6 + i], C[1 * 6 + i], C[2 * 6 + i]}, x[3];
    chol3_solve(L, col, x);
    for (int j = 0; j < 3; ++j) K[i * 3 + j] = x[j];
  }
  mat_mul(6, 3, 6, K, HC, KHC);
  for (int i = 0; i < 6; ++i) s[i] += K[i * 3 + 0] * r[0] + K[i * 3 + 1] * r[1] + K[i * 3 + 2] * r[2];
  for (int k = 0; k < 36; ++k) C[k] -= KHC[k];
  symmetrize6(C);
  if (!finite_n(s, 6) || !finite_n(C, 36)) return OR_NONFINITE;
  return 0;
}

int32_t or_propagate(const or_geometry* g, int64_t n, double* state, double* cov, const int8_t* q,
                     const double* r_target, double r_scalar, double z_half, int32_t material_layer,
                     int32_t* status) {
  if (!g || n < 0 || (n && (!state || !cov || !q || !status))) return -1;
  for (int64_t i = 0; i < n; ++i) {
    double s[6], C[36];
    memcpy(s, state + 6 * i, sizeof s);
    memcpy(C, cov + 36 * i, sizeof C);
    int32_t st = 0;
    // a non-finite track is reported as such before any step, as in or_fit
    if (material_layer >= 0)
      st = (finite_n(s, 6) && finite_n(C, 36)) ? material_impl(g, material_layer, s, C, NULL) : OR_NONFINITE;
    if (!st) st = propagate_impl(g, s, C, q[i], r_target ? r_target[i] : r_scalar, z_half, NULL, NULL, NULL);
    if (!st) {
      memcpy(state + 6 * i, s, sizeof s);
      memcpy(cov + 36 * i, C, sizeof C);
    }
    status[i] = st;
  }
  return 0;
}

int32_t or_update(int64_t n, double* state, double* cov, const double* hit_pos, const double* hit_cov, double* chi2,
                  int32_t* status, int32_t chi2_only) {
  if (n < 0) return -1;
  for (int64_t i = 0; i < n; ++i) {
    double s[6], C[36], c2 = 0.0;
    memcpy(s, state + 6 * i, sizeof s);
    memcpy(C, cov + 36 * i, sizeof C);
    int32_t st = or_update_one(s, C, hit_pos + 3 * i, hit_cov + 9 * i, &c2, chi2_only);
    if (!st && !chi2_only) {
      memcpy(state + 6 * i, s, sizeof s);
      memcpy(cov + 36 * i, C, sizeof C);
    }
    chi2[i] = st ? 0.0 : c2;
    status[i] = st;
  }
  return 0;
}

/* Fit: start from the given prior at the vertex and, layer by layer up to the
 * last layer carrying a hit, propagate, update with the hit if there is one,
 * and add the layer's material unless it is the last hit layer. */
/* Kalman filter of one track over its assigned hits, inside out (layers
 * 0 .. last hit layer).  On success s, C hold the state after the last update.
 * A failed crossing or update keeps the state from before that layer; a failed
 * material step keeps the state after that layer's update.  rows_s [L][6] and
 * rows_C [L][36] (nullable) receive the filtered state of every layer the
 * filter completed (after its update, or the prediction on a layer without a
 * hit, before its material); *done the number of such layers. */
static int32_t fit_track(const or_geometry* g, double* s, double* C, int32_t q, const int32_t* hi,
                         const double* hit_pos, const double* hit_cov, double* chi2_out, int32_t* nhits_out,
                         double* rows_s, double* rows_C, int* done) {
  int L = g->n_layers;
  int last = -1;
  for (int l = 0; l < L; ++l)
    if (hi[l] >= 0) last = l;
  double chi2 = 0.0;
  int nh = 0;
  int32_t st = 0;
  *done = 0;
  for (int l = 0; l <= last; ++l) {
    double s2[6], C2[36];
    memcpy(s2, s, sizeof s2);
    memcpy(C2, C, sizeof C2);
    /* no acceptance check in z: the hits are already assigned to the track */
    st = propagate_impl(g, s2, C2, q, g->r[l], 0.0, NULL, NULL, NULL);
    if (st) break;
    if (hi[l] >= 0) {
      double c2;
      const double* hp = hit_pos + 3 * (int64_t)hi[l];
      const double* hc = hit_cov + 9 * (int64_t)hi[l];
      st = or_update_one(s2, C2, hp, hc, &c2, 0);
      if (st) break;
      chi2 += c2;
      nh += 1;
    }
    memcpy(s, s2, sizeof s2);
    memcpy(C, C2, sizeof C2);
    if (rows_s) {
      memcpy(rows_s + 6 * l, s, sizeof s2);
      memcpy(rows_C + 36 * l, C, sizeof C2);
    }
    *done = l + 1;
    if (l < last) {
      st = material_impl(g, l, s2, C2, NULL);
      if (st) break;
      memcpy(s, s2, sizeof s2);
      memcpy(C, C2, sizeof C2);
    }
  }
  *chi2_out = chi2;
  *nhits_out = nh;
  return st;
}

int32_t or_fit(const or_geometry* g, int64_t n, const double* state_in, const double* cov_in, const int8_t* q,
               const int32_t* hit_idx, const double* hit_pos, const double* hit_cov, double* state_out,
               double* cov_out, double* chi2_out, int32_t* nhits_out, int32_t* status_out) {
  if (!g || n < 0) return -1;
  int L = g->n_layers;
  for (int64_t i = 0; i < n; ++i) {
    double s[6], C[36];
    memcpy(s, state_in + 6 * i, sizeof s);
    memcpy(C, cov_in + 36 * i, sizeof C);
    int done;
    status_out[i] = fit_track(g, s, C, q[i], hit_idx + (int64_t)L * i, hit_pos, hit_cov, chi2_out + i,
                              nhits_out + i, NULL, NULL, &done);
    memcpy(state_out + 6 * i, s, sizeof s);
    memcpy(cov_out + 36 * i, C, sizeof C);
  }
  return 0;
}

/* ------------------------------------------------------------------------
 * Smoother: the backward pass after the fit that gives every layer the
 * estimate from all of the track's hits (a Kalman filter followed by a
 * smoother is the paper's final fit of a found track, Sec. 2).  It is the
 * Rauch-Tung-Striebel recursion, run outside in from the last hit layer:
 *   A_l   = Cf_l F_l^T Cp_{l+1}^+
 *   xs_l  = xf_l + A_l (xs_{l+1} - xp_{l+1})
 *   Cs_l  = Cf_l + A_l (Cs_{l+1} - Cp_{l+1}) A_l^T
 * with xf, Cf the filtered and xp, Cp the predicted estimates and F_l the
 * derivative of the step from layer l to l+1 (material of layer l, then the
 * crossing): F = J diag(1, 1, 1, f, f, f), f the momentum ratio of the energy
 * loss, J the surface-constrained Jacobian.  A prediction on a cylinder has no
 * variance along the radial direction of its position, so Cp is singular and
 * its inverse is replaced by the Moore-Penrose pseudo-inverse on the surface.
 * ---------------------------------------------------------------------- */

/* Cholesky factor A = L L^T of an n x n symmetric matrix (lower triangle
 * read); 0 unless A is positive definite. */
static int chol_n(int n, const double* A, double* L) {
  memset(L, 0, sizeof(double) * n * n);
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
    if (!(d > 0.0)) return 0;
    L[j * n + j] = sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double v = A[i * n + j];
      for (int k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = v / L[j * n + j];
    }
  }
  return 1;
}

/* b <- A^-1 b for A = L L^T */
static void chol_solve_n(int n, const double* L, double* b) {
  for (int i = 0; i < n; ++i) {
    for (int k = 0; k < i; ++k) b[i] -= L[i * n + k] * b[k];
    b[i] /= L[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    for (int k = i + 1; k < n; ++k) b[i] -= L[k * n + i] * b[k];
    b[i] /= L[i * n + i];
  }
}

int32_t or_surface_pinv(const double* C, double x, double y, double* Cp) {
  double r = hypot(x, y);
  if (!(r > 0.0)) return 0;
  /* P: rows (tangent, z, px, py, pz), orthonormal, orthogonal to (x, y, 0, 0, 0, 0) */
  double P[30];
  memset(P, 0, sizeof P);
  P[0 * 6 + 0] = -y / r;
  P[0 * 6 + 1] = x / r;
  for (int k = 1; k < 5; ++k) P[k * 6 + (k + 1)] = 1.0;
  double PC[30], S[25], Lf[25];
  mat_mul(5, 6, 6, P, C, PC);
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 6; ++k) acc += PC[i * 6 + k] * P[j * 6 + k];
      S[i * 5 + j] = acc;
    }
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < i; ++j) S[j * 5 + i] = S[i * 5 + j] = 0.5 * (S[i * 5 + j] + S[j * 5 + i]);
  if (!chol_n(5, S, Lf)) return 0;
  /* Sinv P, column by column of P */
  double SiP[30];
  for (int c = 0; c < 6; ++c) {
    double b[5];
    for (int i = 0; i < 5; ++i) b[i] = P[i * 6 + c];
    chol_solve_n(5, Lf, b);
    for (int i = 0; i < 5; ++i) SiP[i * 6 + c] = b[i];
  }
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 5; ++k) acc += P[k * 6 + i] * SiP[k * 6 + j];
      Cp[i * 6 + j] = acc;
    }
  symmetrize6(Cp);
  return 1;
}

void or_rts_step(const double* xf, const double* Cf, const double* F, const double* xp, const double* Cp,
                 const double* Cp_inv, const double* xs_next, const double* Cs_next, double* xs, double* Cs) {
  double Ft[36], CfFt[36], A[36], At[36], M[36], AM[36], AMAt[36];
  mat_transpose6(F, Ft);
  mat_mul(6, 6, 6, Cf, Ft, CfFt);
  mat_mul(6, 6, 6, CfFt, Cp_inv, A);
  double d[6];
  for (int i = 0; i < 6; ++i) d[i] = xs_next[i] - xp[i];
  for (int i = 0; i < 6; ++i) {
    double acc = 0.0;
    for (int k = 0; k < 6; ++k) acc += A[i * 6 + k] * d[k];
    xs[i] = xf[i] + acc;
  }
  for (int k = 0; k < 36; ++k) M[k] = Cs_next[k] - Cp[k];
  mat_transpose6(A, At);
  mat_mul(6, 6, 6, A, M, AM);
  mat_mul(6, 6, 6, AM, At, AMAt);
  for (int k = 0; k < 36; ++k) Cs[k] = Cf[k] + AMAt[k];
  symmetrize6(Cs);
}

int32_t or_smooth(const or_geometry* g, int64_t n, const double* state_in, const double* cov_in, const int8_t* q,
                  const int32_t* hit_idx, const double* hit_pos, const double* hit_cov, double* state_out,
                  double* cov_out, int32_t* status_out) {
  if (!g || n < 0) return -1;
  int L = g->n_layers;
  for (int64_t i = 0; i < n; ++i) {
    double s[6], C[36], chi2;
    int32_t nh;
    int done;
    double* rs = state_out + (int64_t)6 * L * i;
    double* rc = cov_out + (int64_t)36 * L * i;
    for (int k = 0; k < 6 * L; ++k) rs[k] = NAN;
    for (int k = 0; k < 36 * L; ++k) rc[k] = NAN;
    memcpy(s, state_in + 6 * i, sizeof s);
    memcpy(C, cov_in + 36 * i, sizeof C);
    int32_t st = fit_track(g, s, C, q[i], hit_idx + (int64_t)L * i, hit_pos, hit_cov, &chi2, &nh, rs, rc, &done);
    /* the last row is already smoothed (it has seen every hit); a failed fit keeps its filtered rows */
    for (int l = done - 2; st == 0 && l >= 0; --l) {
      double x[6], Cx[36], J[36], F[36], Cpi[36];
      memcpy(x, rs + 6 * l, sizeof x);
      memcpy(Cx, rc + 36 * l, sizeof Cx);
      double p0 = sqrt(x[3] * x[3] + x[4] * x[4] + x[5] * x[5]);
      /* the same steps the filter took from this layer to the next */
      st = material_impl(g, l, x, Cx, NULL);
      if (st) break;
      double f = sqrt(x[3] * x[3] + x[4] * x[4] + x[5] * x[5]) / p0;
      st = propagate_impl(g, x, Cx, q[i], g->r[l + 1], 0.0, J, NULL, NULL);
      if (st) break;
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) F[a * 6 + b] = J[a * 6 + b] * (b >= 3 ? f : 1.0);
      if (!or_surface_pinv(Cx, x[0], x[1], Cpi)) {
        st = OR_NOT_PD;
        break;
      }
      double xs[6], Cs[36];
      or_rts_step(rs + 6 * l, rc + 36 * l, F, x, Cx, Cpi, rs + 6 * (l + 1), rc + 36 * (l + 1), xs, Cs);
      memcpy(rs + 6 * l, xs, sizeof xs);
      memcpy(rc + 36 * l, Cs, sizeof Cs);
    }
    status_out[i] = st;
  }
  return 0;
}

/* ------------------------------------------------------------------------
 * Hit binning.  Decisions are taken in double precision on the given
 * coordinates: phi = atan2(y, x) in [-pi, pi], i_phi = floor((phi + pi) n_phi
 * / (2 pi)); eta = asinh(z / R_layer), eta_max = asinh(z_half / R_layer),
 * i_eta = floor((eta + eta_max) n_eta / (2 eta_max)); both clamped.
 * ---------------------------------------------------------------------- */
static int phi_bin_of(double phi, int n_phi) {
  int b = (int)floor((phi + M_PI) * (double)n_phi / (2.0 * M_PI));
  if (b < 0) b = 0;
  if (b > n_phi - 1) b = n_phi - 1;
  return b;
}

static int eta_bin_of(double z, double R, double zh, int n_eta) {
  double eta = asinh(z / R);
  double emax = asinh(zh / R);
  int b = (int)floor((eta + emax) * (double)n_eta / (2.0 * emax));
  if (b < 0) b = 0;
  if (b > n_eta - 1) b = n_eta - 1;
  return b;
}

static int hit_bin(const double* p, double R, double zh, int n_phi, int n_eta) {
  return eta_bin_of(p[2], R, zh, n_eta) * n_phi + phi_bin_of(atan2(p[1], p[0]), n_phi);
}

int32_t or_bin_hits(const or_geometry* g, int64_t n_events, const int64_t* layer_offsets, const double* hit_pos,
                    int32_t n_phi, int32_t n_eta, int32_t* bin_offsets, int64_t* perm, int32_t* bin_of) {
  int L = g->n_layers;
  int nb = n_phi * n_eta;
  if (n_phi <= 0 || n_eta <= 0) return -1;
  int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (nb + 1));
  for (int64_t e = 0; e < n_events; ++e)
    for (int l = 0; l < L; ++l) {
      int64_t lo = layer_offsets[e * L + l], hi = layer_offsets[e * L + l + 1];
      int32_t* bo = bin_offsets + (e * L + l) * (int64_t)(nb + 1);
      memset(cnt, 0, sizeof(int64_t) * (nb + 1));
      for (int64_t h = lo; h < hi; ++h) {
        int b = hit_bin(hit_pos + 3 * h, g->r[l], g->z_half[l], n_phi, n_eta);
        if (bin_of) bin_of[h] = b;
        cnt[b + 1] += 1;
      }
      for (int b = 0; b < nb; ++b) cnt[b + 1] += cnt[b];
      for (int b = 0; b <= nb; ++b) bo[b] = (int32_t)(lo + cnt[b]);
      /* stable placement in original index order */
      for (int64_t h = lo; h < hi; ++h) {
        int b = hit_bin(hit_pos + 3 * h, g->r[l], g->z_half[l], n_phi, n_eta);
        perm[lo + cnt[b]] = h;
        cnt[b] += 1;
      }
    }
  free(cnt);
  return 0;
}

void or_layer_vmax(const or_geometry* g, int64_t n_events, const int64_t* layer_offsets, const double* hit_cov,
                   double* vmax) {
  const int64_t n_el = n_events * g->n_layers;
  for (int64_t el = 0; el < n_el; ++el) {
    vmax[2 * el] = 0.0;
    vmax[2 * el + 1] = 0.0;
    for (int64_t h = layer_offsets[el]; h < layer_offsets[el + 1]; ++h) {
      const double* V = hit_cov + 9 * h;
      double a = V[0], b = V[1], c = V[4];
      double lam = 0.5 * (a + c) + sqrt(0.25 * (a - c) * (a - c) + b * b);
      if (lam > vmax[2 * el]) vmax[2 * el] = lam;
      if (V[8] > vmax[2 * el + 1]) vmax[2 * el + 1] = V[8];
    }
  }
}

/* ------------------------------------------------------------------------
 * Combinatorial building.
 * ---------------------------------------------------------------------- */
typedef struct {
  double s[6], C[36];
  double chi2;
  int32_t nhits;
  int32_t status; /* nonzero = stopped */
  int32_t* hits;  /* [L] */
} ocand;

typedef struct {
  int32_t parent;
  int64_t hit; /* global index; -1 = hole, or carried stopped candidate */
  int32_t nhits;
  double chi2;
} ochild;

/* total order: more hits first, then smaller chi2, then parent rank, then
 * hit index, with the hole (no hit) last */
static int child_cmp(const void* pa, const void* pb) {
  const ochild* a = (const ochild*)pa;
  const ochild* b = (const ochild*)pb;
  if (a->nhits != b->nhits) return a->nhits > b->nhits ? -1 : 1;
  if (a->chi2 != b->chi2) return a->chi2 < b->chi2 ? -1 : 1;
  if (a->parent != b->parent) return a->parent < b->parent ? -1 : 1;
  int64_t ha = a->hit < 0 ? INT64_MAX : a->hit;
  int64_t hb = b->hit < 0 ? INT64_MAX : b->hit;
  if (ha != hb) return ha < hb ? -1 : 1;
  return 0;
}

typedef struct {
  ochild* v;
  int64_t n, cap;
} childvec;

static void push_child(childvec* cv, ochild c) {
  if (cv->n == cv->cap) {
    cv->cap = cv->cap ? 2 * cv->cap : 64;
    cv->v = (ochild*)realloc(cv->v, sizeof(ochild) * cv->cap);
  }
  cv->v[cv->n++] = c;
}

static double wrap_pi(double a) {
  while (a >= M_PI) a -= 2.0 * M_PI;
  while (a < -M_PI) a += 2.0 * M_PI;
  return a;
}

/* ------------------------------------------------------------------------
 * Learned search window (project addition).
 * ---------------------------------------------------------------------- */
double or_bf16(double x) {
  /* nearest value with 8 significant bits (ties to even), bfloat16's exponent range */
  if (!isfinite(x) || x == 0.0) return x;
  int e;
  frexp(x, &e); /* |x| = m 2^e, 0.5 <= m < 1 */
  if (e < -125) e = -125;
  double q = ldexp(1.0, e - 8);
  return nearbyint(x / q) * q; /* default rounding mode: half to even */
}

/* the network on parameters already rounded (weights to bfloat16, biases to float32) */
static void mlp_forward_rounded(const double* P, const double x[8], double o[2]) {
  const double* W1 = P;
  const double* b1 = W1 + 64 * 8;
  const double* W2 = b1 + 64;
  const double* b2 = W2 + 64 * 64;
  const double* W3 = b2 + 64;
  const double* b3 = W3 + 2 * 64;
  double xb[8], h1[64], h2[64];
  for (int i = 0; i < 8; ++i) xb[i] = or_bf16(x[i]);
  for (int i = 0; i < 64; ++i) {
    double a = b1[i];
    for (int k = 0; k < 8; ++k) a += W1[i * 8 + k] * xb[k];
    h1[i] = or_bf16(a > 0.0 ? a : 0.0);
  }
  for (int i = 0; i < 64; ++i) {
    double a = b2[i];
    for (int k = 0; k < 64; ++k) a += W2[i * 64 + k] * h1[k];
    h2[i] = or_bf16(a > 0.0 ? a : 0.0);
  }
  for (int i = 0; i < 2; ++i) {
    double a = b3[i];
    for (int k = 0; k < 64; ++k) a += W3[i * 64 + k] * h2[k];
    o[i] = a;
  }
}

static void round_params(const double* P, double* R) {
  /* weight blocks W1 [64][8], W2 [64][64], W3 [2][64] to bfloat16; biases to float32 */
  static const int len[6] = {64 * 8, 64, 64 * 64, 64, 2 * 64, 2};
  int off = 0;
  for (int b = 0; b < 6; ++b) {
    for (int i = 0; i < len[b]; ++i) R[off + i] = (b % 2 == 0) ? or_bf16(P[off + i]) : (double)(float)P[off + i];
    off += len[b];
  }
}

void or_mlp_forward(const double* P, const double x[8], double o[2]) {
  double R[OR_MLP_PARAMS];
  round_params(P, R);
  mlp_forward_rounded(R, x, o);
}

void or_window_features(const double s[6], const double C[36], int q, double r_from, double r_to, double zh,
                        double f[8]) {
  double pt = hypot(s[3], s[4]);
  double r = hypot(s[0], s[1]);
  double tx = -s[1] / r, ty = s[0] / r;
  double ctt = tx * tx * C[0] + 2.0 * tx * ty * C[1] + ty * ty * C[7];
  f[0] = q / pt;
  f[1] = s[5] / pt;
  f[2] = s[2] / zh;
  f[3] = (s[0] * s[4] - s[1] * s[3]) / (pt * r);
  f[4] = r_from / 100.0;
  f[5] = r_to / 100.0;
  f[6] = 0.5 * log(ctt > 1e-30 ? ctt : 1e-30);
  f[7] = 0.5 * log(C[14] > 1e-30 ? C[14] : 1e-30);
}

typedef struct {
  int64_t hit;
  double chi2;
  int inside; /* inside the learned box */
} ohit;

typedef struct {
  ohit* v;
  int64_t n, cap;
} hitvec;

static void push_hit(hitvec* hv, ohit h) {
  if (hv->n == hv->cap) {
    hv->cap = hv->cap ? 2 * hv->cap : 64;
    hv->v = (ohit*)realloc(hv->v, sizeof(ohit) * hv->cap);
  }
  hv->v[hv->n++] = h;
}

int32_t or_build(const or_geometry* g, const or_build_cfg* cfg, int64_t n_events, const int64_t* layer_offsets,
                 const double* hit_pos, const double* hit_cov, int64_t n_seeds, const int64_t* seed_event,
                 const double* seed_state, const double* seed_cov, const int8_t* seed_q, const int64_t* seed_hits,
                 int32_t first_layer, int32_t* n_cands, int32_t* cand_hits, double* cand_chi2, int32_t* cand_nhits,
                 int32_t* cand_status, double* best_state, double* best_cov, double* margin_cut,
                 double* margin_rank, int64_t* hits_examined, double* margin_window, int64_t* fallbacks) {
  const int L = g->n_layers;
  const int N = cfg->max_cands;
  if (N < 1 || first_layer < 0 || n_seeds < 0) return -1;
  const double cut = cfg->chi2_cut;
  const int nphi = cfg->n_phi, neta = cfg->n_eta, nb = nphi * neta;
  int32_t* own_bins = NULL;
  int64_t* own_perm = NULL;
  double* own_vmax = NULL;
  const int32_t* bin_offsets = cfg->bin_offsets;
  const int64_t* perm = cfg->perm;
  const double* vmax = cfg->layer_vmax; /* per (event, layer): max x-y eigenvalue and max zz of the hit covariances */
  int64_t H = layer_offsets[n_events * L];
  if (cfg->mode == 1 && (!bin_offsets || !perm)) {
    own_bins = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_events * L) * (nb + 1));
    own_perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)(H > 0 ? H : 1));
    or_bin_hits(g, n_events, layer_offsets, hit_pos, nphi, neta, own_bins, own_perm, NULL);
    bin_offsets = own_bins;
    perm = own_perm;
  }
  if (!vmax) {
    own_vmax = (double*)malloc(sizeof(double) * (size_t)(n_events * L) * 2);
    or_layer_vmax(g, n_events, layer_offsets, hit_cov, own_vmax);
    vmax = own_vmax;
  }

  ocand* cur = (ocand*)calloc((size_t)N, sizeof(ocand));
  ocand* nxt = (ocand*)calloc((size_t)N, sizeof(ocand));
  ocand* prop = (ocand*)calloc((size_t)N, sizeof(ocand)); /* propagated parents */
  for (int k = 0; k < N; ++k) {
    cur[k].hits = (int32_t*)malloc(sizeof(int32_t) * L);
    nxt[k].hits = (int32_t*)malloc(sizeof(int32_t) * L);
    prop[k].hits = NULL;
  }
  childvec cv = {NULL, 0, 0};
  hitvec hv = {NULL, 0, 0};
  const int learned = cfg->mlp_params != NULL;
  double* mlp_r = NULL;
  if (learned) {
    mlp_r = (double*)malloc(sizeof(double) * OR_MLP_PARAMS);
    round_params(cfg->mlp_params, mlp_r);
  }

  for (int64_t si = 0; si < n_seeds; ++si) {
    int64_t ev = seed_event[si];
    double mcut = INFINITY, mrank = INFINITY, mwin = INFINITY;
    int64_t examined = 0, n_fb = 0;
    int nc = 1;
    memcpy(cur[0].s, seed_state + 6 * si, sizeof cur[0].s);
    memcpy(cur[0].C, seed_cov + 36 * si, sizeof cur[0].C);
    cur[0].chi2 = 0.0;
    cur[0].nhits = 3;
    cur[0].status = finite_n(cur[0].s, 6) && finite_n(cur[0].C, 36) ? 0 : OR_NONFINITE;
    for (int l = 0; l < L; ++l) cur[0].hits[l] = -1;
    for (int l = 0; l < 3 && l < L; ++l) cur[0].hits[l] = (int32_t)seed_hits[3 * si + l];

    for (int l = first_layer; l < L; ++l) {
      int64_t el = ev * L + l;
      int64_t hlo = layer_offsets[el], hhi = layer_offsets[el + 1];
      double R = g->r[l];
      cv.n = 0;
      for (int c = 0; c < nc; ++c) {
        ocand* pc = &cur[c];
        ocand* pp = &prop[c];
        pp->status = pc->status;
        memcpy(pp->s, pc->s, sizeof pp->s);
        memcpy(pp->C, pc->C, sizeof pp->C);
        if (!pc->status) {
          double m1 = INFINITY;
          int32_t st = 0;
          if (l >= 1) st = material_impl(g, l - 1, pp->s, pp->C, &m1);
          if (m1 < mcut) mcut = m1;
          if (!st) {
            double m2 = INFINITY;
            st = propagate_impl(g, pp->s, pp->C, seed_q[si], R, g->z_half[l], NULL, NULL, &m2);
            if (m2 < mcut) mcut = m2;
          }
          if (st) {
            /* stopped: keep the last valid state (before this layer) */
            pp->status = st;
            memcpy(pp->s, pc->s, sizeof pp->s);
            memcpy(pp->C, pc->C, sizeof pp->C);
          }
        }
        if (pp->status) {
          ochild ch = {c, -1, pc->nhits, pc->chi2};
          push_child(&cv, ch);
          continue;
        }
        /* candidate hits: every hit of the layer, or only the window's bins */
        if (cfg->mode == 0) {
          for (int64_t h = hlo; h < hhi; ++h) {
            double c2;
            double s2[6], C2[36];
            memcpy(s2, pp->s, sizeof s2);
            memcpy(C2, pp->C, sizeof C2);
            if (or_update_one(s2, C2, hit_pos + 3 * h, hit_cov + 9 * h, &c2, 1)) continue;
            examined++;
            double mc = fabs(c2 - cut) / cut;
            if (mc < mcut) mcut = mc;
            if (c2 < cut) {
              ohit oh = {h, c2, 1};
              push_hit(&hv, oh);
            }
          }
        } else {
          /* window: |R sin(dphi)| <= sqrt(cut R_tt), |dz| <= sqrt(cut R_zz) bounds the chi2 < cut ellipsoid */
          double php = atan2(pp->s[1], pp->s[0]);
          double tx = -sin(php), ty = cos(php);
          double Rtt = tx * tx * pp->C[0] + 2.0 * tx * ty * pp->C[1] + ty * ty * pp->C[7] + vmax[2 * el];
          double Rzz = pp->C[14] + vmax[2 * el + 1];
          double fac = 1.0 + cfg->window_margin;
          double wt = sqrt(cut * Rtt) * fac / R;
          double dz = sqrt(cut * Rzz) * fac;
          int full_phi = wt >= 1.0;
          double dphi = full_phi ? M_PI : asin(wt);
          int ie0 = eta_bin_of(pp->s[2] - dz, R, g->z_half[l], neta);
          int ie1 = eta_bin_of(pp->s[2] + dz, R, g->z_half[l], neta);
          int ip0 = 0, nspan = nphi;
          if (!full_phi && dphi < 0.5 * M_PI) {
            ip0 = phi_bin_of(wrap_pi(php - dphi), nphi);
            int ip1 = phi_bin_of(wrap_pi(php + dphi), nphi);
            nspan = ((ip1 - ip0) % nphi + nphi) % nphi + 1;
          }
          const int32_t* bo = bin_offsets + el * (int64_t)(nb + 1);
          for (int ie = ie0; ie <= ie1; ++ie)
            for (int k = 0; k < nspan; ++k) {
              int ip = (ip0 + k) % nphi;
              int b = ie * nphi + ip;
              for (int32_t j = bo[b]; j < bo[b + 1]; ++j) {
                int64_t h = perm[j];
                double c2;
                double s2[6], C2[36];
                memcpy(s2, pp->s, sizeof s2);
                memcpy(C2, pp->C, sizeof C2);
                if (or_update_one(s2, C2, hit_pos + 3 * h, hit_cov + 9 * h, &c2, 1)) continue;
                examined++;
                double mc = fabs(c2 - cut) / cut;
                if (mc < mcut) mcut = mc;
                if (c2 < cut) {
                  ohit oh = {h, c2, 1};
                  push_hit(&hv, oh);
                }
              }
            }
        }
        /* learned window: keep the compatible hits inside the learned box, if any */
        int any_inside = 1;
        if (learned) {
          double f[8], o[2];
          or_window_features(pp->s, pp->C, seed_q[si], l >= 1 ? g->r[l - 1] : 0.0, R, g->z_half[l], f);
          mlp_forward_rounded(mlp_r, f, o);
          double wl_t = cfg->learned_nsigma * exp(o[0]), wl_z = cfg->learned_nsigma * exp(o[1]);
          double rr = hypot(pp->s[0], pp->s[1]);
          double tx = -pp->s[1] / rr, ty = pp->s[0] / rr;
          any_inside = 0;
          for (int64_t i = 0; i < hv.n; ++i) {
            const double* m = hit_pos + 3 * hv.v[i].hit;
            double qt = fabs(tx * (m[0] - pp->s[0]) + ty * (m[1] - pp->s[1])) / wl_t;
            double qz = fabs(m[2] - pp->s[2]) / wl_z;
            double q = qt > qz ? qt : qz;
            hv.v[i].inside = q <= 1.0;
            any_inside |= hv.v[i].inside;
            double mw = fabs(q - 1.0);
            if (mw < mwin) mwin = mw;
          }
          if (!any_inside && hv.n > 0) n_fb++;
        }
        for (int64_t i = 0; i < hv.n; ++i)
          if (hv.v[i].inside || !any_inside) {
            ochild ch = {c, hv.v[i].hit, pc->nhits + 1, pc->chi2 + hv.v[i].chi2};
            push_child(&cv, ch);
          }
        hv.n = 0;
        /* hole: the candidate crosses the layer without a hit */
        ochild hole = {c, -1, pc->nhits, pc->chi2};
        push_child(&cv, hole);
      }
      qsort(cv.v, (size_t)cv.n, sizeof(ochild), child_cmp);
      int keep = cv.n < N ? (int)cv.n : N;
      int lim = cv.n - 1 < N ? (int)cv.n - 1 : N;
      for (int i = 0; i < lim; ++i) {
        if (cv.v[i].nhits != cv.v[i + 1].nhits) continue;
        double den = cv.v[i].chi2 > 1.0 ? cv.v[i].chi2 : 1.0;
        double gap = fabs(cv.v[i + 1].chi2 - cv.v[i].chi2) / den;
        if (gap < mrank) mrank = gap;
      }
      for (int k = 0; k < keep; ++k) {
        ochild* ch = &cv.v[k];
        ocand* par = &cur[ch->parent];
        ocand* pp = &prop[ch->parent];
        ocand* nw = &nxt[k];
        memcpy(nw->hits, par->hits, sizeof(int32_t) * L);
        nw->nhits = ch->nhits;
        nw->chi2 = ch->chi2;
        nw->status = pp->status;
        memcpy(nw->s, pp->s, sizeof nw->s);
        memcpy(nw->C, pp->C, sizeof nw->C);
        if (ch->hit >= 0) {
          double c2;
          int32_t st = or_update_one(nw->s, nw->C, hit_pos + 3 * ch->hit, hit_cov + 9 * ch->hit, &c2, 0);
          if (st) nw->status = st;
          nw->hits[l] = (int32_t)ch->hit;
        }
      }
      ocand* tmp = cur;
      cur = nxt;
      nxt = tmp;
      nc = keep;
    }
    n_cands[si] = nc;
    for (int k = 0; k < N; ++k) {
      int32_t* ho = cand_hits + ((int64_t)si * N + k) * L;
      if (k < nc) {
        memcpy(ho, cur[k].hits, sizeof(int32_t) * L);
      } else {
        for (int l = 0; l < L; ++l) ho[l] = -1;
      }
      if (cand_chi2) cand_chi2[si * N + k] = k < nc ? cur[k].chi2 : 0.0;
      if (cand_nhits) cand_nhits[si * N + k] = k < nc ? cur[k].nhits : 0;
      if (cand_status) cand_status[si * N + k] = k < nc ? cur[k].status : 0;
    }
    if (best_state) memcpy(best_state + 6 * si, cur[0].s, sizeof cur[0].s);
    if (best_cov) memcpy(best_cov + 36 * si, cur[0].C, sizeof cur[0].C);
    if (margin_cut) margin_cut[si] = mcut;
    if (margin_rank) margin_rank[si] = mrank;
    if (hits_examined) hits_examined[si] = examined;
    if (margin_window) margin_window[si] = mwin;
    if (fallbacks) fallbacks[si] = n_fb;
  }
  for (int k = 0; k < N; ++k) {
    free(cur[k].hits);
    free(nxt[k].hits);
  }
  free(hv.v);
  free(mlp_r);
  free(cur);
  free(nxt);
  free(prop);
  free(cv.v);
  free(own_bins);
  free(own_perm);
  free(own_vmax);
  return 0;
}
