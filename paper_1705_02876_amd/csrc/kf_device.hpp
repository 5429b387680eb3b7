// kf_device.hpp -- register-resident Kalman-filter arithmetic for gfx950.
//
// One track per lane.  State s[6] = (x, y, z, px, py, pz); covariance c[21]
// packed lower triangle, k = i(i+1)/2 + j.  Everything stays in VGPRs: all
// index expressions below are compile-time constants after unrolling.  HBM
// always holds float32; the register type T of a kernel is float or double
// (gfx950 issues FP64 FMA at the rate of unpacked FP32 FMA), and Kalman
// updates compute in U = double in both cases.
//
// Helix propagation (the paper's core KF step, Sec. 2.1 / Sec. 3): with
// a = -q c bz and kappa = a / pT the transverse direction turns by
// phi = kappa t after transverse path t.  Writing tau = tan(phi / 2) and
// w = tau / kappa, the crossing condition |P(t)| = R becomes the quadratic
//     A w^2 + 2 au w - D / 2 = 0,  A = 2 (1 + kappa an) - kappa^2 D / 2,
// with au = P0.u, an = P0.n, D = R^2 - |P0|^2 (u = direction, n = left normal).
// Its smallest positive root gives the first crossing within half a turn with
// no 1/kappa or rho^2 terms, so stiff tracks keep full precision; sin and cos
// of phi follow from tau algebraically and only t = 2 atan(tau) / kappa needs
// a transcendental.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define KF_DEV __device__ __forceinline__

namespace kfd {

constexpr double kCLight = 0.299792458e-2;  // GeV / (T cm)
constexpr int kMaxLayers = 32;

enum : int32_t { ST_NO_CROSSING = 1, ST_OUT_OF_Z = 2, ST_NONFINITE = 4, ST_NOT_PD = 8, ST_STOPPED = 16 };

struct Geom {
  int32_t n_layers;
  float r[kMaxLayers];
  float z_half[kMaxLayers];
  float x_over_x0[kMaxLayers];
  float bz;
  float eloss_per_x0;
  float mass;
};

constexpr int tri(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

// precision-generic math.  The float versions use the hardware approximations
// (reciprocal, reciprocal square root, square root: about one ulp) instead of
// the correctly rounded software sequences; double stays IEEE.
KF_DEV float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
KF_DEV double rsqrt_t(double x) { return 1.0 / sqrt(x); }
KF_DEV float div_t(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
KF_DEV double div_t(double a, double b) { return a / b; }
KF_DEV float atan_t(float x) { return atanf(x); }
KF_DEV double atan_t(double x) { return atan(x); }
// natural logarithm from the hardware base-2 logarithm (about an ulp; the one use, the Highland width's
// logarithmic term, scales it by 0.038)
KF_DEV float log_t(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
KF_DEV double log_t(double x) { return log(x); }
// Reciprocal and reciprocal square root of a positive, finite, normal value: the
// hardware approximation refined by two Newton steps (each squares the relative
// error), which lands within a few ulp in double precision at a fraction of the
// cost of the correctly rounded sequences.  Used where the argument is known to
// be in that range (a determinant checked positive, a squared layer radius).
KF_DEV float rcp_pos(float x) { return __builtin_amdgcn_rcpf(x); }
KF_DEV double rcp_pos(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = fma(-x, y, 1.0);
  y = fma(y, e, y);
  e = fma(-x, y, 1.0);
  return fma(y, e, y);
}
KF_DEV float rsqrt_pos(float x) { return __builtin_amdgcn_rsqf(x); }
KF_DEV double rsqrt_pos(double x) {
  const double h = 0.5 * x;
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}
KF_DEV float sqrt_t(float x) { return __builtin_amdgcn_sqrtf(x); }
KF_DEV double sqrt_t(double x) { return sqrt(x); }
KF_DEV float abs_t(float x) { return fabsf(x); }
KF_DEV double abs_t(double x) { return fabs(x); }
KF_DEV float copysign_t(float a, float b) { return copysignf(a, b); }
KF_DEV double copysign_t(double a, double b) { return copysign(a, b); }

template <typename T>
KF_DEV bool finite_n(const T* v, int n) {
  T acc = T(0);
  for (int i = 0; i < n; ++i) acc += v[i] * T(0);
  return acc == T(0);
}

template <typename T>
KF_DEV bool finite6_21(const T s[6], const T c[21]) {
  T acc = T(0);
#pragma unroll
  for (int i = 0; i < 6; ++i) acc += s[i] * T(0);
#pragma unroll
  for (int i = 0; i < 21; ++i) acc += c[i] * T(0);
  return acc == T(0);  // any Inf/NaN turns the sum into NaN
}

// Result of a propagation: the Jacobian in its sparse form (23 non-zeros) and
// the new state.  Rows x, y, px, py have non-zeros in columns (x, y, px, py);
// row z in all six columns (with J[z][z] = 1); row pz is e_pz.
template <typename T>
struct Prop {
  T s[6];
  T jx[4], jy[4], jpx[4], jpy[4];  // columns (x, y, px, py)
  T jz[6];                         // columns (x, y, z, px, py, pz)
  T t;                             // transverse path length
};

// Helix crossing of radius R.  Returns status bits (0 on success).
template <typename T>
KF_DEV int32_t helix_to_r(const T s[6], T a, T R, T zh, Prop<T>& o) {
  const T x = s[0], y = s[1], z = s[2], px = s[3], py = s[4], pz = s[5];
  const T pt2 = px * px + py * py;
  const T ipt = rsqrt_t(pt2);
  const T ux = px * ipt, uy = py * ipt;
  const T au = x * ux + y * uy;
  const T an = y * ux - x * uy;
  const T D = R * R - (x * x + y * y);
  const T kap = a * ipt;
  const T A = T(2) * (T(1) + kap * an) - T(0.5) * kap * kap * D;
  const T disc = au * au + T(0.5) * A * D;
  if (!(disc >= T(0))) return ST_NO_CROSSING;
  const T sq = sqrt_t(disc);
  // numerically stable roots of A w^2 + 2 au w - D/2 = 0
  const T qq = -(au + copysign_t(sq, au));
  const T r1 = div_t(qq, A);
  const T r2 = div_t(T(-0.5) * D, qq);
  T w = T(INFINITY);
  if (r1 > T(0)) w = r1;
  if (r2 > T(0) && r2 < w) w = r2;
  if (!(w < T(INFINITY))) return ST_NO_CROSSING;
  const T tau = kap * w;
  const T tau2 = tau * tau;
  // atan(tau) / tau, series near 0
  const T small = sizeof(T) == 4 ? T(1e-3) : T(1e-5);
  const T at_over = (abs_t(tau) < small) ? (T(1) - tau2 * (T(1) / T(3)) + tau2 * tau2 * T(0.2)) : div_t(atan_t(tau), tau);
  const T t = T(2) * w * at_over;
  const T phi = kap * t;
  const T iden = div_t(T(1), T(1) + tau2);
  const T sn = T(2) * tau * iden;
  const T cs = (T(1) - tau2) * iden;
  const T S = T(2) * w * iden;         // sin(phi) / kappa
  const T Cc = T(2) * tau * w * iden;  // (1 - cos(phi)) / kappa
  const T xn = x + S * ux - Cc * uy;
  const T yn = y + S * uy + Cc * ux;
  const T zn = z + pz * ipt * t;
  if (zh > T(0) && abs_t(zn) > zh) return ST_OUT_OF_Z;
  const T pxn = px * cs - py * sn;
  const T pyn = py * cs + px * sn;
  o.s[0] = xn;
  o.s[1] = yn;
  o.s[2] = zn;
  o.s[3] = pxn;
  o.s[4] = pyn;
  o.s[5] = pz;
  o.t = t;
  // fixed-t Jacobian entries (sin(phi)/a = S/pT, (1-cos(phi))/a = Cc/pT)
  const T ipt2 = ipt * ipt;
  const T tp3 = t * ipt2 * ipt;  // t / pT^3
  const T fp2 = phi * ipt2;      // phi / pT^2
  const T Sp = S * ipt, Cp = Cc * ipt;
  const T a03 = Sp - pxn * px * tp3;
  const T a04 = -Cp - pxn * py * tp3;
  const T a13 = Cp - pyn * px * tp3;
  const T a14 = Sp - pyn * py * tp3;
  const T a23 = -pz * px * tp3;
  const T a24 = -pz * py * tp3;
  const T a25 = t * ipt;
  const T a33 = cs + pyn * px * fp2;
  const T a34 = -sn + pyn * py * fp2;
  const T a43 = sn - pxn * px * fp2;
  const T a44 = cs - pxn * py * fp2;
  // surface constraint: J = (I - v w^T) Jt
  const T v0 = pxn * ipt, v1 = pyn * ipt, v2 = pz * ipt, v3 = -kap * pyn, v4 = kap * pxn;
  const T iden2 = div_t(T(1), xn * v0 + yn * v1);
  const T w0 = xn * iden2, w1 = yn * iden2;
  const T w3 = w0 * a03 + w1 * a13;
  const T w4 = w0 * a04 + w1 * a14;
  o.jx[0] = T(1) - v0 * w0;
  o.jx[1] = -v0 * w1;
  o.jx[2] = a03 - v0 * w3;
  o.jx[3] = a04 - v0 * w4;
  o.jy[0] = -v1 * w0;
  o.jy[1] = T(1) - v1 * w1;
  o.jy[2] = a13 - v1 * w3;
  o.jy[3] = a14 - v1 * w4;
  o.jpx[0] = -v3 * w0;
  o.jpx[1] = -v3 * w1;
  o.jpx[2] = a33 - v3 * w3;
  o.jpx[3] = a34 - v3 * w4;
  o.jpy[0] = -v4 * w0;
  o.jpy[1] = -v4 * w1;
  o.jpy[2] = a43 - v4 * w3;
  o.jpy[3] = a44 - v4 * w4;
  o.jz[0] = -v2 * w0;
  o.jz[1] = -v2 * w1;
  o.jz[2] = T(1);
  o.jz[3] = a23 - v2 * w3;
  o.jz[4] = a24 - v2 * w4;
  o.jz[5] = a25;
  return 0;
}

// c <- J c J^T using the 23-non-zero structure.  132 + 89 FMA.
template <typename T>
KF_DEV void transport(T c[21], const Prop<T>& p) {
  T M[6][6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const T c0 = c[tri(0, k)], c1 = c[tri(1, k)], c2 = c[tri(2, k)];
    const T c3 = c[tri(3, k)], c4 = c[tri(4, k)], c5 = c[tri(5, k)];
    M[0][k] = p.jx[0] * c0 + p.jx[1] * c1 + p.jx[2] * c3 + p.jx[3] * c4;
    M[1][k] = p.jy[0] * c0 + p.jy[1] * c1 + p.jy[2] * c3 + p.jy[3] * c4;
    M[2][k] = p.jz[0] * c0 + p.jz[1] * c1 + c2 + p.jz[3] * c3 + p.jz[4] * c4 + p.jz[5] * c5;
    M[3][k] = p.jpx[0] * c0 + p.jpx[1] * c1 + p.jpx[2] * c3 + p.jpx[3] * c4;
    M[4][k] = p.jpy[0] * c0 + p.jpy[1] * c1 + p.jpy[2] * c3 + p.jpy[3] * c4;
    M[5][k] = c5;
  }
  // C'[i][l] = sum_k M[i][k] J[l][k], l <= i
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const T* Mi = M[i];
    c[tri(i, 0)] = p.jx[0] * Mi[0] + p.jx[1] * Mi[1] + p.jx[2] * Mi[3] + p.jx[3] * Mi[4];
    if (i >= 1) c[tri(i, 1)] = p.jy[0] * Mi[0] + p.jy[1] * Mi[1] + p.jy[2] * Mi[3] + p.jy[3] * Mi[4];
    if (i >= 2)
      c[tri(i, 2)] = p.jz[0] * Mi[0] + p.jz[1] * Mi[1] + Mi[2] + p.jz[3] * Mi[3] + p.jz[4] * Mi[4] + p.jz[5] * Mi[5];
    if (i >= 3) c[tri(i, 3)] = p.jpx[0] * Mi[0] + p.jpx[1] * Mi[1] + p.jpx[2] * Mi[3] + p.jpx[3] * Mi[4];
    if (i >= 4) c[tri(i, 4)] = p.jpy[0] * Mi[0] + p.jpy[1] * Mi[1] + p.jpy[2] * Mi[3] + p.jpy[3] * Mi[4];
    if (i >= 5) c[tri(i, 5)] = Mi[5];
  }
}

// Propagate + transport in place; on failure s and c are left unchanged.  A non-finite entry of the state or the
// covariance gives ST_NONFINITE.  Only the state is checked before the crossing: a non-finite covariance entry
// reaches the transported (z, z) entry (every entry of c enters row z of J c with a weight, and every entry of that
// row enters (z, z)), so the check of the result finds it, and a failed crossing checks c before it reports.
template <typename T>
KF_DEV int32_t propagate(T s[6], T c[21], T a, T R, T zh) {
  if (!finite_n(s, 6)) return ST_NONFINITE;
  Prop<T> p;
  int32_t st = helix_to_r(s, a, R, zh, p);
  if (st) return finite_n(c, 21) ? st : ST_NONFINITE;
  T cn[21];
#pragma unroll
  for (int k = 0; k < 21; ++k) cn[k] = c[k];
  transport(cn, p);
  if (!finite6_21(p.s, cn)) return ST_NONFINITE;
#pragma unroll
  for (int k = 0; k < 6; ++k) s[k] = p.s[k];
#pragma unroll
  for (int k = 0; k < 21; ++k) c[k] = cn[k];
  return 0;
}

// Propagate + transport in place for callers that keep the state themselves: the same results as propagate on
// success, unspecified s and c on failure (no copy of the covariance is made).
template <typename T>
KF_DEV int32_t propagate_inplace(T s[6], T c[21], T a, T R, T zh) {
  if (!finite_n(s, 6)) return ST_NONFINITE;
  Prop<T> p;
  const int32_t st = helix_to_r(s, a, R, zh, p);
  if (st) return finite_n(c, 21) ? st : ST_NONFINITE;
  transport(c, p);
#pragma unroll
  for (int k = 0; k < 6; ++k) s[k] = p.s[k];
  return finite6_21(s, c) ? 0 : ST_NONFINITE;
}

// Thin scatterer (multiple scattering, Highland width, and mean energy loss)
// for a track sitting on a layer of normal thickness xx0 radiation lengths.
// f_out (nullable) receives the momentum ratio p'/p of the energy loss.
template <typename T>
KF_DEV int32_t material(T s[6], T c[21], T xx0, T eloss, T mass, T* f_out = nullptr) {
  if (f_out) *f_out = T(1);
  if (!(xx0 > T(0))) return 0;
  const T p2 = s[3] * s[3] + s[4] * s[4] + s[5] * s[5];
  const T ip = rsqrt_t(p2);
  const T p = p2 * ip;
  const T u0 = s[3] * ip, u1 = s[4] * ip, u2 = s[5] * ip;
  const T ir = rsqrt_t(s[0] * s[0] + s[1] * s[1]);
  const T cospsi = abs_t((u0 * s[0] + u1 * s[1]) * ir);
  const T tt = div_t(xx0, cospsi);
  const T m2 = mass * mass;
  const T E = sqrt_t(p2 + m2);
  const T beta = div_t(p, E);
  const T th0 = div_t(T(0.0136), beta * p) * sqrt_t(tt) * (T(1) + T(0.038) * log_t(div_t(tt, beta * beta)));
  const T E2 = E - eloss * tt;
  if (!(E2 > mass)) return ST_STOPPED;
  const T pn = sqrt_t((E2 - mass) * (E2 + mass));
  const T f = div_t(pn, p);
  if (f_out) *f_out = f;
#pragma unroll
  for (int i = 3; i < 6; ++i) s[i] *= f;
#pragma unroll
  for (int i = 3; i < 6; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) c[tri(i, j)] *= f;
#pragma unroll
    for (int j = 3; j <= i; ++j) c[tri(i, j)] *= f * f;
  }
  const T k = pn * pn * th0 * th0;
  const T u[3] = {u0, u1, u2};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) c[tri(i + 3, j + 3)] += k * ((i == j ? T(1) : T(0)) - u[i] * u[j]);
  return 0;
}

// Inverse of a symmetric 3x3 given by its packed entries (00, 10, 11, 20, 21,
// 22), by cofactors; returns false unless positive definite (leading minors).
template <typename T>
KF_DEV bool inv3_packed(const T r[6], T ri[6]) {
  const T a = r[0], b = r[1], d = r[2], e = r[3], f = r[4], g = r[5];
  const T i00 = d * g - f * f;
  const T i10 = e * f - b * g;
  const T i20 = b * f - d * e;
  const T det = a * i00 + b * i10 + e * i20;
  const T m2 = a * d - b * b;
  if (!(a > T(0)) || !(m2 > T(0)) || !(det > T(0))) return false;
  const T id = rcp_pos(det);
  ri[0] = i00 * id;
  ri[1] = i10 * id;
  ri[2] = (a * g - e * e) * id;
  ri[3] = i20 * id;
  ri[4] = (b * e - a * f) * id;
  ri[5] = m2 * id;
  return true;
}

// General Kalman update with the hit (m, v) in global coordinates, computed in
// precision U: r = m - H x, R = H C H^T + V, chi2 = r^T R^-1 r and, with
// A, B, D the position, cross and momentum blocks of C, the algebraically
// identical stable forms C_pos'' = A R^-1 V, C_mom,pos'' = B R^-1 V,
// C_mom'' = D - B R^-1 B^T of C - K H C (no A - A R^-1 A cancellation under
// vague priors).  Makes no assumption on C.
template <typename T, typename U>
KF_DEV int32_t update_global(T s[6], T c[21], const float m[3], const float v[6], T& chi2_out) {
  const U rr[6] = {U(c[0]) + U(v[0]), U(c[1]) + U(v[1]), U(c[2]) + U(v[2]),
                   U(c[3]) + U(v[3]), U(c[4]) + U(v[4]), U(c[5]) + U(v[5])};
  U ri[6];
  if (!inv3_packed<U>(rr, ri)) return ST_NOT_PD;
  const U Ri[3][3] = {{ri[0], ri[1], ri[3]}, {ri[1], ri[2], ri[4]}, {ri[3], ri[4], ri[5]}};
  const U r[3] = {U(m[0]) - U(s[0]), U(m[1]) - U(s[1]), U(m[2]) - U(s[2])};
  U q[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) q[i] = Ri[i][0] * r[0] + Ri[i][1] * r[1] + Ri[i][2] * r[2];
  const U chi2 = r[0] * q[0] + r[1] * q[1] + r[2] * q[2];
  const U V[3][3] = {{U(v[0]), U(v[1]), U(v[3])}, {U(v[1]), U(v[2]), U(v[4])}, {U(v[3]), U(v[4]), U(v[5])}};
  U M[3][3];  // R^-1 V
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[i][j] = Ri[i][0] * V[0][j] + Ri[i][1] * V[1][j] + Ri[i][2] * V[2][j];
  U A[3][3], B[3][3], D[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      A[i][j] = U(c[tri(i, j)]);
      B[i][j] = U(c[tri(i + 3, j)]);
      D[i][j] = U(c[tri(i + 3, j + 3)]);
    }
  U G[3][3];  // B R^-1
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) G[i][j] = B[i][0] * Ri[0][j] + B[i][1] * Ri[1][j] + B[i][2] * Ri[2][j];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    s[i] = static_cast<T>(U(s[i]) + (A[i][0] * q[0] + A[i][1] * q[1] + A[i][2] * q[2]));
    s[i + 3] = static_cast<T>(U(s[i + 3]) + (B[i][0] * q[0] + B[i][1] * q[1] + B[i][2] * q[2]));
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j)
      c[tri(i, j)] = static_cast<T>(A[i][0] * M[0][j] + A[i][1] * M[1][j] + A[i][2] * M[2][j]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      c[tri(i + 3, j)] = static_cast<T>(B[i][0] * M[0][j] + B[i][1] * M[1][j] + B[i][2] * M[2][j]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j)
      c[tri(i + 3, j + 3)] = static_cast<T>(D[i][j] - (G[i][0] * B[j][0] + G[i][1] * B[j][1] + G[i][2] * B[j][2]));
  chi2_out = static_cast<T>(chi2);
  if (!finite6_21(s, c)) return ST_NONFINITE;
  return 0;
}

// ---------------------------------------------------------------------------
// Measurements on a layer, in the frame of the prediction.
//
// After the surface-constrained transport the position block A of the
// predicted covariance has an exact null along the radial unit vector n at the
// predicted point (the crossing stays on the cylinder).  In the orthonormal
// frame (n, t, z), t = (-n_y, n_x, 0), the residual covariance R = A + V is
//     R_loc = V_loc + [[0, 0, 0], [0, A_tt, A_tz], [0, A_tz, A_zz]],
// which is the textbook R rotated, with A's radial row set to its exact value
// 0.  Computing it this way keeps the hit's radial variance intact even when
// the stored A is huge (a vague seed: rounding noise of A along n would swamp
// V_nn in the global frame).  chi2 and the gain are rotation invariant, so
// the results equal the global-frame formulas.
template <typename T>
struct LocalPred {
  T nx, ny, tx, ty;  // radial and tangential unit vectors at the prediction
  T att, atz, azz;   // A in the (t, z) plane
};

template <typename T>
KF_DEV LocalPred<T> local_pred(const T s[6], const T c[21]) {
  LocalPred<T> L;
  const T ir = rsqrt_t(s[0] * s[0] + s[1] * s[1]);
  L.nx = s[0] * ir;
  L.ny = s[1] * ir;
  L.tx = -L.ny;
  L.ty = L.nx;
  L.att = L.tx * L.tx * c[0] + T(2) * L.tx * L.ty * c[1] + L.ty * L.ty * c[2];
  L.atz = L.tx * c[3] + L.ty * c[4];
  L.azz = c[5];
  return L;
}

// R_loc (packed nn, nt, tt, nz, tz, zz) from the hit covariance v (packed
// global xx, yx, yy, zx, zy, zz) and the predicted (t, z) block.
template <typename T>
KF_DEV void r_local(T nx, T ny, T tx, T ty, T att, T atz, T azz, const float v[6], T r[6]) {
  const T vxx = T(v[0]), vyx = T(v[1]), vyy = T(v[2]), vzx = T(v[3]), vzy = T(v[4]), vzz = T(v[5]);
  r[0] = nx * nx * vxx + T(2) * nx * ny * vyx + ny * ny * vyy;
  r[1] = nx * tx * vxx + (nx * ty + ny * tx) * vyx + ny * ty * vyy;
  r[2] = tx * tx * vxx + T(2) * tx * ty * vyx + ty * ty * vyy + att;
  r[3] = nx * vzx + ny * vzy;
  r[4] = tx * vzx + ty * vzy + atz;
  r[5] = vzz + azz;
}

// chi2 of hit (m, v) against a prediction on its layer.
template <typename T>
KF_DEV int32_t chi2_on_layer(const T s[6], const LocalPred<T>& L, const float m[3], const float v[6], T& chi2) {
  T r[6], ri[6];
  r_local<T>(L.nx, L.ny, L.tx, L.ty, L.att, L.atz, L.azz, v, r);
  if (!inv3_packed<T>(r, ri)) return ST_NOT_PD;
  const T dx = T(m[0]) - s[0], dy = T(m[1]) - s[1], dz = T(m[2]) - s[2];
  const T rn = L.nx * dx + L.ny * dy, rt = L.tx * dx + L.ty * dy;
  const T q0 = ri[0] * rn + ri[1] * rt + ri[3] * dz;
  const T q1 = ri[1] * rn + ri[2] * rt + ri[4] * dz;
  const T q2 = ri[3] * rn + ri[4] * rt + ri[5] * dz;
  chi2 = rn * q0 + rt * q1 + dz * q2;
  return 0;
}

// Kalman update of a prediction on its layer, in the prediction's frame and in
// precision U.  With U_c = C H^T Q (6x3, Q = [n t z]; its n column is exactly 0):
//   x'' = x' + U_c R_loc^-1 r_loc,
//   C''_pos = (A Q) R_loc^-1 V_loc Q^T,  C''_mom,pos = (B Q) R_loc^-1 V_loc Q^T,
//   C''_mom = D - (B Q) R_loc^-1 (B Q)^T,
// the stable block forms of C - K H C written in the local frame.
template <typename T, typename U>
KF_DEV int32_t update_on_layer(T s[6], T c[21], const float m[3], const float v[6], T& chi2_out) {
  const U x = U(s[0]), y = U(s[1]);
  const U ir = rsqrt_pos(x * x + y * y);
  const U nx = x * ir, ny = y * ir, tx = -ny, ty = nx;
  U ut[6], uz[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    ut[i] = U(c[tri(i, 0)]) * tx + U(c[tri(i, 1)]) * ty;
    uz[i] = U(c[tri(i, 2)]);
  }
  const U att = tx * ut[0] + ty * ut[1];
  const U atz = uz[0] * tx + uz[1] * ty;
  const U azz = uz[2];
  U r[6], ri[6];
  r_local<U>(nx, ny, tx, ty, att, atz, azz, v, r);
  if (!inv3_packed<U>(r, ri)) return ST_NOT_PD;
  const U dx = U(m[0]) - x, dy = U(m[1]) - y, dz = U(m[2]) - U(s[2]);
  const U rl[3] = {nx * dx + ny * dy, tx * dx + ty * dy, dz};
  const U Ri[3][3] = {{ri[0], ri[1], ri[3]}, {ri[1], ri[2], ri[4]}, {ri[3], ri[4], ri[5]}};
  U q[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) q[i] = Ri[i][0] * rl[0] + Ri[i][1] * rl[1] + Ri[i][2] * rl[2];
  const U chi2 = rl[0] * q[0] + rl[1] * q[1] + rl[2] * q[2];
  // V_loc: R_loc without the A part
  const U Vl[3][3] = {{r[0], r[1], r[3]}, {r[1], r[2] - att, r[4] - atz}, {r[3], r[4] - atz, r[5] - azz}};
  // t and z rows of R_loc^-1 V_loc (the n column of U_c is 0)
  U Ml[2][3];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int j = 0; j < 3; ++j) Ml[a][j] = Ri[a + 1][0] * Vl[0][j] + Ri[a + 1][1] * Vl[1][j] + Ri[a + 1][2] * Vl[2][j];
  const U Q[3][3] = {{nx, tx, U(0)}, {ny, ty, U(0)}, {U(0), U(0), U(1)}};  // columns n, t, z
  U P[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) P[i][k] = ut[i] * Ml[0][k] + uz[i] * Ml[1][k];
  U dn[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) dn[i] = ut[i] * q[1] + uz[i] * q[2];
  U Dn[6];
  {
    int k = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) {
        const U gi1 = ut[3 + i] * Ri[1][1] + uz[3 + i] * Ri[2][1];
        const U gi2 = ut[3 + i] * Ri[1][2] + uz[3 + i] * Ri[2][2];
        Dn[k++] = U(c[tri(3 + i, 3 + j)]) - (gi1 * ut[3 + j] + gi2 * uz[3 + j]);
      }
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) s[i] = static_cast<T>(U(s[i]) + dn[i]);
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 3 && j <= i; ++j)
      c[tri(i, j)] = static_cast<T>(P[i][0] * Q[j][0] + P[i][1] * Q[j][1] + P[i][2] * Q[j][2]);
  {
    int k = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) c[tri(3 + i, 3 + j)] = static_cast<T>(Dn[k++]);
  }
  chi2_out = static_cast<T>(chi2);
  if (!finite6_21(s, c)) return ST_NONFINITE;
  return 0;
}

// Features of a prediction for the learned search window, in this order:
// q/pT, cot(theta), z/z_half, sin of the angle between the transverse momentum
// and the radial direction, r_from/100, r_to/100, and the logs of the
// predicted position's tangential and z standard deviations (cm).
// ---- smoother: one Rauch-Tung-Striebel backward step,
//   K = Cf F^T Cp^+,  xs_l = xf_l + K (xs_{l+1} - xp_{l+1}),  Cs_l = Cf_l + K (Cs_{l+1} - Cp_{l+1}) K^T,
// with Cp^+ = P^T (P Cp P^T)^-1 P the pseudo-inverse on the cylinder (P: the orthonormal rows tangent, z, px,
// py, pz) and F = J diag(1, 1, 1, f, f, f) the derivative of the filter's step from layer l to l+1.

// y <- L^-1 y for the packed lower-triangular 5x5 factor L (row-major lower
// triangle, tri(i, j)) with its reciprocal diagonal id.
template <typename U>
KF_DEV void fwd_subst5(const U Lf[15], const U id[5], U y[5]) {
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    U v = y[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= Lf[tri(i, k)] * y[k];
    y[i] = v * id[i];
  }
}

// One backward step of one track (precision U for the gain).  xs, cs hold the
// smoothed state of layer l+1 on entry and of layer l on exit; xf, cf the
// filtered state of layer l.  Returns 0 or a status bit (ST_NOT_PD: the
// prediction's surface block is not positive definite).
template <typename T, typename U>
KF_DEV int32_t rts_step(const float xf[6], const float cf[21], T a, const Geom& g, int l,
                                            float xs[6], float cs[21]) {
  T xp[6], cp[21];
#pragma unroll
  for (int k = 0; k < 6; ++k) xp[k] = T(xf[k]);
#pragma unroll
  for (int k = 0; k < 21; ++k) cp[k] = T(cf[k]);
  // (in single precision these are the forward pass's own values and cannot fail; a double-precision
  // filter reads back float32 rows, whose step could in principle fail where the filter's did not)
  T f;
  if (int32_t e = material(xp, cp, T(g.x_over_x0[l]), T(g.eloss_per_x0), T(g.mass), &f)) return e;
  Prop<T> pr;
  if (int32_t e = helix_to_r(xp, a, T(g.r[l + 1]), T(0), pr)) return e;
  transport(cp, pr);
  // surface frame at the prediction
  const U px0 = U(pr.s[0]), py0 = U(pr.s[1]);
  const U ir = rsqrt_pos(px0 * px0 + py0 * py0);
  const U tx = -py0 * ir, ty = px0 * ir;
  const U fu = U(f);
  // rows of P J D over the columns (x, y, z, px, py, pz)
  const U Rt[6] = {tx * U(pr.jx[0]) + ty * U(pr.jy[0]), tx * U(pr.jx[1]) + ty * U(pr.jy[1]), U(0),
                   (tx * U(pr.jx[2]) + ty * U(pr.jy[2])) * fu, (tx * U(pr.jx[3]) + ty * U(pr.jy[3])) * fu, U(0)};
  const U Rz[6] = {U(pr.jz[0]), U(pr.jz[1]), U(1), U(pr.jz[3]) * fu, U(pr.jz[4]) * fu, U(pr.jz[5]) * fu};
  const U Rx[6] = {U(pr.jpx[0]), U(pr.jpx[1]), U(0), U(pr.jpx[2]) * fu, U(pr.jpx[3]) * fu, U(0)};
  const U Ry[6] = {U(pr.jpy[0]), U(pr.jpy[1]), U(0), U(pr.jpy[2]) * fu, U(pr.jpy[3]) * fu, U(0)};
  // S = P Cp P^T and its Cholesky factor
  U Sm[15];
  {
    const U c00 = U(cp[0]), c10 = U(cp[1]), c11 = U(cp[2]);
    Sm[0] = tx * tx * c00 + U(2) * tx * ty * c10 + ty * ty * c11;
#pragma unroll
    for (int r = 1; r < 5; ++r) {
      Sm[tri(r, 0)] = tx * U(cp[tri(r + 1, 0)]) + ty * U(cp[tri(r + 1, 1)]);
#pragma unroll
      for (int q = 1; q <= r; ++q) Sm[tri(r, q)] = U(cp[tri(r + 1, q + 1)]);
    }
  }
  U Lf[15], id[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    U d = Sm[tri(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= Lf[tri(j, k)] * Lf[tri(j, k)];
    if (!(d > U(0))) return ST_NOT_PD;
    const U is = rsqrt_pos(d);
    Lf[tri(j, j)] = d * is;
    id[j] = is;
#pragma unroll
    for (int i = j + 1; i < 5; ++i) {
      U v = Sm[tri(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= Lf[tri(i, k)] * Lf[tri(j, k)];
      Lf[tri(i, j)] = v * is;
    }
  }
  // v = L^-1 P (xs - xp)
  U v[5];
  v[0] = tx * (U(xs[0]) - U(pr.s[0])) + ty * (U(xs[1]) - U(pr.s[1]));
#pragma unroll
  for (int k = 1; k < 5; ++k) v[k] = U(xs[k + 1]) - U(pr.s[k + 1]);
  fwd_subst5(Lf, id, v);
  // N = L^-1 P (Cs - Cp) P^T L^-T
  U N[15];
  {
    U Md[21];
#pragma unroll
    for (int k = 0; k < 21; ++k) Md[k] = U(cs[k]) - U(cp[k]);
    U M5[5][5];
    M5[0][0] = tx * tx * Md[0] + U(2) * tx * ty * Md[1] + ty * ty * Md[2];
#pragma unroll
    for (int r = 1; r < 5; ++r) {
      M5[r][0] = M5[0][r] = tx * Md[tri(r + 1, 0)] + ty * Md[tri(r + 1, 1)];
#pragma unroll
      for (int q = 1; q <= r; ++q) M5[r][q] = M5[q][r] = Md[tri(r + 1, q + 1)];
    }
    // Y = L^-1 M5 column by column, then N = L^-1 Y^T (symmetric)
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      U y[5] = {M5[0][c], M5[1][c], M5[2][c], M5[3][c], M5[4][c]};
      fwd_subst5(Lf, id, y);
#pragma unroll
      for (int r = 0; r < 5; ++r) M5[r][c] = y[r];
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      U y[5] = {M5[c][0], M5[c][1], M5[c][2], M5[c][3], M5[c][4]};
      fwd_subst5(Lf, id, y);
#pragma unroll
      for (int r = c; r < 5; ++r) N[tri(r, c)] = y[r];
    }
  }
  // W = B L^-T, row i = L^-1 (P F Cf)[.][i]; then the smoothed state and covariance
  U W[6][5];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    U cfi[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) cfi[k] = U(cf[i >= k ? tri(i, k) : tri(k, i)]);
    U b[5] = {U(0), U(0), U(0), U(0), cfi[5] * fu};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      b[0] += cfi[k] * Rt[k];
      b[1] += cfi[k] * Rz[k];
      b[2] += cfi[k] * Rx[k];
      b[3] += cfi[k] * Ry[k];
    }
    fwd_subst5(Lf, id, b);
#pragma unroll
    for (int r = 0; r < 5; ++r) W[i][r] = b[r];
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const U dx = W[i][0] * v[0] + W[i][1] * v[1] + W[i][2] * v[2] + W[i][3] * v[3] + W[i][4] * v[4];
    xs[i] = float(U(xf[i]) + dx);
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    U wn[5];  // (W N)[i]
#pragma unroll
    for (int r = 0; r < 5; ++r) {
      U acc = U(0);
#pragma unroll
      for (int q = 0; q < 5; ++q) acc += W[i][q] * N[r >= q ? tri(r, q) : tri(q, r)];
      wn[r] = acc;
    }
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      const U d = wn[0] * W[j][0] + wn[1] * W[j][1] + wn[2] * W[j][2] + wn[3] * W[j][3] + wn[4] * W[j][4];
      cs[tri(i, j)] = float(U(cf[tri(i, j)]) + d);
    }
  }
  return 0;
}

template <typename T>
__device__ __forceinline__ void window_features(const T s[6], const T c[21], float q, float r_from, float r_to,
                                                float zh, float f[8]) {
  const float x = float(s[0]), y = float(s[1]), z = float(s[2]), px = float(s[3]), py = float(s[4]),
              pz = float(s[5]);
  const float ipt = __frsqrt_rn(px * px + py * py);
  const float ir = __frsqrt_rn(x * x + y * y);
  const float tx = -y * ir, ty = x * ir;  // tangential unit vector
  const float ctt = tx * tx * float(c[0]) + 2.f * tx * ty * float(c[1]) + ty * ty * float(c[2]);
  f[0] = q * ipt;
  f[1] = pz * ipt;
  f[2] = z / zh;
  f[3] = (x * py - y * px) * ipt * ir;
  f[4] = r_from * 0.01f;
  f[5] = r_to * 0.01f;
  f[6] = 0.5f * logf(fmaxf(ctt, 1e-30f));
  f[7] = 0.5f * logf(fmaxf(float(c[5]), 1e-30f));
}

}  // namespace kfd
