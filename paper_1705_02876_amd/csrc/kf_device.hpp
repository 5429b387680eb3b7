// kf_device.hpp -- register-resident FP32 Kalman-filter arithmetic for gfx950.
//
// One track per lane.  State s[6] = (x, y, z, px, py, pz); covariance c[21]
// packed lower triangle, k = i(i+1)/2 + j.  Everything stays in VGPRs: all
// index expressions below are compile-time constants after unrolling.
//
// Helix propagation (the paper's core KF step, Sec. 2.1 / Sec. 3): with
// a = -q c bz and kappa = a / pT the transverse direction turns by
// phi = kappa t after transverse path t.  Writing tau = tan(phi / 2) and
// w = tau / kappa, the crossing condition |P(t)| = R becomes the quadratic
//     A w^2 + 2 au w - D / 2 = 0,  A = 2 (1 + kappa an) - kappa^2 D / 2,
// with au = P0.u, an = P0.n, D = R^2 - |P0|^2 (u = direction, n = left normal).
// Its smallest positive root gives the first crossing within half a turn with
// no 1/kappa or rho^2 terms, so stiff tracks keep full FP32 precision; sin and
// cos of phi follow from tau algebraically and only t = 2 atan(tau) / kappa
// needs a transcendental.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define KF_DEV __device__ __forceinline__

namespace kfd {

constexpr float kCLight = 0.299792458e-2f;  // GeV / (T cm)
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

KF_DEV bool finite6_21(const float s[6], const float c[21]) {
  float acc = 0.f;
#pragma unroll
  for (int i = 0; i < 6; ++i) acc += s[i] * 0.f;
#pragma unroll
  for (int i = 0; i < 21; ++i) acc += c[i] * 0.f;
  return acc == 0.f;  // any Inf/NaN turns the sum into NaN
}

// Result of a propagation: the Jacobian in its sparse form (23 non-zeros) and
// the new state.  Rows x, y, px, py have non-zeros in columns (x, y, px, py);
// row z in all six columns (with J[z][z] = 1); row pz is e_pz.
struct Prop {
  float s[6];
  float jx[4], jy[4], jpx[4], jpy[4];  // columns (x, y, px, py)
  float jz[6];                         // columns (x, y, z, px, py, pz)
  float t;                             // transverse path length
};

// Helix crossing of radius R.  Returns status bits (0 on success).
KF_DEV int32_t helix_to_r(const float s[6], float a, float R, float zh, Prop& o) {
  const float x = s[0], y = s[1], z = s[2], px = s[3], py = s[4], pz = s[5];
  const float pt2 = px * px + py * py;
  const float ipt = __frsqrt_rn(pt2);
  const float ux = px * ipt, uy = py * ipt;
  const float au = x * ux + y * uy;
  const float an = y * ux - x * uy;
  const float D = R * R - (x * x + y * y);
  const float kap = a * ipt;
  const float A = 2.f * (1.f + kap * an) - 0.5f * kap * kap * D;
  const float disc = au * au + 0.5f * A * D;
  if (!(disc >= 0.f)) return ST_NO_CROSSING;
  const float sq = sqrtf(disc);
  // numerically stable roots of A w^2 + 2 au w - D/2 = 0
  const float qq = -(au + copysignf(sq, au));
  const float r1 = qq / A;
  const float r2 = (-0.5f * D) / qq;
  float w = INFINITY;
  if (r1 > 0.f) w = r1;
  if (r2 > 0.f && r2 < w) w = r2;
  if (!(w < INFINITY)) return ST_NO_CROSSING;
  const float tau = kap * w;
  const float tau2 = tau * tau;
  // atan(tau) / tau, series near 0
  float at_over = (fabsf(tau) < 1e-3f) ? (1.f - tau2 * (1.f / 3.f)) : (atanf(tau) / tau);
  const float t = 2.f * w * at_over;
  const float phi = kap * t;
  const float iden = 1.f / (1.f + tau2);
  const float sn = 2.f * tau * iden;
  const float cs = (1.f - tau2) * iden;
  const float S = 2.f * w * iden;         // sin(phi) / kappa
  const float Cc = 2.f * tau * w * iden;  // (1 - cos(phi)) / kappa
  const float xn = x + S * ux - Cc * uy;
  const float yn = y + S * uy + Cc * ux;
  const float zn = z + pz * ipt * t;
  if (zh > 0.f && fabsf(zn) > zh) return ST_OUT_OF_Z;
  const float pxn = px * cs - py * sn;
  const float pyn = py * cs + px * sn;
  o.s[0] = xn;
  o.s[1] = yn;
  o.s[2] = zn;
  o.s[3] = pxn;
  o.s[4] = pyn;
  o.s[5] = pz;
  o.t = t;
  // fixed-t Jacobian entries (sin(phi)/a = S/pT, (1-cos(phi))/a = Cc/pT)
  const float ipt2 = ipt * ipt;
  const float tp3 = t * ipt2 * ipt;  // t / pT^3
  const float fp2 = phi * ipt2;      // phi / pT^2
  const float Sp = S * ipt, Cp = Cc * ipt;
  const float a03 = Sp - pxn * px * tp3;
  const float a04 = -Cp - pxn * py * tp3;
  const float a13 = Cp - pyn * px * tp3;
  const float a14 = Sp - pyn * py * tp3;
  const float a23 = -pz * px * tp3;
  const float a24 = -pz * py * tp3;
  const float a25 = t * ipt;
  const float a33 = cs + pyn * px * fp2;
  const float a34 = -sn + pyn * py * fp2;
  const float a43 = sn - pxn * px * fp2;
  const float a44 = cs - pxn * py * fp2;
  // surface constraint: J = (I - v w^T) Jt
  const float v0 = pxn * ipt, v1 = pyn * ipt, v2 = pz * ipt, v3 = -kap * pyn, v4 = kap * pxn;
  const float iden2 = 1.f / (xn * v0 + yn * v1);
  const float w0 = xn * iden2, w1 = yn * iden2;
  const float w3 = w0 * a03 + w1 * a13;
  const float w4 = w0 * a04 + w1 * a14;
  o.jx[0] = 1.f - v0 * w0;
  o.jx[1] = -v0 * w1;
  o.jx[2] = a03 - v0 * w3;
  o.jx[3] = a04 - v0 * w4;
  o.jy[0] = -v1 * w0;
  o.jy[1] = 1.f - v1 * w1;
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
  o.jz[2] = 1.f;
  o.jz[3] = a23 - v2 * w3;
  o.jz[4] = a24 - v2 * w4;
  o.jz[5] = a25;
  return 0;
}

// c <- J c J^T using the 23-non-zero structure.  132 + 89 FMA.
KF_DEV void transport(float c[21], const Prop& p) {
  float T[6][6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const float c0 = c[tri(0, k)], c1 = c[tri(1, k)], c2 = c[tri(2, k)];
    const float c3 = c[tri(3, k)], c4 = c[tri(4, k)], c5 = c[tri(5, k)];
    T[0][k] = p.jx[0] * c0 + p.jx[1] * c1 + p.jx[2] * c3 + p.jx[3] * c4;
    T[1][k] = p.jy[0] * c0 + p.jy[1] * c1 + p.jy[2] * c3 + p.jy[3] * c4;
    T[2][k] = p.jz[0] * c0 + p.jz[1] * c1 + c2 + p.jz[3] * c3 + p.jz[4] * c4 + p.jz[5] * c5;
    T[3][k] = p.jpx[0] * c0 + p.jpx[1] * c1 + p.jpx[2] * c3 + p.jpx[3] * c4;
    T[4][k] = p.jpy[0] * c0 + p.jpy[1] * c1 + p.jpy[2] * c3 + p.jpy[3] * c4;
    T[5][k] = c5;
  }
  // C'[i][l] = sum_k T[i][k] J[l][k], l <= i
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const float* Ti = T[i];
    c[tri(i, 0)] = p.jx[0] * Ti[0] + p.jx[1] * Ti[1] + p.jx[2] * Ti[3] + p.jx[3] * Ti[4];
    if (i >= 1) c[tri(i, 1)] = p.jy[0] * Ti[0] + p.jy[1] * Ti[1] + p.jy[2] * Ti[3] + p.jy[3] * Ti[4];
    if (i >= 2)
      c[tri(i, 2)] = p.jz[0] * Ti[0] + p.jz[1] * Ti[1] + Ti[2] + p.jz[3] * Ti[3] + p.jz[4] * Ti[4] + p.jz[5] * Ti[5];
    if (i >= 3) c[tri(i, 3)] = p.jpx[0] * Ti[0] + p.jpx[1] * Ti[1] + p.jpx[2] * Ti[3] + p.jpx[3] * Ti[4];
    if (i >= 4) c[tri(i, 4)] = p.jpy[0] * Ti[0] + p.jpy[1] * Ti[1] + p.jpy[2] * Ti[3] + p.jpy[3] * Ti[4];
    if (i >= 5) c[tri(i, 5)] = Ti[5];
  }
}

// Propagate + transport in place; on failure s and c are left unchanged.
KF_DEV int32_t propagate(float s[6], float c[21], float a, float R, float zh) {
  if (!finite6_21(s, c)) return ST_NONFINITE;
  Prop p;
  int32_t st = helix_to_r(s, a, R, zh, p);
  if (st) return st;
  float cn[21];
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

// Thin scatterer (multiple scattering, Highland width, and mean energy loss)
// for a track sitting on a layer of normal thickness xx0 radiation lengths.
KF_DEV int32_t material(float s[6], float c[21], float xx0, float eloss, float mass) {
  if (!(xx0 > 0.f)) return 0;
  const float p2 = s[3] * s[3] + s[4] * s[4] + s[5] * s[5];
  const float ip = __frsqrt_rn(p2);
  const float p = p2 * ip;
  const float u0 = s[3] * ip, u1 = s[4] * ip, u2 = s[5] * ip;
  const float ir = __frsqrt_rn(s[0] * s[0] + s[1] * s[1]);
  const float cospsi = fabsf((u0 * s[0] + u1 * s[1]) * ir);
  const float tt = xx0 / cospsi;
  const float m2 = mass * mass;
  const float E = sqrtf(p2 + m2);
  const float beta = p / E;
  const float th0 = 0.0136f / (beta * p) * sqrtf(tt) * (1.f + 0.038f * logf(tt / (beta * beta)));
  const float E2 = E - eloss * tt;
  if (!(E2 > mass)) return ST_STOPPED;
  const float pn = sqrtf((E2 - mass) * (E2 + mass));
  const float f = pn / p;
#pragma unroll
  for (int i = 3; i < 6; ++i) s[i] *= f;
#pragma unroll
  for (int i = 3; i < 6; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) c[tri(i, j)] *= f;
#pragma unroll
    for (int j = 3; j <= i; ++j) c[tri(i, j)] *= f * f;
  }
  const float k = pn * pn * th0 * th0;
  const float u[3] = {u0, u1, u2};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) c[tri(i + 3, j + 3)] += k * ((i == j ? 1.f : 0.f) - u[i] * u[j]);
  return 0;
}

// Residual covariance R = C_pos + V, its inverse (symmetric, packed 6) and
// chi2 of the residual r = m - x.  Returns ST_NOT_PD if R is not positive
// definite (leading minors).
KF_DEV int32_t chi2_of(const float s[6], const float c[21], const float m[3], const float v[6], float ri[6],
                       float r[3], float& chi2) {
  const float a = c[0] + v[0], b = c[1] + v[1], d = c[2] + v[2];
  const float e = c[3] + v[3], f = c[4] + v[4], g = c[5] + v[5];
  // R = [[a, b, e], [b, d, f], [e, f, g]]
  const float i00 = d * g - f * f;
  const float i10 = e * f - b * g;
  const float i20 = b * f - d * e;
  const float det = a * i00 + b * i10 + e * i20;
  const float m2 = a * d - b * b;
  if (!(a > 0.f) || !(m2 > 0.f) || !(det > 0.f)) return ST_NOT_PD;
  const float id = 1.f / det;
  ri[0] = i00 * id;
  ri[1] = i10 * id;
  ri[2] = (a * g - e * e) * id;
  ri[3] = i20 * id;
  ri[4] = (b * e - a * f) * id;
  ri[5] = m2 * id;
  r[0] = m[0] - s[0];
  r[1] = m[1] - s[1];
  r[2] = m[2] - s[2];
  const float q0 = ri[0] * r[0] + ri[1] * r[1] + ri[3] * r[2];
  const float q1 = ri[1] * r[0] + ri[2] * r[1] + ri[4] * r[2];
  const float q2 = ri[3] * r[0] + ri[4] * r[1] + ri[5] * r[2];
  chi2 = r[0] * q0 + r[1] * q1 + r[2] * q2;
  return 0;
}

// Kalman update with the hit (m, v), computed in precision T (the state and
// covariance stay float32 in registers and HBM).  The covariance uses the
// algebraically identical forms C_pos'' = A R^-1 V, C_mom,pos'' = B R^-1 V and
// C_mom'' = D - B R^-1 B^T (A, B, D = position, cross and momentum blocks),
// which avoid the cancellation of A - A R^-1 A when the prior is vague.  The
// remaining cancellation in D - B R^-1 B^T and the 3x3 inverse are what limit
// a float32 update; gfx950 runs FP64 FMA at the unpacked FP32 rate, so the fit
// and the build's survivor update use T = double.
template <typename T>
KF_DEV int32_t update_t(float s[6], float c[21], const float m[3], const float v[6], float& chi2_out) {
  const T a = T(c[0]) + T(v[0]), b = T(c[1]) + T(v[1]), d = T(c[2]) + T(v[2]);
  const T e = T(c[3]) + T(v[3]), f = T(c[4]) + T(v[4]), g = T(c[5]) + T(v[5]);
  const T i00 = d * g - f * f;
  const T i10 = e * f - b * g;
  const T i20 = b * f - d * e;
  const T det = a * i00 + b * i10 + e * i20;
  const T m2 = a * d - b * b;
  if (!(a > T(0)) || !(m2 > T(0)) || !(det > T(0))) return ST_NOT_PD;
  const T id = T(1) / det;
  const T Ri[3][3] = {{i00 * id, i10 * id, i20 * id},
                      {i10 * id, (a * g - e * e) * id, (b * e - a * f) * id},
                      {i20 * id, (b * e - a * f) * id, m2 * id}};
  const T r[3] = {T(m[0]) - T(s[0]), T(m[1]) - T(s[1]), T(m[2]) - T(s[2])};
  T q[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) q[i] = Ri[i][0] * r[0] + Ri[i][1] * r[1] + Ri[i][2] * r[2];
  const T chi2 = r[0] * q[0] + r[1] * q[1] + r[2] * q[2];
  const T V[3][3] = {{T(v[0]), T(v[1]), T(v[3])}, {T(v[1]), T(v[2]), T(v[4])}, {T(v[3]), T(v[4]), T(v[5])}};
  T M[3][3];  // R^-1 V
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[i][j] = Ri[i][0] * V[0][j] + Ri[i][1] * V[1][j] + Ri[i][2] * V[2][j];
  T A[3][3], B[3][3], D[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      A[i][j] = T(c[tri(i, j)]);
      B[i][j] = T(c[tri(i + 3, j)]);
      D[i][j] = T(c[tri(i + 3, j + 3)]);
    }
  T G[3][3];  // B R^-1
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) G[i][j] = B[i][0] * Ri[0][j] + B[i][1] * Ri[1][j] + B[i][2] * Ri[2][j];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    s[i] = static_cast<float>(T(s[i]) + (A[i][0] * q[0] + A[i][1] * q[1] + A[i][2] * q[2]));
    s[i + 3] = static_cast<float>(T(s[i + 3]) + (B[i][0] * q[0] + B[i][1] * q[1] + B[i][2] * q[2]));
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j)
      c[tri(i, j)] = static_cast<float>(A[i][0] * M[0][j] + A[i][1] * M[1][j] + A[i][2] * M[2][j]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      c[tri(i + 3, j)] = static_cast<float>(B[i][0] * M[0][j] + B[i][1] * M[1][j] + B[i][2] * M[2][j]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j)
      c[tri(i + 3, j + 3)] = static_cast<float>(D[i][j] - (G[i][0] * B[j][0] + G[i][1] * B[j][1] + G[i][2] * B[j][2]));
  chi2_out = static_cast<float>(chi2);
  if (!finite6_21(s, c)) return ST_NONFINITE;
  return 0;
}

KF_DEV int32_t update(float s[6], float c[21], const float m[3], const float v[6], float& chi2) {
  return update_t<double>(s, c, m, v, chi2);
}

}  // namespace kfd
