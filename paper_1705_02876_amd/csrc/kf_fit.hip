// kf_fit.hip -- context, geometry, and the propagate / update / fit entry
// points of the C ABI (one track per lane, structure-of-arrays in HBM).
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>
#include <string>
#include <type_traits>

#include "kf_internal.hpp"

using namespace kfd;

namespace {

thread_local std::string g_last_error = "no error";

// Coalesced SoA loads/stores of one track's state and packed covariance
// (float32 in HBM, T in registers).
// Element idx of an array row whose start is uniform across the wave: with a 32-bit index the byte offset is
// formed in 32 bits too (the caller keeps every array under 4 GiB), so an access is a scalar base plus a 32-bit
// vector offset, without 64-bit address arithmetic per lane.
template <typename P>
__device__ __forceinline__ P* elem(P* base, uint32_t idx) {
  using C = typename std::conditional<std::is_const<P>::value, const char, char>::type;
  return reinterpret_cast<P*>(reinterpret_cast<C*>(base) + idx * static_cast<uint32_t>(sizeof(P)));
}
template <typename P>
__device__ __forceinline__ P* elem(P* base, int64_t idx) {
  return base + idx;
}

template <typename T, typename I>
__device__ __forceinline__ void load_track(const float* __restrict__ st, const float* __restrict__ cv, I ld, I i,
                                           T s[6], T c[21]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) s[k] = T(__builtin_nontemporal_load(elem(st + k * static_cast<int64_t>(ld), i)));
#pragma unroll
  for (int k = 0; k < 21; ++k) c[k] = T(__builtin_nontemporal_load(elem(cv + k * static_cast<int64_t>(ld), i)));
}

template <typename T, typename I>
__device__ __forceinline__ void store_track(float* __restrict__ st, float* __restrict__ cv, I ld, I i,
                                            const T s[6], const T c[21]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) __builtin_nontemporal_store(static_cast<float>(s[k]), elem(st + k * static_cast<int64_t>(ld), i));
#pragma unroll
  for (int k = 0; k < 21; ++k) __builtin_nontemporal_store(static_cast<float>(c[k]), elem(cv + k * static_cast<int64_t>(ld), i));
}

__global__ void __launch_bounds__(256) propagate_kernel(int64_t n, int64_t ld, float* state, float* cov,
                                                        const int8_t* __restrict__ charge,
                                                        const float* __restrict__ r_target, float r_scalar,
                                                        float z_half, int32_t material_layer, Geom g,
                                                        int32_t* __restrict__ status) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s[6], c[21];
  load_track(state, cov, ld, i, s, c);
  const float a = static_cast<float>(-static_cast<double>(charge[i]) * kCLight * g.bz);
  int32_t st = 0;
  if (material_layer >= 0) {
    if (!finite6_21(s, c))
      st = ST_NONFINITE;
    else
      st = material(s, c, g.x_over_x0[material_layer], g.eloss_per_x0, g.mass);
  }
  if (!st) st = propagate(s, c, a, r_target ? r_target[i] : r_scalar, z_half);
  if (!st) store_track(state, cov, ld, i, s, c);
  status[i] = st;
}

__global__ void __launch_bounds__(256) update_kernel(int64_t n, int64_t ld, float* state, float* cov,
                                                     const float* __restrict__ hit_pos,
                                                     const float* __restrict__ hit_cov, int64_t ldh,
                                                     float* __restrict__ chi2, int32_t* __restrict__ status,
                                                     int chi2_only) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s[6], c[21], m[3], v[6];
  load_track(state, cov, ld, i, s, c);
#pragma unroll
  for (int k = 0; k < 3; ++k) m[k] = hit_pos[k * ldh + i];
#pragma unroll
  for (int k = 0; k < 6; ++k) v[k] = hit_cov[k * ldh + i];
  float c2 = 0.f;
  int32_t st;
  if (!finite6_21(s, c)) {
    st = ST_NONFINITE;
  } else {
    float s2[6], cc[21];
#pragma unroll
    for (int k = 0; k < 6; ++k) s2[k] = s[k];
#pragma unroll
    for (int k = 0; k < 21; ++k) cc[k] = c[k];
    st = update_global<float, double>(s2, cc, m, v, c2);
    if (!st && !chi2_only) store_track(state, cov, ld, i, s2, cc);
  }
  chi2[i] = st ? 0.f : c2;
  status[i] = st;
}

// Training record of a prediction for the learned search window: its
// features, then the tangential and z offsets of the track's own hit.
template <typename T, typename I>
__device__ __forceinline__ void emit_residual(float* __restrict__ out, I ldr, I row, const T s[6],
                                              const T c[21], float q, float r_from, float r_to, float zh,
                                              const float m[3]) {
  float f[KF_RES_FEATURES];
  window_features(s, c, q, r_from, r_to, zh, f);
  const float x = float(s[0]), y = float(s[1]), z = float(s[2]);
  const float ir = __frsqrt_rn(x * x + y * y);
  const float tx = -y * ir, ty = x * ir;
#pragma unroll
  for (int k = 0; k < KF_RES_FEATURES; ++k) *elem(out + k * static_cast<int64_t>(ldr), row) = f[k];
  *elem(out + KF_RES_FEATURES * static_cast<int64_t>(ldr), row) = tx * (m[0] - x) + ty * (m[1] - y);
  *elem(out + (KF_RES_FEATURES + 1) * static_cast<int64_t>(ldr), row) = m[2] - z;
}

template <typename I>
__device__ __forceinline__ void load_hit(const float* __restrict__ hit_pos, const float* __restrict__ hit_cov, I ldh,
                                         int32_t h, float m[3], float v[6]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) m[k] = *elem(hit_pos + k * static_cast<int64_t>(ldh), static_cast<I>(h));
#pragma unroll
  for (int k = 0; k < 6; ++k) v[k] = *elem(hit_cov + k * static_cast<int64_t>(ldh), static_cast<I>(h));
}

template <typename T, typename I>
__device__ __forceinline__ void fit_body(I n, I ld, const float* state_in, const float* cov_in,
                                         const int8_t* __restrict__ charge, const int32_t* __restrict__ hit_idx,
                                         I ld_idx, const float* __restrict__ hit_pos,
                                         const float* __restrict__ hit_cov, I ldh, float* state_out,
                                         float* cov_out, float* __restrict__ chi2_out,
                                         int32_t* __restrict__ nhits_out, int32_t* __restrict__ status_out,
                                         const Geom& g, float* __restrict__ res, I ldr) {
  const I i = static_cast<I>(blockIdx.x) * static_cast<I>(blockDim.x) + static_cast<I>(threadIdx.x);
  if (i >= n) return;
  const int L = g.n_layers;
  T s[6], c[21];
  load_track(state_in, cov_in, ld, i, s, c);
  const int8_t qi = *elem(charge, i);
  const float qf = static_cast<float>(qi);
  const T a = T(-static_cast<double>(qi) * kCLight * g.bz);
  int last = -1;  // last layer with a hit: searched from the outside in (most tracks end near the outer layers)
  for (int l = L - 1; l >= 0; --l)
    if (*elem(hit_idx + l * static_cast<int64_t>(ld_idx), i) >= 0) {
      last = l;
      break;
    }
  T chi2 = T(0);
  int32_t nh = 0, st = 0;
  if (res) {
    for (int l = 1; l < L; ++l)
#pragma unroll
      for (int k = 0; k < KF_RES_FEATURES + 2; ++k) *elem(res + k * static_cast<int64_t>(ldr), i * static_cast<I>(L - 1) + static_cast<I>(l - 1)) = NAN;
  }
  // The hit of layer l is fetched at the start of its iteration, before the
  // crossing, whose arithmetic covers the gather's latency; its index is read
  // one layer ahead.  A layer without a hit loads hit 0 instead (never used;
  // the track has a hit, so the arrays are not empty), so the loads need no
  // branch and no zeroed registers.
  // The state is updated in place.  A failing step stops the track; its last
  // valid state is then recovered by replaying the track up to that step (rare:
  // keeping a copy of the state at every step would cost every track).
  int32_t h_nxt = last >= 0 ? *elem(hit_idx, i) : -1;
  float r_from = 0.f;
  // layer and step that failed: 0 its crossing or its update (one step: the state before the layer is kept),
  // 1 its material (the state after the update is kept)
  int fail_l = 0, fail_step = 0;
  // A failing lane stops stepping (ok turns false) but stays in the loop, so that the state registers are the
  // loop's own on every path (an exit from the loop would copy the covariance into other registers at each layer).
  bool ok = true;
  for (int l = 0; l <= last; ++l) {
    if (!ok) continue;
    const int32_t h_cur = h_nxt;
    float m[3], v[6];
    load_hit(hit_pos, hit_cov, ldh, h_cur >= 0 ? h_cur : 0, m, v);
    h_nxt = (l + 1 <= last) ? *elem(hit_idx + (l + 1) * static_cast<int64_t>(ld_idx), i) : -1;
    st = propagate_inplace(s, c, a, T(g.r[l]), T(0));  // a failure is replayed below
    if (st) {
      fail_l = l;
      fail_step = 0;
      ok = false;
      continue;
    }
    if (h_cur >= 0) {
      T dc2;
      if (res && l >= 1) emit_residual(res, ldr, i * static_cast<I>(L - 1) + static_cast<I>(l - 1), s, c, qf, r_from, g.r[l], g.z_half[l], m);
      st = update_on_layer<T, double>(s, c, m, v, dc2);
      if (st) {
        fail_l = l;
        fail_step = 0;
        ok = false;
        continue;
      }
      chi2 += dc2;
      nh += 1;
    }
    r_from = g.r[l];
    if (l < last) {
      st = material(s, c, T(g.x_over_x0[l]), T(g.eloss_per_x0), T(g.mass));
      if (st) {
        fail_l = l;
        fail_step = 1;
        ok = false;
      }
    }
  }
  if (st) {
    // replay the steps before the failing one (the same arithmetic in the same order: the same values)
    load_track(state_in, cov_in, ld, i, s, c);
    for (int l = 0; l <= fail_l; ++l) {
      if (l == fail_l && fail_step == 0) break;
      propagate(s, c, a, T(g.r[l]), T(0));
      const int32_t h = *elem(hit_idx + l * static_cast<int64_t>(ld_idx), i);
      if (h >= 0) {
        float mm[3], vv[6];
        load_hit(hit_pos, hit_cov, ldh, h, mm, vv);
        T dc2;
        update_on_layer<T, double>(s, c, mm, vv, dc2);
      }
      if (l == fail_l) break;
      material(s, c, T(g.x_over_x0[l]), T(g.eloss_per_x0), T(g.mass));
    }
  }
  store_track(state_out, cov_out, ld, i, s, c);
  *elem(chi2_out, i) = static_cast<float>(chi2);
  *elem(nhits_out, i) = nh;
  *elem(status_out, i) = st;
}

#define KF_FIT_PARAMS                                                                                             \
  int64_t n, int64_t ld, const float *state_in, const float *cov_in, const int8_t *__restrict__ charge,          \
      const int32_t *__restrict__ hit_idx, int64_t ld_idx, const float *__restrict__ hit_pos,                    \
      const float *__restrict__ hit_cov, int64_t ldh, float *state_out, float *cov_out,                           \
      float *__restrict__ chi2_out, int32_t *__restrict__ nhits_out, int32_t *__restrict__ status_out, Geom g,   \
      float *__restrict__ res, int64_t ldr
#define KF_FIT_ARGS                                                                                               \
  n, ld, state_in, cov_in, charge, hit_idx, ld_idx, hit_pos, hit_cov, ldh, state_out, cov_out, chi2_out,         \
      nhits_out, status_out, g, res, ldr
#define KF_FIT_ARGS32                                                                                             \
  static_cast<uint32_t>(n), static_cast<uint32_t>(ld), state_in, cov_in, charge, hit_idx,                         \
      static_cast<uint32_t>(ld_idx), hit_pos, hit_cov, static_cast<uint32_t>(ldh), state_out, cov_out, chi2_out, \
      nhits_out, status_out, g, res, static_cast<uint32_t>(ldr)

// single precision: compiled for three waves per SIMD (at most 168 registers; the fit's dependent chains of
// loads and arithmetic are latency bound); double precision keeps the default
// With every array under 4 GiB the element offsets are computed in 32 bits, so the loads address a scalar base
// plus a 32-bit offset instead of doing 64-bit address arithmetic per access.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) fit_kernel(KF_FIT_PARAMS) {
  fit_body<float, uint32_t>(KF_FIT_ARGS32);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) fit_kernel_i64(KF_FIT_PARAMS) {
  fit_body<float, int64_t>(KF_FIT_ARGS);
}

__global__ void __launch_bounds__(256) fit_kernel_f64(KF_FIT_PARAMS) { fit_body<double, int64_t>(KF_FIT_ARGS); }

// ---------------------------------------------------------------------------
// Smoother: the fit followed by the Rauch-Tung-Striebel backward pass, which
// gives every layer the estimate from all of the track's hits.  With xf, Cf
// the filtered and xp, Cp the predicted estimates and F the derivative of the
// filter's step from layer l to l+1 (material of l, then the crossing of l+1),
//   K = Cf F^T Cp^+,  xs_l = xf_l + K (xs_{l+1} - xp_{l+1}),
//   Cs_l = Cf_l + K (Cs_{l+1} - Cp_{l+1}) K^T.
// A prediction on a cylinder has no radial variance, so Cp^+ is the
// pseudo-inverse on the surface, P^T (P Cp P^T)^-1 P with P the orthonormal
// rows (tangent, z, px, py, pz).  F = J diag(1, 1, 1, f, f, f): the material
// scales the momentum by f, then J is the crossing's surface Jacobian.
//
// One track per lane.  The forward pass writes each layer's filtered state into
// that layer's output row; the backward pass reads it back, repeats the
// filter's step to the next layer (the same arithmetic, so the same prediction
// in single precision), forms the gain in double precision and overwrites the
// row with the smoothed state.  With W = B L^-T (B = Cf F^T P^T, S = P Cp P^T
// = L L^T): K (xs - xp) = W L^-1 P (xs - xp) and K M K^T = W N W^T with
// N = L^-1 P M P^T L^-T, so only triangular solves against L are needed.
template <typename T, typename I>
__device__ __forceinline__ void store_row(float* __restrict__ st, float* __restrict__ cv, I ld, int l, I i,
                                          const T s[6], const T c[21]) {
  float* sr = st + static_cast<int64_t>(l) * 6 * static_cast<int64_t>(ld);
  float* cr = cv + static_cast<int64_t>(l) * 21 * static_cast<int64_t>(ld);
  // ordinary (cached) stores: the rows form 27 L strided streams, which non-temporal stores write back
  // several times slower
#pragma unroll
  for (int k = 0; k < 6; ++k) *elem(sr + k * static_cast<int64_t>(ld), i) = static_cast<float>(s[k]);
#pragma unroll
  for (int k = 0; k < 21; ++k) *elem(cr + k * static_cast<int64_t>(ld), i) = static_cast<float>(c[k]);
}

template <typename I>
__device__ __forceinline__ void load_row(const float* st, const float* cv, I ld, int l, I i, float s[6],
                                         float c[21]) {
  const float* sr = st + static_cast<int64_t>(l) * 6 * static_cast<int64_t>(ld);
  const float* cr = cv + static_cast<int64_t>(l) * 21 * static_cast<int64_t>(ld);
#pragma unroll
  for (int k = 0; k < 6; ++k) s[k] = *elem(sr + k * static_cast<int64_t>(ld), i);
#pragma unroll
  for (int k = 0; k < 21; ++k) c[k] = *elem(cr + k * static_cast<int64_t>(ld), i);
}

// Forward pass: the fit, each completed layer's filtered state stored in its row, NaN in the rows it did not
// reach.  Writes chi2, nhits (nullable) and status.
template <typename T, typename I>
__device__ __forceinline__ void smooth_fwd_body(I n, I ld, const float* state_in, const float* cov_in,
                                                const int8_t* __restrict__ charge, const int32_t* __restrict__ hit_idx,
                                                I ld_idx, const float* __restrict__ hit_pos,
                                                const float* __restrict__ hit_cov, I ldh, float* state_out,
                                                float* cov_out, float* __restrict__ chi2_out,
                                                int32_t* __restrict__ nhits_out, int32_t* __restrict__ status_out,
                                                const Geom& g) {
  const I i = static_cast<I>(blockIdx.x) * static_cast<I>(blockDim.x) + static_cast<I>(threadIdx.x);
  if (i >= n) return;
  const int L = g.n_layers;
  T s[6], c[21];
  load_track(state_in, cov_in, ld, i, s, c);
  const int8_t qi = *elem(charge, i);
  const T a = T(-static_cast<double>(qi) * kCLight * g.bz);
  int last = -1;
  for (int l = L - 1; l >= 0; --l)
    if (*elem(hit_idx + l * static_cast<int64_t>(ld_idx), i) >= 0) {
      last = l;
      break;
    }
  // Every layer's row is written at that layer's iteration by every lane of the wave in one store
  // instruction (the filtered state, or NaN where the lane's filter did not complete the layer), so each
  // cache line of a row is written whole, once.
  T chi2 = T(0);
  int32_t nh = 0, st = 0;
  bool alive = true;  // no step has failed and the layer is not beyond the last hit layer
  int32_t h_nxt = last >= 0 ? *elem(hit_idx, i) : -1;
  for (int l = 0; l < L; ++l) {
    alive = alive && l <= last;
    bool row_ok = false;
    if (alive) {
      const int32_t h_cur = h_nxt;
      float m[3], v[6];
      load_hit(hit_pos, hit_cov, ldh, h_cur >= 0 ? h_cur : 0, m, v);
      h_nxt = (l + 1 <= last) ? *elem(hit_idx + (l + 1) * static_cast<int64_t>(ld_idx), i) : -1;
      st = propagate_inplace(s, c, a, T(g.r[l]), T(0));  // a failure ends the track (its rows are NaN)
      if (!st && h_cur >= 0) {
        T dc2;
        st = update_on_layer<T, double>(s, c, m, v, dc2);
        if (!st) {
          chi2 += dc2;
          nh += 1;
        }
      }
      row_ok = st == 0;
    }
    {
      T rs[6], rc[21];
#pragma unroll
      for (int k = 0; k < 6; ++k) rs[k] = row_ok ? s[k] : T(NAN);
#pragma unroll
      for (int k = 0; k < 21; ++k) rc[k] = row_ok ? c[k] : T(NAN);
      store_row(state_out, cov_out, ld, l, i, rs, rc);
    }
    if (alive) {
      if (!row_ok)
        alive = false;
      else if (l < last) {
        st = material(s, c, T(g.x_over_x0[l]), T(g.eloss_per_x0), T(g.mass));
        if (st) alive = false;
      }
    }
  }
  if (chi2_out) *elem(chi2_out, i) = static_cast<float>(chi2);
  if (nhits_out) *elem(nhits_out, i) = nh;
  *elem(status_out, i) = st;
}

// Backward pass of the tracks whose fit converged: from the last hit layer's row (filtered there = smoothed)
// inward, over a layer index that is uniform across the wave.  A failing step (not positive definite) sets the
// status and leaves the rows below it filtered.
template <typename T, typename I>
__device__ __forceinline__ void smooth_bwd_body(I n, I ld, const int8_t* __restrict__ charge,
                                                const int32_t* __restrict__ hit_idx, I ld_idx, float* state_out,
                                                float* cov_out, int32_t* __restrict__ status_out, const Geom& g) {
  const I i = static_cast<I>(blockIdx.x) * static_cast<I>(blockDim.x) + static_cast<I>(threadIdx.x);
  if (i >= n) return;
  if (*elem(status_out, i) != 0) return;
  const int L = g.n_layers;
  int last = -1;
  for (int l = L - 1; l >= 0; --l)
    if (*elem(hit_idx + l * static_cast<int64_t>(ld_idx), i) >= 0) {
      last = l;
      break;
    }
  if (last < 1) return;
  const int8_t qi = *elem(charge, i);
  const T a = T(-static_cast<double>(qi) * kCLight * g.bz);
  // The carried state (xs, cs) is the smoothed state of the layer outside the current one.  A lane that takes
  // no step at a layer (above its last hit layer, at the last hit layer itself, or after a failed step) takes
  // that layer's row as read, so at its last hit layer it picks up the filtered (= smoothed) state there.
  // Every lane writes every row at that row's iteration, in one store instruction, so the cache lines of a row
  // are written whole (lanes that skipped their store left partial lines, which the cache filled from memory
  // first).  The next row inward is fetched while the current step computes (two waves per SIMD cover little
  // of the latency); rows of every layer exist (NaN above the last hit layer).
  float xs[6], cs[21];
  load_row(state_out, cov_out, ld, L - 1, i, xs, cs);
  float xn[6], cn[21];
  load_row(state_out, cov_out, ld, L - 2, i, xn, cn);
  bool live = true;
  for (int l = L - 2; l >= 0; --l) {
    float xf[6], cf[21];
#pragma unroll
    for (int k = 0; k < 6; ++k) xf[k] = xn[k];
#pragma unroll
    for (int k = 0; k < 21; ++k) cf[k] = cn[k];
    if (l >= 1) load_row(state_out, cov_out, ld, l - 1, i, xn, cn);
    bool stepped = false;
    if (live && l < last) {
      const int32_t st = rts_step<T, double>(xf, cf, a, g, l, xs, cs);
      if (st) {
        *elem(status_out, i) = st;
        live = false;
      } else {
        stepped = true;
      }
    }
    if (!stepped) {
#pragma unroll
      for (int k = 0; k < 6; ++k) xs[k] = xf[k];
#pragma unroll
      for (int k = 0; k < 21; ++k) cs[k] = cf[k];
    }
    store_row(state_out, cov_out, ld, l, i, xs, cs);
  }
}

#define KF_SMOOTH_PARAMS                                                                                          \
  int64_t n, int64_t ld, const float *state_in, const float *cov_in, const int8_t *__restrict__ charge,          \
      const int32_t *__restrict__ hit_idx, int64_t ld_idx, const float *__restrict__ hit_pos,                    \
      const float *__restrict__ hit_cov, int64_t ldh, float *state_out, float *cov_out,                           \
      float *__restrict__ chi2_out, int32_t *__restrict__ nhits_out, int32_t *__restrict__ status_out, Geom g
#define KF_SMOOTH_ARGS                                                                                            \
  n, ld, state_in, cov_in, charge, hit_idx, ld_idx, hit_pos, hit_cov, ldh, state_out, cov_out, chi2_out,         \
      nhits_out, status_out, g
#define KF_SMOOTH_ARGS32                                                                                          \
  static_cast<uint32_t>(n), static_cast<uint32_t>(ld), state_in, cov_in, charge, hit_idx,                         \
      static_cast<uint32_t>(ld_idx), hit_pos, hit_cov, static_cast<uint32_t>(ldh), state_out, cov_out, chi2_out, \
      nhits_out, status_out, g
#define KF_SMOOTH_BWD_PARAMS                                                                                      \
  int64_t n, int64_t ld, const int8_t *__restrict__ charge, const int32_t *__restrict__ hit_idx, int64_t ld_idx, \
      float *state_out, float *cov_out, int32_t *__restrict__ status_out, Geom g
#define KF_SMOOTH_BWD_ARGS n, ld, charge, hit_idx, ld_idx, state_out, cov_out, status_out, g
#define KF_SMOOTH_BWD_ARGS32                                                                                      \
  static_cast<uint32_t>(n), static_cast<uint32_t>(ld), charge, hit_idx, static_cast<uint32_t>(ld_idx),           \
      state_out, cov_out, status_out, g

// the forward pass has the fit's register needs and its occupancy; the backward pass's double-precision
// gain fits two waves per SIMD (at most 256 registers, no spills) in single precision
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) smooth_fwd_kernel(KF_SMOOTH_PARAMS) {
  smooth_fwd_body<float, uint32_t>(KF_SMOOTH_ARGS32);
}
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) smooth_fwd_kernel_i64(KF_SMOOTH_PARAMS) {
  smooth_fwd_body<float, int64_t>(KF_SMOOTH_ARGS);
}
__global__ void __launch_bounds__(256) smooth_fwd_kernel_f64(KF_SMOOTH_PARAMS) { smooth_fwd_body<double, int64_t>(KF_SMOOTH_ARGS); }
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) smooth_bwd_kernel(KF_SMOOTH_BWD_PARAMS) {
  smooth_bwd_body<float, uint32_t>(KF_SMOOTH_BWD_ARGS32);
}
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) smooth_bwd_kernel_i64(KF_SMOOTH_BWD_PARAMS) {
  smooth_bwd_body<float, int64_t>(KF_SMOOTH_BWD_ARGS);
}
__global__ void __launch_bounds__(256) smooth_bwd_kernel_f64(KF_SMOOTH_BWD_PARAMS) {
  smooth_bwd_body<double, int64_t>(KF_SMOOTH_BWD_ARGS);
}

}  // namespace

namespace kfh {

int32_t set_error(int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int32_t enter(kf_ctx* ctx) {
  if (!ctx) return set_error(KF_ERR_INVALID_ARG, "null context");
  return check_hip(hipSetDevice(ctx->device), "hipSetDevice");
}

}  // namespace kfh

using kfh::set_error;

extern "C" {

const char* kf_last_error(void) { return g_last_error.c_str(); }

int32_t kf_ctx_create(kf_ctx** out, int32_t device) {
  if (!out) return set_error(KF_ERR_INVALID_ARG, "null output pointer");
  *out = nullptr;
  int count = 0;
  if (int32_t rc = kfh::check_hip(hipGetDeviceCount(&count), "hipGetDeviceCount")) return rc;
  if (device < 0 || device >= count) return set_error(KF_ERR_INVALID_ARG, "device %d out of range", device);
  hipDeviceProp_t prop;
  if (int32_t rc = kfh::check_hip(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties")) return rc;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return set_error(KF_ERR_UNSUPPORTED, "device %d is %s, this library is built for gfx950", device,
                     prop.gcnArchName);
  kf_ctx* c = new kf_ctx();
  c->device = device;
  c->num_cus = prop.multiProcessorCount;
  std::snprintf(c->arch, sizeof c->arch, "%s", prop.gcnArchName);
  for (char* ch = c->arch; *ch; ++ch)  // the name goes into cache keys: keep it free of separators and quotes
    if (*ch == ':' || *ch == '"' || *ch == ' ') *ch = '.';
  if (int32_t rc = kfh::check_hip(hipSetDevice(device), "hipSetDevice")) {
    delete c;
    return rc;
  }
  if (int32_t rc = kfh::scratch_init(c)) {
    delete c;
    return rc;
  }
  *out = c;
  return KF_OK;
}

void kf_ctx_destroy(kf_ctx* ctx) {
  kfh::ctx_release(ctx);
  delete ctx;
}

int32_t kf_set_geometry(kf_ctx* ctx, const kf_geometry* g) {
  if (!ctx || !g) return set_error(KF_ERR_INVALID_ARG, "null argument");
  if (g->n_layers < 1 || g->n_layers > KF_MAX_LAYERS)
    return set_error(KF_ERR_GEOMETRY, "n_layers %d not in [1, %d]", g->n_layers, KF_MAX_LAYERS);
  for (int l = 0; l < g->n_layers; ++l) {
    if (!(g->r[l] > 0.f) || !std::isfinite(g->r[l])) return set_error(KF_ERR_GEOMETRY, "r[%d] not positive", l);
    if (l > 0 && !(g->r[l] > g->r[l - 1])) return set_error(KF_ERR_GEOMETRY, "radii not strictly increasing");
    if (!(g->z_half[l] > 0.f)) return set_error(KF_ERR_GEOMETRY, "z_half[%d] not positive", l);
    if (!(g->x_over_x0[l] >= 0.f)) return set_error(KF_ERR_GEOMETRY, "x_over_x0[%d] negative", l);
  }
  if (!std::isfinite(g->bz) || !(g->mass > 0.f) || !(g->eloss_per_x0 >= 0.f))
    return set_error(KF_ERR_GEOMETRY, "bad field, mass or energy loss");
  ctx->geom = *g;
  Geom& d = ctx->dgeom;
  std::memset(&d, 0, sizeof d);
  d.n_layers = g->n_layers;
  for (int l = 0; l < KF_MAX_LAYERS; ++l) {
    d.r[l] = g->r[l];
    d.z_half[l] = g->z_half[l];
    d.x_over_x0[l] = g->x_over_x0[l];
  }
  d.bz = g->bz;
  d.eloss_per_x0 = g->eloss_per_x0;
  d.mass = g->mass;
  ctx->has_geometry = true;
  return KF_OK;
}

int32_t kf_propagate_to_r(kf_ctx* ctx, int64_t n, int64_t ld, float* state, float* cov, const int8_t* charge,
                          const float* r_target, float r_scalar, float z_half, int32_t material_layer,
                          int32_t* status, void* stream) {
  if (int32_t rc = kfh::enter(ctx)) return rc;
  if (!ctx->has_geometry) return set_error(KF_ERR_GEOMETRY, "no geometry set");
  if (n < 0 || ld < n) return set_error(KF_ERR_INVALID_ARG, "n=%lld ld=%lld", (long long)n, (long long)ld);
  if (n == 0) return KF_OK;
  if (!state || !cov || !charge || !status) return set_error(KF_ERR_INVALID_ARG, "null array");
  if (!r_target && !(r_scalar > 0.f)) return set_error(KF_ERR_INVALID_ARG, "r_scalar must be > 0");
  if (material_layer >= ctx->geom.n_layers) return set_error(KF_ERR_INVALID_ARG, "material_layer out of range");
  propagate_kernel<<<kfh::grid_for(n, 256), 256, 0, kfh::stream_of(stream)>>>(
      n, ld, state, cov, charge, r_target, r_scalar, z_half, material_layer, ctx->dgeom, status);
  return kfh::check_hip(hipGetLastError(), "propagate_kernel launch");
}

int32_t kf_update(kf_ctx* ctx, int64_t n, int64_t ld, float* state, float* cov, const float* hit_pos,
                  const float* hit_cov, int64_t ldh, float* chi2, int32_t* status, uint32_t flags, void* stream) {
  if (int32_t rc = kfh::enter(ctx)) return rc;
  if (n < 0 || ld < n || ldh < n)
    return set_error(KF_ERR_INVALID_ARG, "n=%lld ld=%lld ldh=%lld", (long long)n, (long long)ld, (long long)ldh);
  if (flags & ~KF_UPDATE_CHI2_ONLY) return set_error(KF_ERR_INVALID_ARG, "unknown flags %u", flags);
  if (n == 0) return KF_OK;
  if (!state || !cov || !hit_pos || !hit_cov || !chi2 || !status) return set_error(KF_ERR_INVALID_ARG, "null array");
  update_kernel<<<kfh::grid_for(n, 256), 256, 0, kfh::stream_of(stream)>>>(
      n, ld, state, cov, hit_pos, hit_cov, ldh, chi2, status, (flags & KF_UPDATE_CHI2_ONLY) ? 1 : 0);
  return kfh::check_hip(hipGetLastError(), "update_kernel launch");
}

int32_t kf_fit(kf_ctx* ctx, const kf_fit_args* a) {
  if (int32_t rc = kfh::enter(ctx)) return rc;
  if (!a) return set_error(KF_ERR_INVALID_ARG, "null args");
  if (!ctx->has_geometry) return set_error(KF_ERR_GEOMETRY, "no geometry set");
  const int L = ctx->geom.n_layers;
  if (a->n < 0 || a->ld < a->n || a->ld_idx < a->n || a->ldh < 0)
    return set_error(KF_ERR_INVALID_ARG, "bad sizes");
  if (a->flags & ~(KF_FIT_EMIT_RESIDUALS | KF_FIT_FP64)) return set_error(KF_ERR_INVALID_ARG, "unknown flags %u", a->flags);
  const bool emit = (a->flags & KF_FIT_EMIT_RESIDUALS) != 0;
  if (emit && (!a->residual_out || L < 2 || a->ld_res < a->n * (L - 1)))
    return set_error(KF_ERR_INVALID_ARG, "residual_out missing or ld_res < n * (n_layers - 1)");
  if (a->n == 0) return KF_OK;
  if (!a->state_in || !a->cov_in || !a->charge || !a->hit_idx || !a->state_out || !a->cov_out || !a->chi2_out ||
      !a->nhits_out || !a->status_out)
    return set_error(KF_ERR_INVALID_ARG, "null array");
  // 32-bit element offsets when every array's byte extent stays below 4 GiB
  const int64_t ext = std::max({21 * a->ld, static_cast<int64_t>(L) * a->ld_idx, 6 * a->ldh,
                                emit ? (KF_RES_FEATURES + 2) * a->ld_res : int64_t(0)});
  const bool narrow = ext < (int64_t(1) << 30);
  auto kern = (a->flags & KF_FIT_FP64) ? fit_kernel_f64 : (narrow ? fit_kernel : fit_kernel_i64);
  int block = 256;  // tuned block size for this problem class, if kf_fit_autotune found one
  if (!ctx->fit_tuned.empty()) {
    auto it = ctx->fit_tuned.find(kfh::fit_tune_key(ctx, a->flags, a->n));
    if (it != ctx->fit_tuned.end()) block = 64 * it->second.waves_per_block;
  }
  kern<<<kfh::grid_for(a->n, block), block, 0, kfh::stream_of(a->stream)>>>(
      a->n, a->ld, a->state_in, a->cov_in, a->charge, a->hit_idx, a->ld_idx, a->hit_pos, a->hit_cov, a->ldh,
      a->state_out, a->cov_out, a->chi2_out, a->nhits_out, a->status_out, ctx->dgeom,
      emit ? a->residual_out : nullptr, a->ld_res);
  return kfh::check_hip(hipGetLastError(), "fit_kernel launch");
}

int32_t kf_smooth(kf_ctx* ctx, const kf_smooth_args* a) {
  if (int32_t rc = kfh::enter(ctx)) return rc;
  if (!a) return set_error(KF_ERR_INVALID_ARG, "null args");
  if (!ctx->has_geometry) return set_error(KF_ERR_GEOMETRY, "no geometry set");
  const int L = ctx->geom.n_layers;
  if (a->n < 0 || a->ld < a->n || a->ld_idx < a->n || a->ldh < 0) return set_error(KF_ERR_INVALID_ARG, "bad sizes");
  if (a->flags & ~KF_FIT_FP64) return set_error(KF_ERR_INVALID_ARG, "unknown flags %u", a->flags);
  if (a->n == 0) return KF_OK;
  if (!a->state_in || !a->cov_in || !a->charge || !a->hit_idx || !a->state_out || !a->cov_out || !a->status_out)
    return set_error(KF_ERR_INVALID_ARG, "null array");
  const int64_t ext = std::max({static_cast<int64_t>(L) * 21 * a->ld, static_cast<int64_t>(L) * a->ld_idx, 6 * a->ldh});
  const bool narrow = ext < (int64_t(1) << 30);
  const bool f64 = (a->flags & KF_FIT_FP64) != 0;
  auto fwd = f64 ? smooth_fwd_kernel_f64 : (narrow ? smooth_fwd_kernel : smooth_fwd_kernel_i64);
  auto bwd = f64 ? smooth_bwd_kernel_f64 : (narrow ? smooth_bwd_kernel : smooth_bwd_kernel_i64);
  hipStream_t sm = kfh::stream_of(a->stream);
  fwd<<<kfh::grid_for(a->n, 256), 256, 0, sm>>>(a->n, a->ld, a->state_in, a->cov_in, a->charge, a->hit_idx,
                                                a->ld_idx, a->hit_pos, a->hit_cov, a->ldh, a->state_out, a->cov_out,
                                                a->chi2_out, a->nhits_out, a->status_out, ctx->dgeom);
  if (int32_t rc = kfh::check_hip(hipGetLastError(), "smooth_fwd_kernel launch")) return rc;
  bwd<<<kfh::grid_for(a->n, 256), 256, 0, sm>>>(a->n, a->ld, a->charge, a->hit_idx, a->ld_idx, a->state_out,
                                                a->cov_out, a->status_out, ctx->dgeom);
  return kfh::check_hip(hipGetLastError(), "smooth_bwd_kernel launch");
}

}  // extern "C"
