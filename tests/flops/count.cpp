// Counts the floating-point operations of the device Kalman-filter arithmetic
// by compiling it for the host with a counting number type (every + - * / on
// it counts one FLOP; square roots, reciprocal square roots, arctangents and
// logarithms are counted apart).  Built by tests/test_flop_model.py from a
// host copy of kf_device.hpp; prints one "name value" line per quantity.
#include <cstdio>

#include "kf_device_cf.hpp"

using namespace kfd;
static void reset() { cnt_flop = cnt_div = cnt_rsqrt = cnt_atan = cnt_log = cnt_sqrt = 0; }
static void report(const char* what) {
  std::printf("%s %lld %lld %lld\n", what, cnt_flop, cnt_div, cnt_rsqrt + cnt_sqrt + cnt_atan + cnt_log);
  reset();
}
int main() {
  // a track at r = 22 cm crossing to r = 28 cm, a full covariance, a hit near the prediction
  CF s[6] = {CF(20.0), CF(9.0), CF(3.0), CF(1.2), CF(0.9), CF(0.4)};
  CF c[21];
  for (int i = 0; i < 21; ++i) c[i] = CF(1e-6 * (i + 1));
  for (int i = 0; i < 6; ++i) c[tri(i, i)] = CF(1e-3 * (i + 1));
  const CF a = CF(-1.0 * kCLight * 3.8);
  reset();
  if (propagate(s, c, a, CF(28.0), CF(50.0))) return 1;
  report("propagate");
  if (material(s, c, CF(0.02), CF(0.0363), CF(0.13957039))) return 1;
  report("material");
  const float m[3] = {static_cast<float>(s[0].v) + 0.004f, static_cast<float>(s[1].v) - 0.003f,
                      static_cast<float>(s[2].v) + 0.05f};
  const float v[6] = {1e-4f, 0.f, 1e-4f, 0.f, 0.f, 1e-2f};
  const LocalPred<CF> lp = local_pred(s, c);
  report("local_pred");
  CF c2;
  if (chi2_on_layer(s, lp, m, v, c2)) return 1;
  report("chi2");
  CF dc2;
  if (update_on_layer<CF, CF>(s, c, m, v, dc2)) return 1;
  report("update");
  // one smoother step from layer 0 (r = 22 cm) back from layer 1 (r = 28 cm): the filter's step repeated
  // (material, crossing, transport) and the gain
  Geom g{};
  g.n_layers = 2;
  g.r[0] = 22.f;
  g.r[1] = 28.f;
  g.z_half[0] = g.z_half[1] = 50.f;
  g.x_over_x0[0] = g.x_over_x0[1] = 0.02f;
  g.bz = 3.8f;
  g.eloss_per_x0 = 0.0363f;
  g.mass = 0.13957039f;
  float xf[6] = {20.0f, 9.0f, 3.0f, 1.2f, 0.9f, 0.4f}, cf[21];
  const float nx = 20.0f / std::sqrt(481.0f), ny = 9.0f / std::sqrt(481.0f);
  // a covariance with no radial variance at (20, 9): position block along the tangent (-ny, nx) and z
  for (int i = 0; i < 21; ++i) cf[i] = 0.f;
  const float vt = 1e-4f;
  cf[tri(0, 0)] = vt * ny * ny;
  cf[tri(1, 0)] = -vt * nx * ny;
  cf[tri(1, 1)] = vt * nx * nx;
  cf[tri(2, 2)] = 1e-2f;
  for (int i = 3; i < 6; ++i) cf[tri(i, i)] = 1e-4f * (i + 1);
  float xs[6], cs[21];
  {
    CF s2[6], c2[21];
    for (int k = 0; k < 6; ++k) s2[k] = CF(xf[k]);
    for (int k = 0; k < 21; ++k) c2[k] = CF(cf[k]);
    if (material(s2, c2, CF(0.02), CF(0.0363), CF(0.13957039))) return 1;
    if (propagate(s2, c2, a, CF(28.0), CF(0.0))) return 1;
    for (int k = 0; k < 6; ++k) xs[k] = static_cast<float>(s2[k].v) + (k == 2 ? 0.01f : 0.f);
    for (int k = 0; k < 21; ++k) cs[k] = 0.5f * static_cast<float>(c2[k].v);
  }
  reset();
  if (rts_step<CF, CF>(xf, cf, a, g, 0, xs, cs)) return 2;
  report("smooth_step");
  return 0;
}
