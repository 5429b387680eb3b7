// kf_mlp.hip -- learned search-window network on the gfx950 matrix cores.
//
// Network 8 -> 64 -> 64 -> 2 (ReLU), computed in the orientation
// features x records with v_mfma_f32_16x16x16_bf16: a 16-record tile is the N
// dimension of every product, weights are the A operand (kept in registers as
// bf16 tiles), activations the B operand.  In this instruction's register
// layout the accumulator tile of one layer is exactly the B-operand tile of
// the next (lane l holds rows 4(l/16)..+3 of column l%16), so the forward pass
// moves no data between layers.  Backward products that contract over
// features reuse the transposed weight tiles the same way; the weight
// gradients contract over records, so their operands go through LDS once per
// tile.  Partial gradients of a fixed set of waves are reduced in a fixed
// order (deterministic).
#include <hip/hip_runtime.h>

#include <cmath>

#include "kf_internal.hpp"
#include "kf_mlp_device.hpp"

namespace {

using namespace kfm;

constexpr int kGradWaves = 1024;
constexpr int kPartial = KF_MLP_PARAMS + 2;  // + loss, count

// parameter feeding element e of lane `lane` in tile t of each packed block
__device__ float packed_source(const float* P, int block, int t, int lane, int e) {
  const int r = lane & 15, kq = 4 * (lane >> 4) + e;
  switch (block) {
    case 0:  // W1: row 16t + r, input kq
      return kq < kIn ? P[kOffW1 + (16 * t + r) * kIn + kq] : 0.f;
    case 1: {  // W2: tile t = mt*4+kt, row 16mt + r, col 16kt + kq
      const int mt = t >> 2, kt = t & 3;
      return P[kOffW2 + (16 * mt + r) * kH + 16 * kt + kq];
    }
    case 2:  // W3: tile kt, row (output) r, col 16kt + kq
      return r < kOut ? P[kOffW3 + r * kH + 16 * t + kq] : 0.f;
    case 3: {  // W2^T: tile t = mt*4+kt, row 16mt + r (input), col 16kt + kq (output) = W2[16kt+kq][16mt+r]
      const int mt = t >> 2, kt = t & 3;
      return P[kOffW2 + (16 * kt + kq) * kH + 16 * mt + r];
    }
    default:  // W3^T: tile mt, row 16mt + r (hidden), col kq (output) = W3[kq][16mt + r]
      return kq < kOut ? P[kOffW3 + kq * kH + 16 * t + r] : 0.f;
  }
}

__global__ void __launch_bounds__(256) pack_kernel(const float* __restrict__ P, unsigned char* __restrict__ packed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  constexpr int nval = (4 + 16 + 4 + 16 + 4) * 64 * 4;
  if (i < nval) {
    const int e = i & 3, lane = (i >> 2) & 63, tile = i >> 8;
    int block, t;
    if (tile < 4) { block = 0; t = tile; }
    else if (tile < 20) { block = 1; t = tile - 4; }
    else if (tile < 24) { block = 2; t = tile - 20; }
    else if (tile < 40) { block = 3; t = tile - 24; }
    else { block = 4; t = tile - 40; }
    reinterpret_cast<uint16_t*>(packed)[i] = f2bf(packed_source(P, block, t, lane, e));
  } else if (i < nval + kH + kH + kOut) {
    const int j = i - nval;
    float* fb = reinterpret_cast<float*>(packed + kPkB1);
    fb[j] = j < kH ? P[kOffB1 + j] : (j < 2 * kH ? P[kOffB2 + j - kH] : P[kOffB3 + j - 2 * kH]);
  }
}

__device__ __forceinline__ bf16x4 load_x_tile(const float* __restrict__ x, int64_t ldx, int64_t rec, bool valid,
                                              int lane) {
  const int q = 4 * (lane >> 4);
  f32x4 v = {0.f, 0.f, 0.f, 0.f};
  if (valid && q < kIn) {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = x[(q + e) * ldx + rec];
  }
  return to_bf16x4(v);
}

__global__ void __launch_bounds__(256) forward_kernel(int64_t n, const float* __restrict__ x, int64_t ldx,
                                                      const unsigned char* __restrict__ packed, float* __restrict__ y,
                                                      int64_t ldy) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  FwdWeights W;
  load_fwd(packed, lane, W);
  for (int64_t base = wave * 16; base < n; base += nwaves * 16) {
    const int64_t rec = base + (lane & 15);
    const bool valid = rec < n;
    const bf16x4 xb = load_x_tile(x, ldx, rec, valid, lane);
    f32x4 h1[4], h2[4];
    bf16x4 h1b[4], h2b[4];
    const f32x4 o = forward_tile(W, xb, h1, h2, h1b, h2b);
    if (valid && lane < 16) {
      y[rec] = o[0];
      y[ldy + rec] = o[1];
    }
  }
}

// LDS staging of one wave's tile, feature-major with the 16 records contiguous
struct alignas(16) GradLds {
  uint16_t da2[kH][16], da1[kH][16], h1[kH][16], h2[kH][16], x[16][16], dout[16][16];
};

__device__ __forceinline__ void stage_tile(uint16_t (*S)[16], int mt, f32x4 v, int lane) {
  const int row = 16 * mt + 4 * (lane >> 4), col = lane & 15;
  const bf16x4 b = to_bf16x4(v);
#pragma unroll
  for (int e = 0; e < 4; ++e) S[row + e][col] = static_cast<uint16_t>(b[e]);
}

// operand with rows 16*tile + l%16 and the 4 records 4(l/16).. from an LDS block
__device__ __forceinline__ bf16x4 lds_operand(const uint16_t (*S)[16], int tile, int lane) {
  return *reinterpret_cast<const bf16x4*>(&S[16 * tile + (lane & 15)][4 * (lane >> 4)]);
}

__global__ void __launch_bounds__(256) grad_kernel(int64_t n, const float* __restrict__ x, int64_t ldx,
                                                   const float* __restrict__ t, int64_t ldt,
                                                   const unsigned char* __restrict__ packed,
                                                   float* __restrict__ partial) {
  __shared__ GradLds lds_all[4];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  GradLds& S = lds_all[wv];
  const int64_t wave = static_cast<int64_t>(blockIdx.x) * 4 + wv;  // 0 .. kGradWaves-1
  const int64_t per = ((n + kGradWaves - 1) / kGradWaves + 15) / 16 * 16;
  const int64_t r0 = wave * per;
  const int64_t r1 = (r0 + per < n) ? r0 + per : n;
  FwdWeights W;
  load_fwd(packed, lane, W);
  bf16x4 w2t[16], w3t[4];
#pragma unroll
  for (int k = 0; k < 16; ++k) w2t[k] = load_tile(packed, kPkW2T, k, lane);
#pragma unroll
  for (int k = 0; k < 4; ++k) w3t[k] = load_tile(packed, kPkW3T, k, lane);
  const f32x4 z = {0.f, 0.f, 0.f, 0.f};
  f32x4 gw1[4], gw2[16], gw3[4];
  f32x4 gb1[4], gb2[4], gb3 = z;
#pragma unroll
  for (int k = 0; k < 4; ++k) gw1[k] = gw3[k] = gb1[k] = gb2[k] = z;
#pragma unroll
  for (int k = 0; k < 16; ++k) gw2[k] = z;
  float loss = 0.f, count = 0.f;
  for (int64_t base = r0; base < r1; base += 16) {
    const int64_t rec = base + (lane & 15);
    bool valid = rec < r1;
    float tt0 = 0.f, tt1 = 0.f;
    if (valid) {
      tt0 = t[rec];
      tt1 = t[ldt + rec];
      bool fin = isfinite(tt0) && isfinite(tt1);
#pragma unroll
      for (int f = 0; f < kIn; ++f) fin = fin && isfinite(x[f * ldx + rec]);
      valid = fin;  // records with a non-finite entry are skipped
    }
    const bf16x4 xb = load_x_tile(x, ldx, rec, valid, lane);
    f32x4 h1[4], h2[4];
    bf16x4 h1b[4], h2b[4];
    const f32x4 o = forward_tile(W, xb, h1, h2, h1b, h2b);
    // d loss / d output (only lanes 0..15, elements 0 and 1 are real outputs)
    f32x4 dout = z;
    if (lane < 16 && valid) {
      const float e0 = __expf(-2.f * o[0]), e1 = __expf(-2.f * o[1]);
      dout[0] = 1.f - tt0 * tt0 * e0;
      dout[1] = 1.f - tt1 * tt1 * e1;
      loss += 0.5f * tt0 * tt0 * e0 + o[0] + 0.5f * tt1 * tt1 * e1 + o[1];
      count += 1.f;
    }
    const bf16x4 doutb = to_bf16x4(dout);
    // back through layer 3 and 2 (contract over features: weights^T as A operand)
    f32x4 da2[4];
    bf16x4 da2b[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 a = mfma(w3t[mt], doutb, z);
#pragma unroll
      for (int e = 0; e < 4; ++e) a[e] = h2[mt][e] > 0.f ? a[e] : 0.f;
      da2[mt] = a;
      da2b[mt] = to_bf16x4(a);
    }
    f32x4 da1[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 a = z;
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) a = mfma(w2t[mt * 4 + kt], da2b[kt], a);
#pragma unroll
      for (int e = 0; e < 4; ++e) a[e] = h1[mt][e] > 0.f ? a[e] : 0.f;
      da1[mt] = a;
    }
    // bias gradients: per-lane sums over this lane's record
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      gb1[mt] += da1[mt];
      gb2[mt] += da2[mt];
    }
    gb3 += dout;
    // weight gradients contract over the 16 records: stage feature-major in LDS
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      stage_tile(S.da2, mt, da2[mt], lane);
      stage_tile(S.da1, mt, da1[mt], lane);
      stage_tile(S.h1, mt, h1[mt], lane);
      stage_tile(S.h2, mt, h2[mt], lane);
    }
    {
      f32x4 xv = z;
      const int q = 4 * (lane >> 4);
      if (valid && q < kIn)
#pragma unroll
        for (int e = 0; e < 4; ++e) xv[e] = x[(q + e) * ldx + rec];
      stage_tile(S.x, 0, xv, lane);
      stage_tile(S.dout, 0, dout, lane);
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wave's LDS writes are done
    __builtin_amdgcn_wave_barrier();
    // dW2[out][in] += sum_r da2[out][r] h1[in][r]
#pragma unroll
    for (int mo = 0; mo < 4; ++mo) {
      const bf16x4 a = lds_operand(S.da2, mo, lane);
#pragma unroll
      for (int ni = 0; ni < 4; ++ni) gw2[mo * 4 + ni] = mfma(a, lds_operand(S.h1, ni, lane), gw2[mo * 4 + ni]);
    }
    // dW1[out][in] += sum_r da1[out][r] x[in][r]
    {
      const bf16x4 bx = lds_operand(S.x, 0, lane);
#pragma unroll
      for (int mo = 0; mo < 4; ++mo) gw1[mo] = mfma(lds_operand(S.da1, mo, lane), bx, gw1[mo]);
    }
    // dW3[out][in] += sum_r dout[out][r] h2[in][r]
    {
      const bf16x4 ad = lds_operand(S.dout, 0, lane);
#pragma unroll
      for (int ni = 0; ni < 4; ++ni) gw3[ni] = mfma(ad, lds_operand(S.h2, ni, lane), gw3[ni]);
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
  }
  // write this wave's partial sums (accumulator tile: rows 4(l/16)+e, column l%16)
  float* out = partial + wave * kPartial;
  const int q = 4 * (lane >> 4), c = lane & 15;
#pragma unroll
  for (int mo = 0; mo < 4; ++mo)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (c < kIn) out[kOffW1 + (16 * mo + q + e) * kIn + c] = gw1[mo][e];
#pragma unroll
      for (int ni = 0; ni < 4; ++ni) out[kOffW2 + (16 * mo + q + e) * kH + 16 * ni + c] = gw2[mo * 4 + ni][e];
    }
#pragma unroll
  for (int ni = 0; ni < 4; ++ni)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (q + e < kOut) out[kOffW3 + (q + e) * kH + 16 * ni + c] = gw3[ni][e];
  // bias sums: reduce over the 16 lanes that share l/16
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float s1 = gb1[mt][e], s2 = gb2[mt][e];
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        s1 += __shfl_xor(s1, off);
        s2 += __shfl_xor(s2, off);
      }
      if (c == 0) {
        out[kOffB1 + 16 * mt + q + e] = s1;
        out[kOffB2 + 16 * mt + q + e] = s2;
      }
    }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    float s3 = gb3[e];
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) s3 += __shfl_xor(s3, off);
    if (c == 0 && q + e < kOut) out[kOffB3 + q + e] = s3;
  }
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    loss += __shfl_xor(loss, off);
    count += __shfl_xor(count, off);
  }
  if (lane == 0) {
    out[KF_MLP_PARAMS] = loss;
    out[KF_MLP_PARAMS + 1] = count;
  }
}

__global__ void __launch_bounds__(256) reduce_kernel(const float* __restrict__ partial, float* __restrict__ grad,
                                                     float* __restrict__ loss, float* __restrict__ count) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kPartial) return;
  double cnt = 0.0;
  for (int w = 0; w < kGradWaves; ++w) cnt += partial[w * kPartial + KF_MLP_PARAMS + 1];
  double s = 0.0;
  for (int w = 0; w < kGradWaves; ++w) s += partial[w * kPartial + p];
  const double inv = cnt > 0.0 ? 1.0 / cnt : 0.0;
  if (p < KF_MLP_PARAMS) grad[p] = static_cast<float>(s * inv);
  else if (p == KF_MLP_PARAMS) loss[0] = static_cast<float>(s * inv);
  else if (count) count[0] = static_cast<float>(cnt);
}

__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ P, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                                   float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= KF_MLP_PARAMS) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

constexpr int kPackThreads = (4 + 16 + 4 + 16 + 4) * 64 * 4 + 2 * kH + kOut;

}  // namespace

using kfh::set_error;

extern "C" {

int32_t kf_mlp_pack(kf_ctx* ctx, const float* params, void* packed, void* stream) {
  if (int32_t rc = kfh::enter(ctx)) return rc;
  if (!params || !packed) return set_error(KF_ERR_INVALID_ARG, "null array");
  pack_kernel<<<(kPackThreads + 255) / 256, 256, 0, kfh::stream_of(stream)>>>(
      params, static_cast<unsigned char*>(packed));
  return kfh::check_hip(hipGetLastError(), "mlp pack launch");
}

int32_t kf_mlp_forward(kf_ctx* ctx, int64_t n, const float* x, int64_t ldx, const void* packed, float* y, int64_t ldy,
                       void* stream) {
  if (int32_t rc = kfh::enter(ctx)) return rc;
  if (n < 0 || ldx < n || ldy < n) return set_error(KF_ERR_INVALID_ARG, "bad sizes");
  if (n == 0) return KF_OK;
  if (!x || !packed || !y) return set_error(KF_ERR_INVALID_ARG, "null array");
  const int64_t tiles = (n + 15) / 16;
  const int64_t waves = tiles < 4096 ? tiles : 4096;
  forward_kernel<<<static_cast<unsigned>((waves + 3) / 4), 256, 0, kfh::stream_of(stream)>>>(
      n, x, ldx, static_cast<const unsigned char*>(packed), y, ldy);
  return kfh::check_hip(hipGetLastError(), "mlp forward launch");
}

size_t kf_mlp_grad_workspace_size(void) { return static_cast<size_t>(kGradWaves) * kPartial * sizeof(float); }

int32_t kf_mlp_grad(kf_ctx* ctx, int64_t n, const float* x, int64_t ldx, const float* t, int64_t ldt,
                    const void* packed, float* grad, float* loss, float* count, void* workspace,
                    size_t workspace_bytes, void* stream) {
  if (int32_t rc = kfh::enter(ctx)) return rc;
  if (n < 0 || ldx < n || ldt < n) return set_error(KF_ERR_INVALID_ARG, "bad sizes");
  if (!x || !t || !packed || !grad || !loss) return set_error(KF_ERR_INVALID_ARG, "null array");
  if (!workspace || workspace_bytes < kf_mlp_grad_workspace_size())
    return set_error(KF_ERR_WORKSPACE, "workspace of %zu bytes needed", kf_mlp_grad_workspace_size());
  hipStream_t s = kfh::stream_of(stream);
  float* part = static_cast<float*>(workspace);
  grad_kernel<<<kGradWaves / 4, 256, 0, s>>>(n, x, ldx, t, ldt, static_cast<const unsigned char*>(packed), part);
  if (int32_t rc = kfh::check_hip(hipGetLastError(), "mlp grad launch")) return rc;
  reduce_kernel<<<(kPartial + 255) / 256, 256, 0, s>>>(part, grad, loss, count);
  return kfh::check_hip(hipGetLastError(), "mlp reduce launch");
}

int32_t kf_mlp_adam(kf_ctx* ctx, float* params, const float* grad, float* m, float* v, int32_t step, float lr,
                    float beta1, float beta2, float eps, void* packed, void* stream) {
  if (int32_t rc = kfh::enter(ctx)) return rc;
  if (!params || !grad || !m || !v || !packed) return set_error(KF_ERR_INVALID_ARG, "null array");
  if (step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return set_error(KF_ERR_INVALID_ARG, "bad Adam hyper-parameters");
  hipStream_t s = kfh::stream_of(stream);
  const float c1 = 1.f - powf(beta1, static_cast<float>(step));
  const float c2 = 1.f - powf(beta2, static_cast<float>(step));
  adam_kernel<<<(KF_MLP_PARAMS + 255) / 256, 256, 0, s>>>(params, grad, m, v, lr, beta1, beta2, eps, c1, c2);
  if (int32_t rc = kfh::check_hip(hipGetLastError(), "adam launch")) return rc;
  return kf_mlp_pack(ctx, params, packed, stream);
}

}  // extern "C"
