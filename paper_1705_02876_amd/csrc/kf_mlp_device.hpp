// kf_mlp_device.hpp -- device side of the search-window network 8 -> 64 -> 64 -> 2
// (ReLU) on the bf16 matrix cores, shared by the training kernels and the
// track builder.
//
// Products run in the orientation features x records with
// v_mfma_f32_16x16x16_bf16: a 16-record tile is the N dimension, the weights
// are the A operand (bf16 tiles, pre-arranged by the pack kernel), the
// activations the B operand.  Register layouts of that instruction (64 lanes):
//   A[i][k]: lane i + 16 (k / 4), element k % 4
//   B[k][j]: lane j + 16 (k / 4), element k % 4
//   D[i][j]: lane j + 16 (i / 4), element i % 4
// so the accumulator tile of one layer is the B operand of the next and the
// forward pass moves no data between layers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kfmi.h"

namespace kfm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 8, kH = 64, kOut = 2;
constexpr int kOffW1 = 0;                            // W1 [64][8]
constexpr int kOffB1 = kOffW1 + kH * kIn;            // 512
constexpr int kOffW2 = kOffB1 + kH;                  // 576
constexpr int kOffB2 = kOffW2 + kH * kH;             // 4672
constexpr int kOffW3 = kOffB2 + kH;                  // 4736
constexpr int kOffB3 = kOffW3 + kOut * kH;           // 4864
static_assert(kOffB3 + kOut == KF_MLP_PARAMS, "parameter count");

// packed buffer: bf16 tiles of 64 lanes x 4 values (512 bytes each), then biases
constexpr int kTileBytes = 512;
constexpr int kPkW1 = 0;                        // 4 tiles   (rows 16mt.., k = input 0..15, 8..15 zero)
constexpr int kPkW2 = kPkW1 + 4 * kTileBytes;   // 16 tiles  (mt, kt)
constexpr int kPkW3 = kPkW2 + 16 * kTileBytes;  // 4 tiles   (rows = outputs 0..15, 2..15 zero; kt)
constexpr int kPkW2T = kPkW3 + 4 * kTileBytes;  // 16 tiles  (W2^T: rows = inputs, k = outputs)
constexpr int kPkW3T = kPkW2T + 16 * kTileBytes;  // 4 tiles (W3^T: rows = hidden 16mt.., k = outputs 0..15)
constexpr int kPkB1 = kPkW3T + 4 * kTileBytes;  // float b1[64]
constexpr int kPkB2 = kPkB1 + 4 * kH;
constexpr int kPkB3 = kPkB2 + 4 * kH;
static_assert(kPkB3 + 4 * kOut == KF_MLP_PACKED_BYTES, "packed size");

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u) return static_cast<uint16_t>((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return static_cast<uint16_t>(u >> 16);
}

// four floats to bfloat16 (round to nearest even) with the packed hardware conversion
__device__ __forceinline__ bf16x4 to_bf16x4(f32x4 v) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  const f32x2 a = {v[0], v[1]}, b = {v[2], v[3]};
  const bf16x2 lo = __builtin_convertvector(a, bf16x2);
  const bf16x2 hi = __builtin_convertvector(b, bf16x2);
  const uint32_t ulo = __builtin_bit_cast(uint32_t, lo), uhi = __builtin_bit_cast(uint32_t, hi);
  bf16x4 r;
  r[0] = static_cast<short>(ulo & 0xFFFFu);
  r[1] = static_cast<short>(ulo >> 16);
  r[2] = static_cast<short>(uhi & 0xFFFFu);
  r[3] = static_cast<short>(uhi >> 16);
  return r;
}

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// One K = 32 product (v_mfma_f32_16x16x32_bf16) standing for two K = 16 products over consecutive K tiles:
// each operand is its two K = 16 lane fragments side by side.  A given (lane group, element) slot then holds the
// same K index in both operands, so the sum is over the same 32 indices, in the hardware's accumulation order.
__device__ __forceinline__ f32x4 mfma32(bf16x4 a0, bf16x4 a1, bf16x4 b0, bf16x4 b1, f32x4 c) {
  typedef short s16x8 __attribute__((ext_vector_type(8)));
  typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
  const s16x8 a = {a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
  const s16x8 b = {b0[0], b0[1], b0[2], b0[3], b1[0], b1[1], b1[2], b1[3]};
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                 0, 0, 0);
}

__device__ __forceinline__ bf16x4 load_tile(const unsigned char* packed, int off, int t, int lane) {
  return reinterpret_cast<const bf16x4*>(packed + off + t * kTileBytes)[lane];
}

struct FwdWeights {
  bf16x4 w1[4], w2[16], w3[4];
  f32x4 b1[4], b2[4], b3;
};

__device__ __forceinline__ void load_fwd(const unsigned char* packed, int lane, FwdWeights& W) {
#pragma unroll
  for (int t = 0; t < 4; ++t) W.w1[t] = load_tile(packed, kPkW1, t, lane);
#pragma unroll
  for (int t = 0; t < 16; ++t) W.w2[t] = load_tile(packed, kPkW2, t, lane);
#pragma unroll
  for (int t = 0; t < 4; ++t) W.w3[t] = load_tile(packed, kPkW3, t, lane);
  const float* fb1 = reinterpret_cast<const float*>(packed + kPkB1);
  const float* fb2 = reinterpret_cast<const float*>(packed + kPkB2);
  const float* fb3 = reinterpret_cast<const float*>(packed + kPkB3);
  const int q = 4 * (lane >> 4);
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      W.b1[mt][e] = fb1[16 * mt + q + e];
      W.b2[mt][e] = fb2[16 * mt + q + e];
    }
#pragma unroll
  for (int e = 0; e < 4; ++e) W.b3[e] = (q + e < kOut) ? fb3[q + e] : 0.f;
}

// Forward pass of one 16-record tile.  xb: B operand (lane l: record l%16,
// features 4(l/16)..+3, zero beyond 8).  Returns the output tile (lanes 0..15:
// elements 0, 1 = log s_t, log s_z of record l) and keeps the hidden tiles.
__device__ __forceinline__ f32x4 forward_tile(const FwdWeights& W, bf16x4 xb, f32x4 h1[4], f32x4 h2[4],
                                              bf16x4 h1b[4], bf16x4 h2b[4]) {
  const f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 a = mfma(W.w1[mt], xb, z);
#pragma unroll
    for (int e = 0; e < 4; ++e) a[e] = fmaxf(a[e] + W.b1[mt][e], 0.f);
    h1[mt] = a;
    h1b[mt] = to_bf16x4(a);
  }
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    f32x4 a = z;
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) a = mfma(W.w2[mt * 4 + kt], h1b[kt], a);
#pragma unroll
    for (int e = 0; e < 4; ++e) a[e] = fmaxf(a[e] + W.b2[mt][e], 0.f);
    h2[mt] = a;
    h2b[mt] = to_bf16x4(a);
  }
  f32x4 o = z;
#pragma unroll
  for (int kt = 0; kt < 4; ++kt) o = mfma(W.w3[kt], h2b[kt], o);
#pragma unroll
  for (int e = 0; e < 4; ++e) o[e] += W.b3[e];
  return o;
}

// One prediction per lane (64 records): features f[8] in, (log s_t, log s_z)
// out.  Must be called by all 64 lanes of the wave together (wave-uniform
// control flow); lanes without a record pass zeros and ignore the result.
__device__ __forceinline__ void eval_wave(const unsigned char* packed, const float f[kIn], int lane, float& o0,
                                          float& o1) {
  FwdWeights W;
  load_fwd(packed, lane, W);
  const int g = lane >> 4;
  o0 = 0.f;
  o1 = 0.f;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int src = 16 * t + (lane & 15);
    f32x4 v;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float lo = __shfl(f[e], src);
      const float hi = __shfl(f[4 + e], src);
      v[e] = g == 0 ? lo : (g == 1 ? hi : 0.f);
    }
    f32x4 h1[4], h2[4];
    bf16x4 h1b[4], h2b[4];
    const f32x4 o = forward_tile(W, to_bf16x4(v), h1, h2, h1b, h2b);
    // lanes 0..15 hold the outputs of records 16 t + lane
    const float r0 = __shfl(o[0], lane & 15);
    const float r1 = __shfl(o[1], lane & 15);
    if (g == t) {
      o0 = r0;
      o1 = r1;
    }
  }
}

// Forward weights staged in LDS for the builder: W1, W2, W3 operand tiles
// (12288 bytes) then b1, b2, b3 (float), copied once per block.
constexpr int kFwdTileBytes = kPkW2T;               // W1, W2, W3 tiles
constexpr int kFwdBytes = kFwdTileBytes + 4 * (2 * kH + kOut);
constexpr int kLdsB1 = kFwdTileBytes, kLdsB2 = kLdsB1 + 4 * kH, kLdsB3 = kLdsB2 + 4 * kH;

// block-cooperative copy (all threads of the block, then a block barrier)
__device__ __forceinline__ void stage_forward(const unsigned char* __restrict__ packed, unsigned char* lds) {
  for (int i = threadIdx.x; i < kFwdTileBytes / 16; i += blockDim.x)
    reinterpret_cast<uint4*>(lds)[i] = reinterpret_cast<const uint4*>(packed)[i];
  for (int i = threadIdx.x; i < 2 * kH + kOut; i += blockDim.x)
    reinterpret_cast<float*>(lds + kFwdTileBytes)[i] = reinterpret_cast<const float*>(packed + kPkB1)[i];
  __syncthreads();
}

// eval_wave with the weights read from LDS right before each product, so that
// only one record tile's activations are live at a time, and only for the
// lanes that hold a record: `src` maps compacted record k < n to its lane (a
// per-wave LDS table), `pos` is this lane's compacted index (or -1).  Tiles
// past n records are skipped, so a wave with few live candidates pays for few
// products.  The 64-wide layers use K = 32 products (14 per record tile
// instead of 24).
__device__ __forceinline__ void eval_compact_lds(const unsigned char* lds, const float f[kIn], int lane,
                                                 const int32_t* src_lane, int n, int pos, float& o0, float& o1) {
  const int g = lane >> 4, q = 4 * g;
  const float* b1 = reinterpret_cast<const float*>(lds + kLdsB1);
  const float* b2 = reinterpret_cast<const float*>(lds + kLdsB2);
  const float* b3 = reinterpret_cast<const float*>(lds + kLdsB3);
  o0 = 0.f;
  o1 = 0.f;
  const f32x4 z = {0.f, 0.f, 0.f, 0.f};
  const int tiles = (n + 15) >> 4;
#pragma unroll 1
  for (int t = 0; t < tiles; ++t) {
    int woff = 0;
    asm volatile("" : "+v"(woff));  // keeps the weight reads inside this loop
    const unsigned char* wl = lds + woff;
    const int k = 16 * t + (lane & 15);
    const int src = k < n ? src_lane[k] : 0;
    f32x4 v;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float lo = __shfl(f[e], src);
      const float hi = __shfl(f[4 + e], src);
      v[e] = (k < n) ? (g == 0 ? lo : (g == 1 ? hi : 0.f)) : 0.f;
    }
    const bf16x4 xb = to_bf16x4(v);
    bf16x4 h1b[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 a = mfma(load_tile(wl, kPkW1, mt, lane), xb, z);
#pragma unroll
      for (int e = 0; e < 4; ++e) a[e] = fmaxf(a[e] + b1[16 * mt + q + e], 0.f);
      h1b[mt] = to_bf16x4(a);
    }
    bf16x4 h2b[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 a = z;
#pragma unroll
      for (int kt = 0; kt < 4; kt += 2)
        a = mfma32(load_tile(wl, kPkW2, mt * 4 + kt, lane), load_tile(wl, kPkW2, mt * 4 + kt + 1, lane), h1b[kt],
                   h1b[kt + 1], a);
#pragma unroll
      for (int e = 0; e < 4; ++e) a[e] = fmaxf(a[e] + b2[16 * mt + q + e], 0.f);
      h2b[mt] = to_bf16x4(a);
    }
    f32x4 o = z;
#pragma unroll
    for (int kt = 0; kt < 4; kt += 2)
      o = mfma32(load_tile(wl, kPkW3, kt, lane), load_tile(wl, kPkW3, kt + 1, lane), h2b[kt], h2b[kt + 1], o);
    // record 16 t + j's outputs sit in lane j; its owner has compacted index 16 t + j
    const int from = pos >= 0 ? (pos & 15) : 0;
    const float r0 = __shfl(o[0] + b3[0], from);
    const float r1 = __shfl(o[1] + b3[1], from);
    if (pos >= 0 && (pos >> 4) == t) {
      o0 = r0;
      o1 = r1;
    }
  }
}

// all 64 lanes hold a record
__device__ __forceinline__ void eval_wave_lds(const unsigned char* lds, const float f[kIn], int lane, float& o0,
                                              float& o1) {
  const int g = lane >> 4, q = 4 * g;
  const float* b1 = reinterpret_cast<const float*>(lds + kLdsB1);
  const float* b2 = reinterpret_cast<const float*>(lds + kLdsB2);
  const float* b3 = reinterpret_cast<const float*>(lds + kLdsB3);
  o0 = 0.f;
  o1 = 0.f;
  const f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
  for (int t = 0; t < 4; ++t) {
    int woff = 0;
    asm volatile("" : "+v"(woff));  // keeps the weight reads inside this loop
    const unsigned char* wl = lds + woff;
    const int src = 16 * t + (lane & 15);
    f32x4 v;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float lo = __shfl(f[e], src);
      const float hi = __shfl(f[4 + e], src);
      v[e] = g == 0 ? lo : (g == 1 ? hi : 0.f);
    }
    const bf16x4 xb = to_bf16x4(v);
    bf16x4 h1b[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 a = mfma(load_tile(wl, kPkW1, mt, lane), xb, z);
#pragma unroll
      for (int e = 0; e < 4; ++e) a[e] = fmaxf(a[e] + b1[16 * mt + q + e], 0.f);
      h1b[mt] = to_bf16x4(a);
    }
    bf16x4 h2b[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 a = z;
#pragma unroll
      for (int kt = 0; kt < 4; ++kt) a = mfma(load_tile(wl, kPkW2, mt * 4 + kt, lane), h1b[kt], a);
#pragma unroll
      for (int e = 0; e < 4; ++e) a[e] = fmaxf(a[e] + b2[16 * mt + q + e], 0.f);
      h2b[mt] = to_bf16x4(a);
    }
    f32x4 o = z;
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) o = mfma(load_tile(wl, kPkW3, kt, lane), h2b[kt], o);
    const float r0 = __shfl(o[0] + b3[0], lane & 15);
    const float r1 = __shfl(o[1] + b3[1], lane & 15);
    if (g == t) {
      o0 = r0;
      o1 = r1;
    }
  }
}

}  // namespace kfm
