// kf_build.hip -- hit binning and combinatorial track building on gfx950.
//
// Binning: one 1024-thread workgroup per (event, layer).  Each of its 16
// waves owns a contiguous slice of the layer's hits: it computes their bins
// (double precision, the decision the oracle takes too), counts them in its
// own LDS histogram, and after a block-wide prefix over (bin, wave) scatters
// its slice in order, ranking equal bins inside a 64-hit chunk with ballots.
// The result is a stable counting sort with no global atomics.
//
// Building: one wave holds 64/G seeds and G >= max_cands lanes per seed, one
// lane per candidate slot.  All layers of a tile run inside the kernel with
// the candidates in registers: propagate, window, scan the window's bins
// (box pre-test, then chi2), keep a per-candidate sorted list of its best
// max_cands children, merge the lists of a seed with G-lane reductions of a
// 64-bit rank key, and update only the survivors (clone engine).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstring>
#include <type_traits>

#include "kf_internal.hpp"
#include "kf_mlp_device.hpp"

using namespace kfd;

namespace {

constexpr int kBinWaves = 16;
constexpr int kBinThreads = kBinWaves * 64;
constexpr int kMaxBins = 2048;         // per-wave histogram binning (bin_kernel)
constexpr int kMaxBinsFine = 32768;    // one-histogram binning (bin_fine_kernel)
constexpr uint32_t kHole = 0xFFFFFFu;
constexpr int kScanUnroll = 4;                  // work items per lane and scan iteration
constexpr int kQueueCap = 64 + 64 * kScanUnroll;  // box-passing (candidate, slot) pairs awaiting their chi2
constexpr int kQueueDefer = 256;                  // learned window: pairs outside the learned box, deferred
constexpr int kXcds = 8;                          // accelerator dies of the device (work-queue chunks)
constexpr int kXcdRun = 256;                      // tiled launch: consecutive blocks given to one die
constexpr int kRangeChunk = 4;                    // slot ranges per candidate flattened together
constexpr int kSerialMax = 8;                     // serial-candidate build: candidates per seed (max_cands <= 8)

// Inclusive prefix sum (Max false) or maximum (Max true) over the wave's 64 lanes from DPP lane moves, with no
// LDS traffic: shifts by 1, 2, 4 and 8 within each row of 16 lanes, then the rows joined by broadcasting lanes 15
// and 31 to the rows after them.  Lanes shifted in from outside a row read 0, the identity of both (maxima are
// taken of non-negative values).  All lanes of the wave take part.
template <bool Max>
__device__ __forceinline__ int wave_incl_scan(int x) {
  auto op = [](int a, int b) { return Max ? max(a, b) : a + b; };
  x = op(x, __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, true));   // row_shr:1
  x = op(x, __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, true));   // row_shr:2
  x = op(x, __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, true));   // row_shr:4
  x = op(x, __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, true));   // row_shr:8
  x = op(x, __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false));  // row_bcast:15 into rows 1 and 3
  x = op(x, __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false));  // row_bcast:31 into rows 2 and 3
  return x;
}

__device__ __forceinline__ int hit_bin(float xf, float yf, float zf, double R, double zh, int n_phi, int n_eta) {
#pragma clang fp contract(off)
  const double phi = atan2(static_cast<double>(yf), static_cast<double>(xf));
  int ip = static_cast<int>(floor((phi + M_PI) * static_cast<double>(n_phi) / (2.0 * M_PI)));
  ip = ip < 0 ? 0 : (ip > n_phi - 1 ? n_phi - 1 : ip);
  const double eta = asinh(static_cast<double>(zf) / R);
  const double emax = asinh(zh / R);
  int ie = static_cast<int>(floor((eta + emax) * static_cast<double>(n_eta) / (2.0 * emax)));
  ie = ie < 0 ? 0 : (ie > n_eta - 1 ? n_eta - 1 : ie);
  return ie * n_phi + ip;
}

// asinh from the hardware base-2 logarithm and square root (each within about an ulp), for the hit binning's
// single-precision estimate and the build window's eta rows: both need it only to a few parts in a million and
// allow for more, and the library's asinhf takes five times the instructions.
__device__ __forceinline__ float asinh_hw(float x) {
  const float a = fabsf(x);
  const float l2 = __builtin_amdgcn_logf(a + __builtin_amdgcn_sqrtf(fmaf(a, a, 1.f)));
  return copysignf(l2 * 0.693147180559945309f, x);
}

// Bin of a hit from single-precision phi and eta, falling back to hit_bin's double-precision definition only
// where a bin edge lies within the single-precision error of the point.  The bounds taken (phi within 6 ulp of
// atan2f plus the rounding of the sum and product, eta within 2.5e-6 (1 + |eta|) from the hardware logarithm,
// both in bin units, with a factor of two to three to spare) exceed the single-precision error, so the bin is
// hit_bin's in every case; a few hits in a thousand take the double-precision path.
struct BinScale {
  float phi_scale, eta_scale, emax, inv_r;  // n_phi / 2 pi, n_eta / 2 emax, emax = asinh(z_half / R), 1 / R
  float dphi, deta0, deta1;                 // error bounds in bin units: dphi, and deta0 + deta1 |eta|
};

__device__ __forceinline__ BinScale bin_scale(double R, double zh, int n_phi, int n_eta) {
  BinScale s;
  const double emax = asinh(zh / R);
  s.phi_scale = static_cast<float>(static_cast<double>(n_phi) / (2.0 * M_PI));
  s.eta_scale = static_cast<float>(static_cast<double>(n_eta) / (2.0 * emax));
  s.emax = static_cast<float>(emax);
  s.inv_r = static_cast<float>(1.0 / R);
  s.dphi = 1e-6f * static_cast<float>(n_phi) + 1e-6f;
  s.deta0 = 5e-6f * s.eta_scale + 1e-6f * static_cast<float>(n_eta) + 1e-6f;
  s.deta1 = 5e-6f * s.eta_scale;
  return s;
}

__device__ __forceinline__ int hit_bin_fast(float x, float y, float z, const BinScale& s, double R, double zh,
                                            int n_phi, int n_eta) {
  const float tp = (atan2f(y, x) + 3.14159265358979f) * s.phi_scale;
  const float eta = asinh_hw(z * s.inv_r);
  const float te = (eta + s.emax) * s.eta_scale;
  const float de = s.deta0 + s.deta1 * fabsf(eta);
  const float pm = static_cast<float>(n_phi - 1), em = static_cast<float>(n_eta - 1);
  const float p0 = fminf(fmaxf(floorf(tp - s.dphi), 0.f), pm), p1 = fminf(fmaxf(floorf(tp + s.dphi), 0.f), pm);
  const float e0 = fminf(fmaxf(floorf(te - de), 0.f), em), e1 = fminf(fmaxf(floorf(te + de), 0.f), em);
  if (fabsf(tp) < 1e30f && fabsf(te) < 1e30f && p0 == p1 && e0 == e1)
    return static_cast<int>(e0) * n_phi + static_cast<int>(p0);
  return hit_bin(x, y, z, R, zh, n_phi, n_eta);
}

// Launch order of the binning blocks: (event, layer) pairs by decreasing hit count (ties by index), so that
// the largest pairs start first and the small ones fill in behind them (event sizes span a factor of 50; in
// index order a large pair starting late holds the whole launch).  One block; the rank of each pair is counted
// against every other pair, staged in LDS.  The result of the binning does not depend on the order.
// kOrderThreads pairs per block, one per thread, the blocks on as many compute units (a single block had taken
// 56 us, a twentieth of the binning, for 1088 pairs).
constexpr int kOrderMax = 8192;
constexpr int kOrderThreads = 256;
__global__ void __launch_bounds__(kOrderThreads) el_order_kernel(int32_t n_el,
                                                                 const int64_t* __restrict__ layer_offsets,
                                                                 int32_t* __restrict__ el_order) {
  __shared__ int32_t sz[kOrderMax];
  for (int e = threadIdx.x; e < n_el; e += blockDim.x)
    sz[e] = static_cast<int32_t>(layer_offsets[e + 1] - layer_offsets[e]);
  __syncthreads();
  const int e = static_cast<int>(blockIdx.x) * kOrderThreads + static_cast<int>(threadIdx.x);
  if (e >= n_el) return;
  const int32_t v = sz[e];
  int rank = 0;
#pragma unroll 4
  for (int f = 0; f < n_el; ++f) {
    const int32_t w = sz[f];  // the same address in every lane: a broadcast read
    rank += static_cast<int>((w > v) | ((w == v) & (f < e)));
  }
  el_order[rank] = e;
}

__global__ void __launch_bounds__(kBinThreads) bin_kernel(int32_t L, const int64_t* __restrict__ layer_offsets,
                                                          const float* __restrict__ hit_pos,
                                                          const float* __restrict__ hit_cov, int64_t ldh,
                                                          int32_t n_phi, int32_t n_eta, Geom g,
                                                          int32_t* __restrict__ bins, int32_t* __restrict__ bin_offsets,
                                                          int32_t* __restrict__ perm, float* __restrict__ binned,
                                                          float* __restrict__ layer_vmax,
                                                          const int32_t* __restrict__ el_order) {
  // per-wave bin counters [kBinWaves][nb] and bin totals [nb], sized by the launch (dynamic LDS) so that
  // a 64 x 16 binning takes 68 KB and two blocks share a compute unit
  extern __shared__ int32_t bin_lds[];
  const int nb_ = n_phi * n_eta;
  int32_t* const cnt_flat = bin_lds;
  int32_t* const tot = bin_lds + kBinWaves * nb_;
#define cnt(w, b) cnt_flat[(w) * nb_ + (b)]
  __shared__ int32_t wsum[kBinWaves];
  __shared__ uint32_t vmax_bits[2];
  const int el = el_order ? el_order[blockIdx.x] : static_cast<int>(blockIdx.x);
  const int l = el % L;
  const int nb = n_phi * n_eta;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int64_t lo = layer_offsets[el], hi = layer_offsets[el + 1];
  const int64_t nh = hi - lo;
  for (int i = tid; i < kBinWaves * nb; i += kBinThreads) cnt(i / nb, i % nb) = 0;
  if (tid < 2) vmax_bits[tid] = 0u;
  __syncthreads();
  // this wave's contiguous slice
  const int64_t per = (nh + kBinWaves - 1) / kBinWaves;
  const int64_t a = lo + per * wave;
  const int64_t b = (a + per < hi) ? a + per : hi;
  const double R = static_cast<double>(g.r[l]);
  const double zh = static_cast<double>(g.z_half[l]);
  const BinScale bs = bin_scale(R, zh, n_phi, n_eta);
  float my_vxy = 0.f, my_vz = 0.f;
  for (int64_t h = a + lane; h < b; h += 64) {
    const int bin = hit_bin_fast(hit_pos[h], hit_pos[ldh + h], hit_pos[2 * ldh + h], bs, R, zh, n_phi, n_eta);
    bins[h] = bin;
    atomicAdd(&cnt(wave, bin), 1);
    const float vxx = hit_cov[h], vyx = hit_cov[ldh + h], vyy = hit_cov[2 * ldh + h], vzz = hit_cov[5 * ldh + h];
    const float d = 0.5f * (vxx - vyy);
    my_vxy = fmaxf(my_vxy, 0.5f * (vxx + vyy) + sqrtf(d * d + vyx * vyx));
    my_vz = fmaxf(my_vz, vzz);
  }
  atomicMax(&vmax_bits[0], __float_as_uint(my_vxy));  // non-negative floats order like their bits
  atomicMax(&vmax_bits[1], __float_as_uint(my_vz));
  __syncthreads();
  // per bin: exclusive prefix over waves, bin totals
  for (int bin = tid; bin < nb; bin += kBinThreads) {
    int run = 0;
#pragma unroll
    for (int w = 0; w < kBinWaves; ++w) {
      const int c = cnt(w, bin);
      cnt(w, bin) = run;
      run += c;
    }
    tot[bin] = run;
  }
  __syncthreads();
  // exclusive scan of the bin totals (each wave scans a contiguous block of bins)
  const int per_w = (nb + kBinWaves - 1) / kBinWaves;
  const int b0 = wave * per_w;
  const int b1 = (b0 + per_w < nb) ? b0 + per_w : nb;
  int wrun = 0;
  for (int base = b0; base < b1; base += 64) {
    const int bin = base + lane;
    int v = (bin < b1) ? tot[bin] : 0;
    const int x = wave_incl_scan<false>(v);
    if (bin < b1) tot[bin] = wrun + x - v;  // exclusive within this wave's block
    wrun += __builtin_amdgcn_readlane(x, 63);
  }
  if (lane == 0) wsum[wave] = wrun;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int w = 0; w < kBinWaves; ++w) {
      const int c = wsum[w];
      wsum[w] = run;
      run += c;
    }
  }
  __syncthreads();
  int32_t* bo = bin_offsets + static_cast<int64_t>(el) * (nb + 1);
  for (int bin = tid; bin < nb; bin += kBinThreads) {
    const int off = tot[bin] + wsum[bin / per_w];
    tot[bin] = off;
    bo[bin] = static_cast<int32_t>(lo + off);
  }
  if (tid == 0) {
    bo[nb] = static_cast<int32_t>(hi);
    layer_vmax[2 * el] = __uint_as_float(vmax_bits[0]);
    layer_vmax[2 * el + 1] = __uint_as_float(vmax_bits[1]);
  }
  __syncthreads();
  for (int bin = tid; bin < nb; bin += kBinThreads) {
    const int base = tot[bin];
#pragma unroll
    for (int w = 0; w < kBinWaves; ++w) cnt(w, bin) += base;
  }
  __syncthreads();
  // stable scatter of this wave's slice, 64 hits at a time, in index order
  int nbits = 0;
  while ((1 << nbits) < nb) ++nbits;
  for (int64_t base = a; base < b; base += 64) {
    const int64_t h = base + lane;
    const bool valid = h < b;
    const int bin = valid ? bins[h] : 0;
    uint64_t m = __ballot(valid);
    for (int bit = 0; bit < nbits; ++bit) {
      const bool one = (bin >> bit) & 1;
      const uint64_t bb = __ballot(one);
      m &= one ? bb : ~bb;
    }
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int rank = __popcll(m & lt);
    int dest = 0;
    if (valid) dest = cnt(wave, bin) + rank;
    __builtin_amdgcn_wave_barrier();
    if (valid && rank == 0) cnt(wave, bin) += __popcll(m);
    __builtin_amdgcn_wave_barrier();
    if (valid) {
      const int64_t slot = lo + dest;
      perm[slot] = static_cast<int32_t>(h);
      float4* rec = reinterpret_cast<float4*>(binned + slot * KF_BINNED_FLOATS);
      rec[0] = make_float4(hit_pos[h], hit_pos[ldh + h], hit_pos[2 * ldh + h],
                           __int_as_float(static_cast<int32_t>(h - lo)));
      rec[1] = make_float4(hit_cov[h], hit_cov[ldh + h], hit_cov[2 * ldh + h], hit_cov[3 * ldh + h]);
      rec[2] = make_float4(hit_cov[4 * ldh + h], hit_cov[5 * ldh + h], 0.f, 0.f);
    }
  }
}

#undef cnt

// Binning for fine grids (more bins than the per-wave histograms hold): one
// LDS histogram per (event, layer) with atomics, a block scan, an unordered
// scatter of hit indices, then each bin's segment sorted by hit index (bins are
// small), so the result is the same stable order as bin_kernel's.  A block of
// 1024 threads owns one (event, layer) pair; the memory passes take several
// hits per thread with their loads issued together, since each is a chain of
// dependent accesses and one compute unit holds one block.
constexpr int kFineUnroll = 4;  // hits per thread and iteration of the memory passes
__global__ void __launch_bounds__(kBinThreads) bin_fine_kernel(int32_t L, const int64_t* __restrict__ layer_offsets,
                                                               const float* __restrict__ hit_pos,
                                                               const float* __restrict__ hit_cov, int64_t ldh,
                                                               int32_t n_phi, int32_t n_eta, Geom g,
                                                               int32_t* __restrict__ bins,
                                                               int32_t* __restrict__ bin_offsets,
                                                               int32_t* __restrict__ perm, float* __restrict__ binned,
                                                               float* __restrict__ layer_vmax,
                                                               const int32_t* __restrict__ el_order) {
  extern __shared__ int32_t cnt_fine[];  // [nb] counts, then scatter cursors, which end as the bins' ends
  __shared__ int32_t wsum[kBinWaves];
  __shared__ uint32_t vmax_bits[2];
  constexpr int U = kFineUnroll;
  constexpr int64_t kStep = static_cast<int64_t>(kBinThreads) * U;
  const int el = el_order ? el_order[blockIdx.x] : static_cast<int>(blockIdx.x);
  const int l = el % L;
  const int nb = n_phi * n_eta;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int64_t lo = layer_offsets[el], hi = layer_offsets[el + 1];
  for (int i = tid; i < nb; i += kBinThreads) cnt_fine[i] = 0;
  if (tid < 2) vmax_bits[tid] = 0u;
  __syncthreads();
  const double R = static_cast<double>(g.r[l]);
  const double zh = static_cast<double>(g.z_half[l]);
  const BinScale bs = bin_scale(R, zh, n_phi, n_eta);
  float my_vxy = 0.f, my_vz = 0.f;
  for (int64_t h = lo + tid; h < hi; h += kBinThreads) {
    const int bin = hit_bin_fast(hit_pos[h], hit_pos[ldh + h], hit_pos[2 * ldh + h], bs, R, zh, n_phi, n_eta);
    bins[h] = bin;
    atomicAdd(&cnt_fine[bin], 1);
    const float vxx = hit_cov[h], vyx = hit_cov[ldh + h], vyy = hit_cov[2 * ldh + h], vzz = hit_cov[5 * ldh + h];
    const float d = 0.5f * (vxx - vyy);
    my_vxy = fmaxf(my_vxy, 0.5f * (vxx + vyy) + sqrtf(d * d + vyx * vyx));
    my_vz = fmaxf(my_vz, vzz);
  }
  atomicMax(&vmax_bits[0], __float_as_uint(my_vxy));
  atomicMax(&vmax_bits[1], __float_as_uint(my_vz));
  __syncthreads();
  // exclusive scan of the counts: each wave a contiguous block of bins, then the waves' totals
  const int per_w = (nb + kBinWaves - 1) / kBinWaves;
  const int b0 = wave * per_w;
  const int b1 = (b0 + per_w < nb) ? b0 + per_w : nb;
  int wrun = 0;
  for (int base = b0; base < b1; base += 64) {
    const int bin = base + lane;
    const int v = (bin < b1) ? cnt_fine[bin] : 0;
    const int x = wave_incl_scan<false>(v);
    if (bin < b1) cnt_fine[bin] = wrun + x - v;
    wrun += __builtin_amdgcn_readlane(x, 63);
  }
  if (lane == 0) wsum[wave] = wrun;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int w = 0; w < kBinWaves; ++w) {
      const int c = wsum[w];
      wsum[w] = run;
      run += c;
    }
  }
  __syncthreads();
  int32_t* bo = bin_offsets + static_cast<int64_t>(el) * (nb + 1);
  for (int bin = tid; bin < nb; bin += kBinThreads) {
    const int off = cnt_fine[bin] + wsum[bin / per_w];
    cnt_fine[bin] = off;
    bo[bin] = static_cast<int32_t>(lo + off);
  }
  if (tid == 0) {
    bo[nb] = static_cast<int32_t>(hi);
    layer_vmax[2 * el] = __uint_as_float(vmax_bits[0]);
    layer_vmax[2 * el + 1] = __uint_as_float(vmax_bits[1]);
  }
  __syncthreads();
  // unordered scatter of hit indices; afterwards cnt_fine[b] is the end of bin b (the start of bin b + 1)
  for (int64_t h0 = lo + tid; h0 < hi; h0 += kStep) {
    int32_t b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t h = h0 + u * kBinThreads;
      b[u] = h < hi ? bins[h] : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t h = h0 + u * kBinThreads;
      if (h < hi) perm[lo + atomicAdd(&cnt_fine[b[u]], 1)] = static_cast<int32_t>(h);
    }
  }
  __syncthreads();
  // each bin's segment in hit-index order, its bounds from LDS: up to eight hits are loaded at once and sorted
  // in registers by a sorting network (Batcher's odd-even merge sort of eight), longer segments by insertion
  for (int bin = tid; bin < nb; bin += kBinThreads) {
    const int64_t s0 = lo + (bin > 0 ? cnt_fine[bin - 1] : 0), s1 = lo + cnt_fine[bin];
    const int64_t len = s1 - s0;
    if (len < 2) continue;
    if (len <= 8) {
      int32_t v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = k < len ? perm[s0 + k] : INT32_MAX;
      constexpr int kNet[19][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3}, {4, 6}, {5, 7}, {1, 2}, {5, 6},
                                   {0, 4}, {1, 5}, {2, 6}, {3, 7}, {2, 4}, {3, 5}, {1, 2}, {3, 4}, {5, 6}};
#pragma unroll
      for (int c = 0; c < 19; ++c) {
        const int32_t x = v[kNet[c][0]], y = v[kNet[c][1]];
        v[kNet[c][0]] = min(x, y);
        v[kNet[c][1]] = max(x, y);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (k < len) perm[s0 + k] = v[k];
    } else {
      for (int64_t i = s0 + 1; i < s1; ++i) {
        const int32_t v = perm[i];
        int64_t j = i - 1;
        while (j >= s0 && perm[j] > v) {
          perm[j + 1] = perm[j];
          --j;
        }
        perm[j + 1] = v;
      }
    }
  }
  __syncthreads();
  // Records: the inverse permutation (into the bin-number array, no longer needed) lets the hits be read in index
  // order, coalesced, and each record be written to its slot.  Gathering the hits in slot order instead reads
  // scattered words from hit arrays that, over all blocks of a die, do not fit in its L2 (measured three times
  // slower).
  for (int64_t s0 = lo + tid; s0 < hi; s0 += kStep) {
    int32_t hh[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t slot = s0 + u * kBinThreads;
      hh[u] = slot < hi ? perm[slot] : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t slot = s0 + u * kBinThreads;
      if (slot < hi) bins[hh[u]] = static_cast<int32_t>(slot - lo);
    }
  }
  __syncthreads();
  for (int64_t h0 = lo + tid; h0 < hi; h0 += kStep) {
    int32_t sl[U];
    float4 r0[U], r1[U], r2[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t h = h0 + u * kBinThreads;
      const int64_t hc = h < hi ? h : h0;
      sl[u] = bins[hc];
      r0[u] = make_float4(hit_pos[hc], hit_pos[ldh + hc], hit_pos[2 * ldh + hc],
                          __int_as_float(static_cast<int32_t>(hc - lo)));
      r1[u] = make_float4(hit_cov[hc], hit_cov[ldh + hc], hit_cov[2 * ldh + hc], hit_cov[3 * ldh + hc]);
      r2[u] = make_float4(hit_cov[4 * ldh + hc], hit_cov[5 * ldh + hc], 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t h = h0 + u * kBinThreads;
      if (h < hi) {
        float4* rec = reinterpret_cast<float4*>(binned + (lo + sl[u]) * KF_BINNED_FLOATS);
        rec[0] = r0[u];
        rec[1] = r1[u];
        rec[2] = r2[u];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// building
// ---------------------------------------------------------------------------

struct BuildP {
  int64_t n_seeds, ld_seed;
  int32_t n_events, first_layer, max_cands, n_phi, n_eta;
  float chi2_cut, margin;
  const int64_t* seed_offsets;
  const float* seed_state;
  const float* seed_cov;
  const int8_t* seed_charge;
  const int32_t* seed_hits;
  const int64_t* layer_offsets;
  const int32_t* bin_offsets;
  const float* binned;
  const float* layer_vmax;
  int32_t* n_cands;
  int32_t* cand_hits;
  float* cand_chi2;
  int32_t* cand_nhits;
  int32_t* cand_status;
  float* best_state;
  float* best_cov;
  unsigned long long* counters;
  int32_t* queue;
  const int32_t* order;      // tile position -> seed index (seeds grouped by direction), or null
  const unsigned char* mlp;  // packed search-window network, or null for the plain window
  float nsigma;
  float* cand_buf;  // serial-candidate build: two candidate buffers [2][kSerialWords][max_cands][buf_ld]
  int64_t buf_ld;   // tile positions (tiles x 64)
  Geom g;
};

__device__ __forceinline__ uint64_t make_key(int nhits, float chi2, int parent, uint32_t hit) {
  const uint64_t nh = static_cast<uint64_t>(63 - nhits) & 63u;
  const uint64_t cb = static_cast<uint64_t>(__float_as_uint(chi2) & 0x7FFFFFFFu);
  return (nh << 58) | (cb << 27) | (static_cast<uint64_t>(parent & 7) << 24) | (hit & kHole);
}

__device__ __forceinline__ int key_nhits(uint64_t k) { return 63 - static_cast<int>(k >> 58); }
__device__ __forceinline__ float key_chi2(uint64_t k) {
  return __uint_as_float(static_cast<uint32_t>((k >> 27) & 0x7FFFFFFFu));
}
__device__ __forceinline__ int key_parent(uint64_t k) { return static_cast<int>((k >> 24) & 7u); }
__device__ __forceinline__ uint32_t key_hit(uint64_t k) { return static_cast<uint32_t>(k & kHole); }

// minimum of k over the G lanes of this lane's seed group (groups of G consecutive lanes)
template <int G>
__device__ __forceinline__ uint64_t group_min(uint64_t k) {
  if constexpr ((G & (G - 1)) == 0) {
#pragma unroll
    for (int off = 1; off < G; off <<= 1) {
      const uint64_t o = __shfl_xor(k, off);
      k = o < k ? o : k;
    }
    return k;
  } else {
    // rotations by 1, 2, 4 within the group cover it (G <= 8); lanes past the last whole group get no minimum
    const int lane = threadIdx.x & 63;
    const int slot = lane % G, base = lane - slot;
#pragma unroll
    for (int r = 1; r < G; r <<= 1) {
      const int from = base + (slot + r < G ? slot + r : slot + r - G);
      const uint64_t o = __shfl(k, from);
      k = o < k ? o : k;
    }
    return lane < (64 / G) * G ? k : ~0ull;
  }
}

// Minimum of (k, s) by k over a seed group of six lanes (groups start at even lanes), the slot s travelling with its
// key: the two lanes of a pair (lane, lane ^ 1) exchange by a DPP quad permutation, then every lane reads the pair
// minima of the group's other two pairs, whose lanes' byte addresses are a1 and a2, in one round of LDS permutes.
// Lanes past the last whole group (a1 = a2 = their own) get no minimum.
__device__ __forceinline__ void group6_min(uint64_t& k, int32_t& s, int a1, int a2, bool in_group) {
  constexpr int kSwapPairs = 0xB1;  // quad_perm [1, 0, 3, 2]
  const uint32_t plo = static_cast<uint32_t>(
      __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(k)), kSwapPairs, 0xF, 0xF, true));
  const uint32_t phi = static_cast<uint32_t>(
      __builtin_amdgcn_update_dpp(0, static_cast<int>(static_cast<uint32_t>(k >> 32)), kSwapPairs, 0xF, 0xF, true));
  const int32_t ps = __builtin_amdgcn_update_dpp(0, s, kSwapPairs, 0xF, 0xF, true);
  const uint64_t pk = (static_cast<uint64_t>(phi) << 32) | plo;
  const bool take = pk < k;
  k = take ? pk : k;
  s = take ? ps : s;
  const int lo = static_cast<int>(static_cast<uint32_t>(k)), hi = static_cast<int>(static_cast<uint32_t>(k >> 32));
  const uint64_t k1 = (static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(a1, hi))) << 32) |
                      static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(a1, lo));
  const uint64_t k2 = (static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(a2, hi))) << 32) |
                      static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(a2, lo));
  const int32_t s1 = __builtin_amdgcn_ds_bpermute(a1, s), s2 = __builtin_amdgcn_ds_bpermute(a2, s);
  if (k1 < k) {
    k = k1;
    s = s1;
  }
  if (k2 < k) {
    k = k2;
    s = s2;
  }
  if (!in_group) k = ~0ull;
}

__device__ __forceinline__ int phi_bin_f(float phi, int n_phi) {
  int b = static_cast<int>(floorf((phi + 3.14159265358979f) * (static_cast<float>(n_phi) * 0.159154943091895f)));
  return b < 0 ? 0 : (b > n_phi - 1 ? n_phi - 1 : b);
}

// Eta row of pseudorapidity eta on a layer whose rows span [-emax, emax] in n_eta rows (escale = n_eta / 2 emax),
// after moving eta by dir * (2e-5 + 2e-5 |eta|): the low end of a window moves down and the high end up, by more
// than the error of asinh_hw and of the single-precision arithmetic, so that the rows cover the bins the binning
// kernel assigns (in double precision) to every hit of the window's z interval.  Clamped in floating point, so
// that an infinite or NaN end maps to a row.
__device__ __forceinline__ int eta_row(float eta, float dir, float emax, float escale, int n_eta) {
  const float e = eta + dir * (2e-5f + 2e-5f * fabsf(eta));
  const float t = floorf((e + emax) * escale);
  return static_cast<int>(fminf(fmaxf(t, 0.f), static_cast<float>(n_eta - 1)));
}

// atan2(y, x) of a point off the origin: an odd polynomial for atan on [0, 1] (its coefficients fitted to atan(a)/a
// in a^2 by weighted least squares; absolute error below 4e-7 when evaluated in single precision, 5e-7 with the
// hardware reciprocal) and the symmetries of the octants.
__device__ __forceinline__ float atan2_poly(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float a = fminf(ax, ay) * __builtin_amdgcn_rcpf(fmaxf(ax, ay));
  const float q = a * a;
  float r = 0.006811752f;
  r = fmaf(r, q, -0.033604082f);
  r = fmaf(r, q, 0.07962349f);
  r = fmaf(r, q, -0.13233331f);
  r = fmaf(r, q, 0.19807811f);
  r = fmaf(r, q, -0.33317366f);
  r = fmaf(r, q, 0.9999961f);
  r *= a;
  if (ay > ax) r = 1.57079633f - r;
  if (x < 0.f) r = 3.14159265f - r;
  return copysignf(r, y);
}

__device__ __forceinline__ float wrap_pi(float a) {
  if (a >= 3.14159265358979f) a -= 6.28318530717959f;
  if (a < -3.14159265358979f) a += 6.28318530717959f;
  return a;
}

// Wave-cooperative window scan.  All 64 lanes share the box tests of the wave's
// candidates: the candidates' slot ranges (one range index r at a time: row
// ie0 + r/2, segment r%2) are laid end to end and lane i takes items
// base + 64u + i, so a wide window no longer holds the whole wave to one lane.
// Box-passing (candidate, slot) pairs are queued in LDS in item order, which is
// candidate order within a range index; the queue is evaluated 64 pairs at a
// time (one chi2 per lane) and each candidate then inserts its own compatible
// hits, which are contiguous in the result list, into its register top-N.
template <typename T, bool LW>
struct ScanLds {
  // per candidate lane: x, y, z, nx, ny, att, atz, azz (what the box test and a chi2 need of the candidate), and
  // the plain window's half widths wt, wz; candidate-major, so that a reader takes them in two or three wide loads
  alignas(16) T pred[64][8];
  alignas(8) float box[64][2];
  int32_t rbias[kRangeChunk][64];  // per lane and range: slot of an item of the range minus its flat item index
  int32_t q_slot[kQueueCap];
  int32_t r_idx[64], r_slot[64];  // during the scan: the 256 16-bit owner codes of a block of items
  T r_c2[64];
  int32_t cnt[64], rstart[64];  // compatible results per candidate in a batch, and where they start
  int32_t live_lane[64];        // compacted live candidates -> lane (window network)
  uint8_t q_own[kQueueCap];     // owner lane of a queued pair; bit 6: outside the learned box
  // learned window only (one element otherwise)
  float lbox[2][LW ? 64 : 1];            // learned box half widths wt, wz
  int32_t qb_slot[LW ? kQueueDefer : 1];  // pairs waiting for a fallback
  int32_t need[LW ? 64 : 1];             // candidate (still) marked for the fallback
  uint8_t qb_own[LW ? kQueueDefer : 1];
};

// The per-layer back-pointers of the candidates (parent slot, hit) stay in LDS for the plain window,
// [layers from first_layer][64] per wave after the scan tables, so that the backtrack at the end of a tile reads
// LDS and cand_hits is written once; with the learned window (whose staged network weights already take the
// block's LDS) they go to the cand_hits output array and are rewritten there in place.
template <bool LW>
constexpr bool kBackLds = !LW;

// orders this lane's LDS accesses of the wave before and after (the wave executes in lockstep; this keeps the
// compiler from moving LDS accesses across the point)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// the value of the lane below (0 in lane 0), by a DPP shift of the whole wave
__device__ __forceinline__ int wave_shift_up1(int x) { return __builtin_amdgcn_update_dpp(0, x, 0x138, 0xF, 0xF, true); }

// maximum of a non-negative value over the wave, uniform
__device__ __forceinline__ int wave_max_i(int v) { return __builtin_amdgcn_readlane(wave_incl_scan<true>(v), 63); }

// A candidate's best children, in rank order: accumulated chi2, hit index within the (event, layer) (bit 30 set:
// outside the learned box, ranked after every hit inside it) and slot.  insert() keeps them sorted by (flag,
// chi2, index); positions past the N a build keeps hold children that are never used.
template <typename T, int Q>
struct ChildList {
  T key[Q];
  int32_t idx[Q], slot[Q];
  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int t = 0; t < Q; ++t) {
      key[t] = T(INFINITY);
      idx[t] = 0x7FFFFFFF;
      slot[t] = 0;
    }
  }
  __device__ __forceinline__ void insert(T nk, int32_t ni, int32_t nj, bool flags) {
#pragma unroll
    for (int t = 0; t < Q; ++t) {
      bool sw;
      if (flags) {
        const int fn = ni >> 30, ft = idx[t] >> 30;
        sw = fn < ft || (fn == ft && (nk < key[t] || (nk == key[t] && ni < idx[t])));
      } else {
        sw = nk < key[t] || (nk == key[t] && ni < idx[t]);
      }
      const T tk = key[t];
      const int32_t ti = idx[t], tj = slot[t];
      key[t] = sw ? nk : tk;
      idx[t] = sw ? ni : ti;
      slot[t] = sw ? nj : tj;
      nk = sw ? tk : nk;
      ni = sw ? ti : ni;
      nj = sw ? tj : nj;
    }
  }
  __device__ __forceinline__ T chi2_at(int t) const { return key[t]; }
  __device__ __forceinline__ int32_t idx_at(int t) const { return idx[t]; }
  __device__ __forceinline__ int32_t slot_at(int t) const { return slot[t]; }
  __device__ __forceinline__ void pop() {
#pragma unroll
    for (int t = 0; t + 1 < Q; ++t) {
      key[t] = key[t + 1];
      idx[t] = idx[t + 1];
      slot[t] = slot[t + 1];
    }
    key[Q - 1] = T(INFINITY);
  }
  __device__ __forceinline__ void strip_flags() {
#pragma unroll
    for (int t = 0; t < Q; ++t) idx[t] &= 0x3FFFFFFF;
  }
};

// Single precision: the flag, the chi2's bits (non-negative floats order as their bits) and the index form one
// 64-bit key that orders as the comparison above, so an insertion compares once per position, and every
// position's new value depends only on its own comparison and its left neighbour's (no chain along the list).
template <int Q>
struct ChildList<float, Q> {
  uint64_t key[Q];  // flag << 63 | chi2 bits << 32 | index without its flag; empty: all ones
  int32_t slot[Q];
  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int t = 0; t < Q; ++t) {
      key[t] = ~0ull;
      slot[t] = 0;
    }
  }
  __device__ __forceinline__ void insert(float nk, int32_t ni, int32_t nj, bool) {
    const uint64_t nkey = (static_cast<uint64_t>((static_cast<uint32_t>(ni) >> 30) & 1u) << 63) |
                          (static_cast<uint64_t>(__float_as_uint(nk)) << 32) |
                          static_cast<uint32_t>(ni & 0x3FFFFFFF);
    bool lt[Q];
#pragma unroll
    for (int t = 0; t < Q; ++t) lt[t] = nkey < key[t];
#pragma unroll
    for (int t = Q - 1; t >= 0; --t) {
      const bool shift = t > 0 && lt[t - 1];
      key[t] = shift ? key[t - 1] : (lt[t] ? nkey : key[t]);
      slot[t] = shift ? slot[t - 1] : (lt[t] ? nj : slot[t]);
    }
  }
  __device__ __forceinline__ float chi2_at(int t) const {
    return __uint_as_float(static_cast<uint32_t>(key[t] >> 32) & 0x7FFFFFFFu);
  }
  __device__ __forceinline__ int32_t idx_at(int t) const {
    return static_cast<int32_t>(static_cast<uint32_t>(key[t]) | (static_cast<uint32_t>(key[t] >> 63) << 30));
  }
  __device__ __forceinline__ int32_t slot_at(int t) const { return slot[t]; }
  __device__ __forceinline__ void pop() {
#pragma unroll
    for (int t = 0; t + 1 < Q; ++t) {
      key[t] = key[t + 1];
      slot[t] = slot[t + 1];
    }
    key[Q - 1] = ~0ull;
  }
  __device__ __forceinline__ void strip_flags() {
#pragma unroll
    for (int t = 0; t < Q; ++t) key[t] &= ~(1ull << 63);
  }
};

// Plain window, single precision, grouped build: the list holds the children's rank keys of the merge itself
// (nhits + 1, chi2 bits, parent slot, hit index).  Within one candidate nhits + 1 and the parent slot are fixed,
// so the keys order as (chi2, index) do, and the merge takes the head key as it is.
template <int Q>
struct ChildListMerge {
  uint64_t key[Q];  // empty: all ones
  int32_t slot[Q];
  uint64_t prefix;  // (63 - (nhits + 1)) << 58 | parent slot << 24
  __device__ __forceinline__ void clear(int nhits_child, int parent) {
    prefix = (static_cast<uint64_t>(63 - nhits_child) << 58) | (static_cast<uint64_t>(parent & 7) << 24);
#pragma unroll
    for (int t = 0; t < Q; ++t) {
      key[t] = ~0ull;
      slot[t] = 0;
    }
  }
  __device__ __forceinline__ void insert(float nk, int32_t ni, int32_t nj, bool) {
    const uint64_t nkey = prefix | (static_cast<uint64_t>(__float_as_uint(nk) & 0x7FFFFFFFu) << 27) |
                          static_cast<uint32_t>(ni & 0xFFFFFF);
    bool lt[Q];
#pragma unroll
    for (int t = 0; t < Q; ++t) lt[t] = nkey < key[t];
#pragma unroll
    for (int t = Q - 1; t >= 0; --t) {
      const bool shift = t > 0 && lt[t - 1];
      key[t] = shift ? key[t - 1] : (lt[t] ? nkey : key[t]);
      slot[t] = shift ? slot[t - 1] : (lt[t] ? nj : slot[t]);
    }
  }
  __device__ __forceinline__ float chi2_at(int t) const {
    return __uint_as_float(static_cast<uint32_t>((key[t] >> 27) & 0x7FFFFFFFu));
  }
  __device__ __forceinline__ int32_t idx_at(int t) const { return static_cast<int32_t>(key[t] & 0xFFFFFFu); }
  __device__ __forceinline__ int32_t slot_at(int t) const { return slot[t]; }
  __device__ __forceinline__ void pop() {
#pragma unroll
    for (int t = 0; t + 1 < Q; ++t) {
      key[t] = key[t + 1];
      slot[t] = slot[t + 1];
    }
    key[Q - 1] = ~0ull;
  }
  __device__ __forceinline__ void strip_flags() {}
};

// Scans the plain window of this lane's candidate (the wave's 64 candidates together) and leaves in
// kids the candidate's best children by (chi2, hit index): their accumulated chi2, hit index
// within the (event, layer) and slot, cnt of them (at most N); with the learned window, the definition of the
// learned search window with its fallback (see below).  Wave-uniform work counters are accumulated.
template <int Q, typename T, bool LW, typename List>
__device__ __forceinline__ void scan_window(const BuildP& p, ScanLds<T, LW>& C, const unsigned char* mlp_lds, int l,
                                            int64_t el, bool live, const T (&ps)[6], const T (&pc)[21], float qf,
                                            T chi2, int N, int lane, uint64_t lanes_below, const float4* recs,
                                            List& kids, int& cnt,
                                            int& cnt_in, uint32_t& n_box, uint32_t& n_chi2, uint32_t& n_comp,
                                            uint32_t& n_fb) {
  // Window geometry of this lane's candidate (dead lanes only work for others).
    const float R = p.g.r[l];
  const LocalPred<T> lp = local_pred(ps, pc);
  const float px0 = float(ps[0]), py0 = float(ps[1]), pz0 = float(ps[2]);
  const float rtt = live ? float(lp.att) + p.layer_vmax[2 * el] : 0.f;
  const float rzz = live ? float(pc[5]) + p.layer_vmax[2 * el + 1] : 0.f;
  const float fac = 1.f + p.margin;
  // plain half widths bound the chi2 < cut region (Cauchy-Schwarz on R^-1)
  // (hardware square roots, within about an ulp: the margin covers far more)
  const float wt_plain = __builtin_amdgcn_sqrtf(p.chi2_cut * rtt) * fac;
  const float wz_plain = __builtin_amdgcn_sqrtf(p.chi2_cut * rzz) * fac;
  // Learned window: one network evaluation per live candidate, all lanes of the wave together.  Its box
  // (never wider than the plain one) decides which compatible hits count; when none is inside it, the
  // compatible hits of the plain window count instead (fallback).  One scan of the plain window's bins
  // serves both: pairs inside the learned box are evaluated at once, the other pairs inside the plain box
  // wait in a second queue.  A candidate with no pair inside its learned box falls back for certain: its
  // waiting pairs join the last batches of the scan.  One whose inside pairs all fail the cut (rare) takes
  // them after it.
  float wt_in = wt_plain, wz_in = wz_plain;
  bool tighter = false;
  if (LW) {
    float f[8];
    if (live) {
      window_features(ps, pc, qf, p.g.r[l - 1], R, p.g.z_half[l], f);
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) f[k] = 0.f;
    }
    float o0, o1;
    const uint64_t um = __ballot(live);
    const int lpos = live ? __popcll(um & lanes_below) : -1;
    wave_lds_sync();
    if (live) C.live_lane[lpos] = lane;
    wave_lds_sync();
    kfm::eval_compact_lds(mlp_lds, f, lane, C.live_lane, __popcll(um), lpos, o0, o1);
    if (live) {
      const float lwt = p.nsigma * __expf(o0);
      const float lwz = p.nsigma * __expf(o1);
      tighter = lwt < wt_plain || lwz < wz_plain;
      wt_in = fminf(lwt, wt_plain);
      wz_in = fminf(lwz, wz_plain);
    }
    C.lbox[0][lane] = wt_in;
    C.lbox[1][lane] = wz_in;
    C.need[lane] = tighter ? 1 : 0;  // cleared by the first pair inside the learned box
  }
  const float php = atan2_poly(py0, px0);
  const float iR = __builtin_amdgcn_rcpf(R);  // hardware reciprocals (about an ulp), inside the rows' widening
  const float emax = asinh_hw(p.g.z_half[l] * iR);
  const float escale = static_cast<float>(p.n_eta) * __builtin_amdgcn_rcpf(2.f * emax);
  const int32_t* bo = p.bin_offsets + el * (p.n_phi * p.n_eta + 1);
  C.pred[lane][0] = ps[0];
  C.pred[lane][1] = ps[1];
  C.pred[lane][2] = ps[2];
  C.pred[lane][3] = lp.nx;
  C.pred[lane][4] = lp.ny;
  C.pred[lane][5] = lp.att;
  C.pred[lane][6] = lp.atz;
  C.pred[lane][7] = lp.azz;
  C.box[lane][0] = wt_plain;
  C.box[lane][1] = wz_plain;
  // bins the plain window overlaps: the cyclic phi interval [ip0, ip0 + nspan) and the eta rows ie0..ie1
  int ip0 = 0, nspan = p.n_phi, ie0 = 0, ie1 = -1;
  if (live) {
    // the window spans asin(sphi) either side of the prediction's azimuth; tan(asin(sphi)) = sphi / sqrt(1 - sphi^2)
    // bounds it from above, and the interval is widened by more than the errors of atan2_poly, of the hardware
    // reciprocal square root and of the single-precision bin arithmetic, so that its bins cover those the binning
    // kernel assigns (in double precision) to every hit of the box.  Wide windows (sphi >= 0.9) take the whole ring.
    const float sphi = wt_plain * iR;
    if (sphi < 0.9f) {
      const float dphi = fmaf(sphi * __builtin_amdgcn_rsqf(fmaf(-sphi, sphi, 1.f)), 1.000002f, 4e-6f);
      ip0 = phi_bin_f(wrap_pi(php - dphi), p.n_phi);
      const int ip1 = phi_bin_f(wrap_pi(php + dphi), p.n_phi);
      const int d = ip1 - ip0;  // both in [0, n_phi): the cyclic distance without an integer division
      nspan = (d < 0 ? d + p.n_phi : d) + 1;
    }
    ie0 = eta_row(asinh_hw((pz0 - wz_plain) * iR), -1.f, emax, escale, p.n_eta);
    ie1 = eta_row(asinh_hw((pz0 + wz_plain) * iR), 1.f, emax, escale, p.n_eta);
  }
  const int first_end = (ip0 + nspan <= p.n_phi) ? ip0 + nspan : p.n_phi;
  const int wrap_end = ip0 + nspan - p.n_phi;  // > 0 if the span wraps
  const int nr = live ? 2 * (ie1 - ie0 + 1) : 0;
  const int max_nr = wave_max_i(nr);
  // bounds of this lane's r-th slot range (row ie0 + r/2, segment r%2)
  auto range_of = [&](int r, int& ra, int& rn) {
    ra = 0;
    rn = 0;
    if (r < nr) {
      const int row = (ie0 + (r >> 1)) * p.n_phi;
      if ((r & 1) == 0) {
        ra = bo[row + ip0];
        rn = bo[row + first_end] - ra;
      } else if (wrap_end > 0) {
        ra = bo[row];
        rn = bo[row + wrap_end] - ra;
      }
    }
  };
  int qn = 0;  // pairs awaiting their chi2, carried across the ranges
  int qh = 0;  // ring position of the oldest of them: the queue is a ring of kQueueCap entries (never more queued)
  // ring position of the pair k places after the oldest (k < kQueueCap)
  auto qpos = [&](int k) {
    const int r = qh + k;
    return r >= kQueueCap ? r - kQueueCap : r;
  };
  int qb = 0;  // learned window: pairs inside the plain box but outside the learned one, waiting
  // Evaluates the queue 64 pairs at a time (all of it when final) and inserts the compatible hits into the
  // owners' lists.  A queued owner with bit 6 set marks a pair outside the learned box: its hit is flagged
  // (bit 30 of the index) and ranks after every unflagged hit of the list.
  auto flush = [&](bool final_batch) {
    while (qn >= 64 || (final_batch && qn > 0)) {
      wave_lds_sync();
      const int nb = qn < 64 ? qn : 64;
      bool comp = false;
      T c2 = T(0);
      int32_t hidx = 0, jq = 0, oq = 0;
      if (lane < nb) {
        const int qi = qpos(lane);
        jq = C.q_slot[qi];
        const int qo = C.q_own[qi];
        oq = qo & 63;
        const float4 h = recs[static_cast<int64_t>(jq) * 3];
        const float4 c0 = recs[static_cast<int64_t>(jq) * 3 + 1];
        const float4 c1 = recs[static_cast<int64_t>(jq) * 3 + 2];
        const float mm[3] = {h.x, h.y, h.z};
        const float vv[6] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y};
        T pos3[6];
        T pq[8];
        if constexpr (std::is_same<T, float>::value) {  // two 16-byte LDS loads
          const float4 q0 = *reinterpret_cast<const float4*>(&C.pred[oq][0]);
          const float4 q1 = *reinterpret_cast<const float4*>(&C.pred[oq][4]);
          pq[0] = q0.x; pq[1] = q0.y; pq[2] = q0.z; pq[3] = q0.w;
          pq[4] = q1.x; pq[5] = q1.y; pq[6] = q1.z; pq[7] = q1.w;
        } else {
#pragma unroll
          for (int k = 0; k < 8; ++k) pq[k] = C.pred[oq][k];
        }
        pos3[0] = pq[0];
        pos3[1] = pq[1];
        pos3[2] = pq[2];
        LocalPred<T> L;
        L.nx = pq[3];
        L.ny = pq[4];
        L.tx = -L.ny;
        L.ty = L.nx;
        L.att = pq[5];
        L.atz = pq[6];
        L.azz = pq[7];
        if (!chi2_on_layer(pos3, L, mm, vv, c2) && c2 < T(p.chi2_cut)) {
          comp = true;
          hidx = __float_as_int(h.w) | (LW ? ((qo >> 6) << 30) : 0);
        }
      }
      n_chi2 += nb;
      n_comp += __popcll(__ballot(comp));
      // group the compatible results by candidate: per-candidate counts, their prefix, then each
      // result at its candidate's start plus its rank (the insertion order does not matter: the
      // top-N list orders by its key)
      wave_lds_sync();  // queue entries read
      C.cnt[lane] = 0;
      wave_lds_sync();
      const int rank = comp ? atomicAdd(&C.cnt[oq], 1) : 0;
      wave_lds_sync();
      const int count = C.cnt[lane];
      const int cinc = wave_incl_scan<false>(count);
      const int first = cinc - count;
      C.rstart[lane] = first;
      wave_lds_sync();
      if (comp) {
        const int rp = C.rstart[oq] + rank;
        C.r_idx[rp] = hidx;
        C.r_slot[rp] = jq;
        C.r_c2[rp] = c2;
      }
      // the batch leaves the ring
      qh = qpos(nb);
      qn -= nb;
      wave_lds_sync();
      const int rounds = wave_max_i(count);
      for (int k = 0; k < rounds; ++k) {
        if (k < count) {
          const int e = first + k;
          const T cc = C.r_c2[e];
          const T nk = chi2 + (cc > T(0) ? cc : T(0));
          const int32_t ni = C.r_idx[e];
          if (LW && (ni >> 30) == 0) cnt_in = cnt_in + 1 < N ? cnt_in + 1 : N;
          kids.insert(nk, ni, C.r_slot[e], LW);
          cnt = cnt + 1 < N ? cnt + 1 : N;
        }
      }
    }
  };
  // Appends the waiting pairs whose owner is marked in C.need to the queue, flagged as outside the learned
  // box (the queue holds them: at most 63 + kQueueDefer pairs).
  auto take_waiting = [&]() {
    wave_lds_sync();
    for (int b0 = 0; b0 < qb; b0 += 64) {
      const int i = b0 + lane;
      int jb = 0, ob = 0;
      bool take = false;
      if (i < qb) {
        jb = C.qb_slot[i];
        ob = C.qb_own[i];
        take = C.need[ob] != 0;
      }
      const uint64_t mt = __ballot(take);
      if (take) {
        const int pos = qpos(qn + __popcll(mt & lanes_below));
        C.q_slot[pos] = jb;
        C.q_own[pos] = static_cast<uint8_t>(ob | 64);
      }
      qn += __popcll(mt);
    }
  };
  // Ranges are taken kRangeChunk per lane at a time: their bounds load together, each lane's ranges are
  // laid end to end and the lanes' totals end to end, so one flat item space covers them all; the slot of an
  // item is its flat index plus its range's bias (in LDS).
  for (int r0 = 0; r0 < max_nr; r0 += kRangeChunk) {
    int ra[kRangeChunk], rn[kRangeChunk];
#pragma unroll
    for (int j = 0; j < kRangeChunk; ++j) range_of(r0 + j, ra[j], rn[j]);
    int mine = 0;
    int cum[kRangeChunk];  // items of this lane before each of its ranges
#pragma unroll
    for (int j = 0; j < kRangeChunk; ++j) {
      cum[j] = mine;
      mine += rn[j];
    }
    const int incl = wave_incl_scan<false>(mine);
    const int total = __builtin_amdgcn_readlane(incl, 63);
    const int my_off = incl - mine;  // flat index of this lane's first item
    int first[kRangeChunk];          // flat index of the first item of each non-empty range (-1: empty)
    wave_lds_sync();                 // the previous chunk's readers are done with the table
#pragma unroll
    for (int j = 0; j < kRangeChunk; ++j) {
      C.rbias[j][lane] = ra[j] - (my_off + cum[j]);
      first[j] = rn[j] > 0 ? my_off + cum[j] : -1;
    }
    wave_lds_sync();
    int carry = 0;  // owner code of the item before the current block of items (0: none)
    for (int base = 0; base < total; base += 64 * kScanUnroll) {
      n_box += min(total - base, 64 * kScanUnroll);
      // Owners of the block's 64 kScanUnroll items: the first item of each non-empty range (lane, j) is marked
      // with the code lane * kRangeChunk + j + 1, and an item's owner code is the largest mark at or before it, or
      // the carry (the ranges are laid out in code order).  The 16-bit codes sit in the batch result tables,
      // which are idle until the flush.
      static_assert(64 * kScanUnroll == 256, "one 16-bit owner code per item of a block");
      static_assert(kRangeChunk == 4, "the owner code holds the range in its low two bits");
      using Lds = ScanLds<T, LW>;
      static_assert(offsetof(Lds, r_slot) == offsetof(Lds, r_idx) + 256, "the owner codes take r_idx and r_slot");
      uint2* const own8 = reinterpret_cast<uint2*>(C.r_idx);
      uint16_t* const own2 = reinterpret_cast<uint16_t*>(C.r_idx);
      wave_lds_sync();
      own8[lane] = make_uint2(0u, 0u);
      wave_lds_sync();
#pragma unroll
      for (int j = 0; j < kRangeChunk; ++j)
        if (first[j] >= base && first[j] < base + 256)
          own2[first[j] - base] = static_cast<uint16_t>(lane * kRangeChunk + j + 1);
      wave_lds_sync();
      const uint2 h = own8[lane];  // items base + 4 lane .. base + 4 lane + 3
      const int m0 = static_cast<int>(h.x & 0xFFFFu), m1 = max(m0, static_cast<int>(h.x >> 16));
      const int m2 = max(m1, static_cast<int>(h.y & 0xFFFFu)), m3 = max(m2, static_cast<int>(h.y >> 16));
      const int sc = wave_incl_scan<true>(m3);  // inclusive maximum over the lanes
      const int before = max(wave_shift_up1(sc), carry);
      const uint2 ow = make_uint2(static_cast<uint32_t>(max(before, m0)) | (static_cast<uint32_t>(max(before, m1)) << 16),
                                  static_cast<uint32_t>(max(before, m2)) | (static_cast<uint32_t>(max(before, m3)) << 16));
      carry = max(carry, __builtin_amdgcn_readlane(sc, 63));
      wave_lds_sync();
      own8[lane] = ow;  // the owner codes in item order
      wave_lds_sync();
      int own[kScanUnroll], js[kScanUnroll];
      float4 hv[kScanUnroll];
#pragma unroll
      for (int u = 0; u < kScanUnroll; ++u) {
        const int w = base + 64 * u + lane;
        const int wc = w < total ? w : total - 1;
        const int code = own2[wc - base];
        const int c = code > 0 ? code - 1 : 0;
        const int lo = c >> 2;  // the candidate lane whose range holds item wc
        own[u] = lo;
        js[u] = wc + C.rbias[c & 3][lo];
        hv[u] = recs[static_cast<int64_t>(js[u]) * 3];
      }
#pragma unroll
      for (int u = 0; u < kScanUnroll; ++u) {
        const int w = base + 64 * u + lane;
        bool in_box = false, out_box = false;
        if (w < total) {
          const int o = own[u];
          // tangent (-ny, nx) at the prediction
          float px, py, pz, pnx, pny;
          if constexpr (std::is_same<T, float>::value) {  // one 16-byte and one 4-byte LDS load
            const float4 q = *reinterpret_cast<const float4*>(&C.pred[o][0]);
            px = q.x;
            py = q.y;
            pz = q.z;
            pnx = q.w;
            pny = C.pred[o][4];
          } else {
            px = float(C.pred[o][0]);
            py = float(C.pred[o][1]);
            pz = float(C.pred[o][2]);
            pnx = float(C.pred[o][3]);
            pny = float(C.pred[o][4]);
          }
          const float2 bx = *reinterpret_cast<const float2*>(&C.box[o][0]);
          const float dx = hv[u].x - px, dy = hv[u].y - py;
          const float az = fabsf(hv[u].z - pz);
          const float at = fabsf(-pny * dx + pnx * dy);
          const bool plain_box = at <= bx.x && az <= bx.y;
          if (LW) {
            in_box = at <= C.lbox[0][o] && az <= C.lbox[1][o];
            out_box = !in_box && plain_box;
            if (in_box) C.need[o] = 0;
          } else {
            in_box = plain_box;
          }
        }
        bool to_q = in_box;
        int flag = 0;
        if (LW) {
          const uint64_t mo = __ballot(out_box);
          const int no = __popcll(mo);
          if (qb + no <= kQueueDefer) {
            if (out_box) {
              const int pos = qb + __popcll(mo & lanes_below);
              C.qb_slot[pos] = js[u];
              C.qb_own[pos] = static_cast<uint8_t>(own[u]);
            }
            qb += no;
          } else {
            // waiting queue full: evaluate these pairs now, flagged as outside the learned box
            to_q = in_box || out_box;
            flag = out_box ? 64 : 0;
          }
        }
        const uint64_t m = __ballot(to_q);
        if (to_q) {
          const int pos = qpos(qn + __popcll(m & lanes_below));
          C.q_slot[pos] = js[u];
          C.q_own[pos] = static_cast<uint8_t>(own[u] | flag);
        }
        qn += __popcll(m);
      }
      flush(false);  // full batches of 64
    }
  }
  // candidates without any pair inside their learned box fall back for certain: their waiting pairs join the
  // last batches
  if (LW && qb > 0) take_waiting();
  flush(true);
  if (LW) {
    const bool need = tighter && cnt_in == 0;
    n_fb += __popcll(__ballot(need));
    if (qb > 0) {
      // the rest of the fallbacks: candidates whose pairs inside the learned box all failed the cut
      wave_lds_sync();
      const bool late = need && C.need[lane] == 0;
      if (__ballot(late) != 0) {
        wave_lds_sync();
        C.need[lane] = late ? 1 : 0;
        take_waiting();
        flush(true);
      }
    }
    // a candidate with a compatible hit inside its learned box keeps only those (they rank first)
    if (cnt_in > 0) cnt = cnt_in;
    kids.strip_flags();
  }
}

template <int G, typename T, bool LW>
__device__ void build_tile(const BuildP& p, int64_t tile, const unsigned char* mlp_lds) {
  constexpr int SPW = 64 / G;  // seeds per wave (G = 6: ten seeds, lanes 60..63 hold none)
  const int lane = threadIdx.x & 63;
  const int slot = lane % G;
  const int gbase = lane - slot;
  const int64_t pos = tile * SPW + lane / G;
  const bool seed_ok = lane < SPW * G && pos < p.n_seeds;
  const int64_t s = (seed_ok && p.order) ? static_cast<int64_t>(p.order[pos]) : pos;
  const int L = p.g.n_layers;
  const int N = p.max_cands;
  // event of this seed
  int ev = 0;
  if (seed_ok) {
    int lo = 0, hi = p.n_events;  // seed_offsets[lo] <= s < seed_offsets[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (p.seed_offsets[mid] <= s) lo = mid; else hi = mid;
    }
    ev = lo;
  }
  const T a = T(-static_cast<double>(seed_ok ? p.seed_charge[s] : 1) * kCLight * p.g.bz);
  T st[6], cv[21];
  int32_t status = 0;
  if (seed_ok && slot == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) st[k] = T(p.seed_state[k * p.ld_seed + s]);
#pragma unroll
    for (int k = 0; k < 21; ++k) cv[k] = T(p.seed_cov[k * p.ld_seed + s]);
    status = finite6_21(st, cv) ? 0 : ST_NONFINITE;
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) st[k] = T(0);
#pragma unroll
    for (int k = 0; k < 21; ++k) cv[k] = T(0);
  }
  T chi2 = T(0);
  int nhits = 3;
  int nc = seed_ok ? 1 : 0;  // candidates of this seed (same in all its lanes)
  // work counters of the wave and tile: kept wave-uniform (counted with ballots at converged points) so that they
  // occupy scalar registers rather than six vector registers for the whole tile
  uint32_t n_box = 0, n_chi2 = 0, n_comp = 0, n_steps = 0, n_upd = 0, n_fb = 0;
  const float qf = seed_ok ? static_cast<float>(p.seed_charge[s]) : 1.f;
  // one ScanLds per wave of the block, in dynamic LDS sized by the launch (blockDim / 64 of them)
  extern __shared__ __align__(16) unsigned char build_lds[];
  ScanLds<T, LW>& C = reinterpret_cast<ScanLds<T, LW>*>(build_lds)[threadIdx.x >> 6];
  const int n_back = L - p.first_layer;  // layers with a back-pointer
  int32_t* const back = reinterpret_cast<int32_t*>(build_lds + (blockDim.x >> 6) * sizeof(ScanLds<T, LW>)) +
                        (threadIdx.x >> 6) * n_back * 64;
  const uint64_t lanes_below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const float4* recs = reinterpret_cast<const float4*>(p.binned);

  for (int l = p.first_layer; l < L; ++l) {
    const bool active = slot < nc;
    const int64_t el = static_cast<int64_t>(ev) * L + l;
    // ---- propagate (material of the layer the candidate sits on, then the crossing)
    T ps[6], pc[21];
#pragma unroll
    for (int k = 0; k < 6; ++k) ps[k] = st[k];
#pragma unroll
    for (int k = 0; k < 21; ++k) pc[k] = cv[k];
    int32_t pstat = status;
    n_steps += __popcll(__ballot(active && status == 0));
    if (active && status == 0) {
      int32_t r = material(ps, pc, T(p.g.x_over_x0[l - 1]), T(p.g.eloss_per_x0), T(p.g.mass));
      if (!r) r = propagate(ps, pc, a, T(p.g.r[l]), T(p.g.z_half[l]));
      if (r) {
        pstat = r;
#pragma unroll
        for (int k = 0; k < 6; ++k) ps[k] = st[k];
#pragma unroll
        for (int k = 0; k < 21; ++k) pc[k] = cv[k];
      }
    }
    // ---- scan the window's bins, keep the best N children of this candidate
    // the merge's own rank keys for the plain single-precision build (the head key is then the merge key)
    constexpr bool kMergeKeys = std::is_same<T, float>::value && !LW;
    std::conditional_t<kMergeKeys, ChildListMerge<G>, ChildList<T, G>> kids;
    if constexpr (kMergeKeys)
      kids.clear(nhits + 1, slot);
    else
      kids.clear();
    int cnt = 0;     // children in the list (at most N)
    int cnt_in = 0;  // learned window: those inside the learned box (at most N)
    scan_window<G, T, LW>(p, C, mlp_lds, l, el, active && pstat == 0, ps, pc, qf, chi2, N, lane, lanes_below, recs,
                          kids, cnt, cnt_in, n_box, n_chi2, n_comp, n_fb);
    // ---- merge the seed's lists: N rounds of a G-lane minimum of the rank key
    bool hole_left = active;
    uint64_t mine = ~0ull;  // the child that becomes this slot's candidate
    int32_t mine_slot = -1;
    T mine_chi2 = T(0);
    int new_nc = 0;
    // six-lane groups: byte addresses of a lane in each of the other two pairs of the group
    const int pair = slot >> 1;
    const bool in_group = lane < SPW * G;
    const int a1 = 4 * (in_group ? gbase + 2 * (pair == 2 ? 0 : pair + 1) : lane);
    const int a2 = 4 * (in_group ? gbase + 2 * (pair == 0 ? 2 : pair - 1) : lane);
    for (int r = 0; r < N; ++r) {
      uint64_t k = ~0ull;
      const bool has_hit = active && pstat == 0 && cnt > 0;
      if (has_hit) {
        if constexpr (kMergeKeys)
          k = kids.key[0];
        else
          k = make_key(nhits + 1, float(kids.chi2_at(0)), slot, static_cast<uint32_t>(kids.idx_at(0)));
      }
      else if (hole_left)
        k = make_key(nhits, float(chi2), slot, kHole);
      uint64_t kmin;
      int32_t wslot;
      if constexpr (G == 6) {
        kmin = k;
        wslot = has_hit ? kids.slot_at(0) : -1;
        group6_min(kmin, wslot, a1, a2, in_group);
      } else {
        kmin = group_min<G>(k);
      }
      if (__ballot(kmin != ~0ull) == 0) break;  // no seed of the wave has a child left
      const int winner = gbase + key_parent(kmin);
      if constexpr (G != 6) wslot = __shfl(has_hit ? kids.slot_at(0) : -1, winner);
      // in single precision the key holds the child's chi2 exactly; in double precision it comes from the winner
      T wchi2;
      if constexpr (std::is_same<T, float>::value)
        wchi2 = key_chi2(kmin);
      else
        wchi2 = __shfl(has_hit ? kids.chi2_at(0) : chi2, winner);
      if (kmin != ~0ull) {
        new_nc = r + 1;
        if (slot == r) {
          mine = kmin;
          mine_slot = wslot;
          mine_chi2 = wchi2;
        }
        if (k == kmin) {
          if (has_hit) {
            kids.pop();
            cnt--;
          } else {
            hole_left = false;
          }
        }
      }
    }
    // ---- update the survivors from their parent's propagated state
    const int src = gbase + (mine != ~0ull ? key_parent(mine) : slot);
#pragma unroll
    for (int k = 0; k < 6; ++k) st[k] = __shfl(ps[k], src);
#pragma unroll
    for (int k = 0; k < 21; ++k) cv[k] = __shfl(pc[k], src);
    status = __shfl(pstat, src);
    n_upd += __popcll(__ballot(mine != ~0ull && key_hit(mine) != kHole && status == 0));
    if (mine != ~0ull) {
      nhits = key_nhits(mine);
      chi2 = mine_chi2;
      const uint32_t hid = key_hit(mine);
      if (hid != kHole && status == 0) {
        const float4 h = recs[static_cast<int64_t>(mine_slot) * 3];
        const float4 c0 = recs[static_cast<int64_t>(mine_slot) * 3 + 1];
        const float4 c1 = recs[static_cast<int64_t>(mine_slot) * 3 + 2];
        const float m[3] = {h.x, h.y, h.z};
        const float v[6] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y};
        T dc2;
        const int32_t r = update_on_layer<T, double>(st, cv, m, v, dc2);
        if (r) status = r;
      }
      const int32_t rec = static_cast<int32_t>((static_cast<uint32_t>(key_parent(mine)) << 24) | hid);
      if (kBackLds<LW>)
        back[(l - p.first_layer) * 64 + lane] = rec;
      else
        p.cand_hits[static_cast<int64_t>(l) * p.n_seeds * N + s * N + slot] = rec;
    }
    nc = new_nc;
  }
  // ---- outputs
  if (seed_ok) {
    if (slot == 0) p.n_cands[s] = nc;
    if (slot < N) {
      const bool live = slot < nc;
      p.cand_chi2[s * N + slot] = live ? static_cast<float>(chi2) : 0.f;
      p.cand_nhits[s * N + slot] = live ? nhits : 0;
      p.cand_status[s * N + slot] = live ? status : 0;
    }
    if (slot == 0 && p.best_state) {
#pragma unroll
      for (int k = 0; k < 6; ++k) p.best_state[k * p.ld_seed + s] = static_cast<float>(st[k]);
#pragma unroll
      for (int k = 0; k < 21; ++k) p.best_cov[k * p.ld_seed + s] = static_cast<float>(cv[k]);
    }
  }
  // backtrack the parent chain (from LDS, or in place in cand_hits: at each layer every lane reads its
  // record before any lane of the wave writes that layer, a data dependence)
  int kk = slot;
  const bool live = seed_ok && slot < nc;
  if (kBackLds<LW>) wave_lds_sync();
  for (int l = L - 1; l >= p.first_layer; --l) {
    int32_t out = -1;
    int64_t at = static_cast<int64_t>(l) * p.n_seeds * N + s * N + slot;
    if (live) {
      const uint32_t rec =
          kBackLds<LW> ? static_cast<uint32_t>(back[(l - p.first_layer) * 64 + gbase + kk])
                       : static_cast<uint32_t>(p.cand_hits[static_cast<int64_t>(l) * p.n_seeds * N + s * N + kk]);
      const uint32_t hid = rec & kHole;
      kk = static_cast<int>(rec >> 24);
      out = (hid == kHole) ? -1 : static_cast<int32_t>(p.layer_offsets[static_cast<int64_t>(ev) * L + l] + hid);
    }
    __builtin_amdgcn_wave_barrier();
    if (seed_ok && slot < N) p.cand_hits[at] = out;
  }
  if (seed_ok && slot < N) {
    for (int l = 0; l < p.first_layer; ++l) {
      int32_t out = -1;
      if (live && l < 3) out = p.seed_hits[l * p.ld_seed + s];
      p.cand_hits[static_cast<int64_t>(l) * p.n_seeds * N + s * N + slot] = out;
    }
  }
  if (p.counters && lane == 0) {
    const uint32_t v[KF_BUILD_COUNTERS] = {n_box, n_chi2, n_comp, n_steps, n_upd, n_fb};
#pragma unroll
    for (int i = 0; i < KF_BUILD_COUNTERS; ++i)
      if (v[i]) atomicAdd(&p.counters[i], static_cast<unsigned long long>(v[i]));
  }
}

// ---------------------------------------------------------------------------
// Serial-candidate building: one lane per seed (64 seeds a wave) holding all
// of its candidates, which it takes one after the other (the paper's proposed
// one thread per seed).  A candidate's state, covariance and (hits, chi2,
// status) live in a device buffer indexed by tile position, so that the loads
// of a wave are coalesced: buffer A holds the layer's candidates (overwritten
// by their propagated states), buffer B the survivors.  For every candidate
// index c the wave propagates and scans the c-th candidate of each of its
// seeds together (the same wave-cooperative scan as the grouped build), and
// each lane merges the children into its seed's top-N list in registers.
// Results are those of the grouped build: same rank key, same order of keys.
// ---------------------------------------------------------------------------
constexpr int kSerialWords = 30;  // 6 state + 21 covariance + nhits, chi2, status (as float bits)

__device__ __forceinline__ uint64_t sel_key(const uint64_t (&k)[kSerialMax], int r) {
  uint64_t v = k[0];
#pragma unroll
  for (int t = 1; t < kSerialMax; ++t) v = (r == t) ? k[t] : v;
  return v;
}
__device__ __forceinline__ int32_t sel_i32(const int32_t (&k)[kSerialMax], int r) {
  int32_t v = k[0];
#pragma unroll
  for (int t = 1; t < kSerialMax; ++t) v = (r == t) ? k[t] : v;
  return v;
}
__device__ __forceinline__ float sel_f(const float (&k)[kSerialMax], int r) {
  float v = k[0];
#pragma unroll
  for (int t = 1; t < kSerialMax; ++t) v = (r == t) ? k[t] : v;
  return v;
}

__device__ void build_serial_tile(const BuildP& p, int64_t tile) {
  using T = float;
  const int lane = threadIdx.x & 63;
  const int64_t pos = tile * 64 + lane;
  const bool seed_ok = pos < p.n_seeds;
  const int64_t s = (seed_ok && p.order) ? static_cast<int64_t>(p.order[pos]) : pos;
  const int L = p.g.n_layers;
  const int N = p.max_cands;
  int ev = 0;
  if (seed_ok) {
    int lo = 0, hi = p.n_events;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (p.seed_offsets[mid] <= s) lo = mid; else hi = mid;
    }
    ev = lo;
  }
  const T a = T(-static_cast<double>(seed_ok ? p.seed_charge[s] : 1) * kCLight * p.g.bz);
  const float qf = seed_ok ? static_cast<float>(p.seed_charge[s]) : 1.f;
  const int64_t ld = p.buf_ld;
  const int64_t bstride = static_cast<int64_t>(kSerialWords) * N * ld;  // one buffer
  // word k of candidate c in buffer b
  auto at = [&](int b, int c, int k) -> float& { return p.cand_buf[b * bstride + (static_cast<int64_t>(k) * N + c) * ld + pos]; };
  int cur = 0;
  int nc = seed_ok ? 1 : 0;
  if (seed_ok) {
    T st[6], cv[21];
#pragma unroll
    for (int k = 0; k < 6; ++k) st[k] = T(p.seed_state[k * p.ld_seed + s]);
#pragma unroll
    for (int k = 0; k < 21; ++k) cv[k] = T(p.seed_cov[k * p.ld_seed + s]);
#pragma unroll
    for (int k = 0; k < 6; ++k) at(cur, 0, k) = st[k];
#pragma unroll
    for (int k = 0; k < 21; ++k) at(cur, 0, 6 + k) = cv[k];
    at(cur, 0, 27) = __int_as_float(3);
    at(cur, 0, 28) = 0.f;
    at(cur, 0, 29) = __int_as_float(finite6_21(st, cv) ? 0 : ST_NONFINITE);
  }
  uint32_t n_box = 0, n_chi2 = 0, n_comp = 0, n_steps = 0, n_upd = 0, n_fb = 0;
  extern __shared__ __align__(16) unsigned char build_lds[];
  ScanLds<T, false>& C = reinterpret_cast<ScanLds<T, false>*>(build_lds)[threadIdx.x >> 6];
  const uint64_t lanes_below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const float4* recs = reinterpret_cast<const float4*>(p.binned);

  for (int l = p.first_layer; l < L; ++l) {
    const int64_t el = static_cast<int64_t>(ev) * L + l;
    // the seed's best N children over all of its candidates: rank keys, slots, accumulated chi2
    uint64_t skey[kSerialMax];
    int32_t sslot[kSerialMax];
    float sc2[kSerialMax];
#pragma unroll
    for (int t = 0; t < kSerialMax; ++t) {
      skey[t] = ~0ull;
      sslot[t] = -1;
      sc2[t] = 0.f;
    }
    const int max_nc = wave_max_i(nc);
#pragma unroll 1
    for (int c = 0; c < max_nc; ++c) {
      const bool active = c < nc;
      T ps[6], pc[21];
      int nhits = 0;
      T chi2 = T(0);
      int32_t status = 0;
      if (active) {
#pragma unroll
        for (int k = 0; k < 6; ++k) ps[k] = at(cur, c, k);
#pragma unroll
        for (int k = 0; k < 21; ++k) pc[k] = at(cur, c, 6 + k);
        nhits = __float_as_int(at(cur, c, 27));
        chi2 = at(cur, c, 28);
        status = __float_as_int(at(cur, c, 29));
      } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) ps[k] = T(0);
#pragma unroll
        for (int k = 0; k < 21; ++k) pc[k] = T(0);
      }
      // propagate (material of the layer the candidate sits on, then the crossing); a failing step keeps the
      // state before it and the candidate is carried unchanged
      int32_t pstat = status;
      n_steps += __popcll(__ballot(active && status == 0));
      if (active && status == 0) {
        T ss[6], sv[21];
#pragma unroll
        for (int k = 0; k < 6; ++k) ss[k] = ps[k];
#pragma unroll
        for (int k = 0; k < 21; ++k) sv[k] = pc[k];
        int32_t r = material(ps, pc, T(p.g.x_over_x0[l - 1]), T(p.g.eloss_per_x0), T(p.g.mass));
        if (!r) r = propagate(ps, pc, a, T(p.g.r[l]), T(p.g.z_half[l]));
        if (r) {
          pstat = r;
#pragma unroll
          for (int k = 0; k < 6; ++k) ps[k] = ss[k];
#pragma unroll
          for (int k = 0; k < 21; ++k) pc[k] = sv[k];
        }
      }
      if (active) {  // the propagated state replaces the candidate's (the survivors start from it)
#pragma unroll
        for (int k = 0; k < 6; ++k) at(cur, c, k) = ps[k];
#pragma unroll
        for (int k = 0; k < 21; ++k) at(cur, c, 6 + k) = pc[k];
        at(cur, c, 29) = __int_as_float(pstat);
      }
      ChildList<T, kSerialMax> kids;
      kids.clear();
      int cnt = 0, cnt_in = 0;
      scan_window<kSerialMax, T, false>(p, C, nullptr, l, el, active && pstat == 0, ps, pc, qf, chi2, N, lane,
                                        lanes_below, recs, kids, cnt, cnt_in, n_box, n_chi2, n_comp, n_fb);
      // the candidate's children into the seed's list: its compatible hits (if it was propagated), else or
      // besides them its hole child
      if (active) {
#pragma unroll
        for (int t = 0; t <= kSerialMax; ++t) {
          uint64_t nk;
          int32_t nj;
          float nc2;
          if (t < kSerialMax) {
            if (!(pstat == 0 && t < cnt)) continue;
            nk = make_key(nhits + 1, float(kids.chi2_at(t)), c, static_cast<uint32_t>(kids.idx_at(t)));
            nj = kids.slot_at(t);
            nc2 = float(kids.chi2_at(t));
          } else {
            nk = make_key(nhits, float(chi2), c, kHole);
            nj = -1;
            nc2 = float(chi2);
          }
#pragma unroll
          for (int u = 0; u < kSerialMax; ++u) {
            const bool sw = u < N && nk < skey[u];
            const uint64_t tk = skey[u];
            const int32_t tj = sslot[u];
            const float tc = sc2[u];
            skey[u] = sw ? nk : tk;
            sslot[u] = sw ? nj : tj;
            sc2[u] = sw ? nc2 : tc;
            nk = sw ? tk : nk;
            nj = sw ? tj : nj;
            nc2 = sw ? tc : nc2;
          }
        }
      }
    }
    // the survivors: each starts from its parent's propagated state and, with a hit, is updated (clone engine)
    int new_nc = 0;
#pragma unroll
    for (int t = 0; t < kSerialMax; ++t) new_nc += (t < N && skey[t] != ~0ull) ? 1 : 0;
    const int nxt = cur ^ 1;
    const int max_new = wave_max_i(new_nc);
#pragma unroll 1
    for (int r = 0; r < max_new; ++r) {
      const bool on = r < new_nc;
      const uint64_t k = sel_key(skey, r);
      const int par = on ? key_parent(k) : 0;
      const uint32_t hid = key_hit(k);
      T st[6], cv[21];
      int32_t status = 0;
      if (on) {
#pragma unroll
        for (int q = 0; q < 6; ++q) st[q] = at(cur, par, q);
#pragma unroll
        for (int q = 0; q < 21; ++q) cv[q] = at(cur, par, 6 + q);
        status = __float_as_int(at(cur, par, 29));
      }
      n_upd += __popcll(__ballot(on && hid != kHole && status == 0));
      if (on && hid != kHole && status == 0) {
        const int32_t sl = sel_i32(sslot, r);
        const float4 h = recs[static_cast<int64_t>(sl) * 3];
        const float4 c0 = recs[static_cast<int64_t>(sl) * 3 + 1];
        const float4 c1 = recs[static_cast<int64_t>(sl) * 3 + 2];
        const float m[3] = {h.x, h.y, h.z};
        const float v[6] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y};
        T dc2;
        const int32_t rr = update_on_layer<T, double>(st, cv, m, v, dc2);
        if (rr) status = rr;
      }
      if (on) {
#pragma unroll
        for (int q = 0; q < 6; ++q) at(nxt, r, q) = st[q];
#pragma unroll
        for (int q = 0; q < 21; ++q) at(nxt, r, 6 + q) = cv[q];
        at(nxt, r, 27) = __int_as_float(key_nhits(k));
        at(nxt, r, 28) = sel_f(sc2, r);
        at(nxt, r, 29) = __int_as_float(status);
        p.cand_hits[static_cast<int64_t>(l) * p.n_seeds * N + s * N + r] =
            static_cast<int32_t>((static_cast<uint32_t>(par) << 24) | hid);
      }
    }
    nc = new_nc;
    cur = nxt;
  }
  // ---- outputs
  if (seed_ok) {
    p.n_cands[s] = nc;
    for (int r = 0; r < N; ++r) {
      const bool live = r < nc;
      p.cand_chi2[s * N + r] = live ? at(cur, r, 28) : 0.f;
      p.cand_nhits[s * N + r] = live ? __float_as_int(at(cur, r, 27)) : 0;
      p.cand_status[s * N + r] = live ? __float_as_int(at(cur, r, 29)) : 0;
    }
    if (p.best_state) {
#pragma unroll
      for (int k = 0; k < 6; ++k) p.best_state[k * p.ld_seed + s] = at(cur, 0, k);
#pragma unroll
      for (int k = 0; k < 21; ++k) p.best_cov[k * p.ld_seed + s] = at(cur, 0, 6 + k);
    }
    // backtrack each final candidate's parent chain: one lane holds all of the seed's chains, so it reads a
    // layer's records before it rewrites them
    int32_t kk[kSerialMax];
#pragma unroll
    for (int r = 0; r < kSerialMax; ++r) kk[r] = r;
    for (int l = L - 1; l >= p.first_layer; --l) {
      int32_t* row = p.cand_hits + static_cast<int64_t>(l) * p.n_seeds * N + s * N;
      int32_t out[kSerialMax];
#pragma unroll
      for (int r = 0; r < kSerialMax; ++r) {
        out[r] = -1;
        if (r < nc) {
          const uint32_t rec = static_cast<uint32_t>(row[kk[r]]);
          const uint32_t hid = rec & kHole;
          kk[r] = static_cast<int>(rec >> 24);
          out[r] = (hid == kHole) ? -1 : static_cast<int32_t>(p.layer_offsets[static_cast<int64_t>(ev) * L + l] + hid);
        }
      }
#pragma unroll
      for (int r = 0; r < kSerialMax; ++r)
        if (r < N) row[r] = out[r];
    }
    for (int l = 0; l < p.first_layer; ++l)
      for (int r = 0; r < N; ++r)
        p.cand_hits[static_cast<int64_t>(l) * p.n_seeds * N + s * N + r] =
            (r < nc && l < 3) ? p.seed_hits[l * p.ld_seed + s] : -1;
  }
  if (p.counters && lane == 0) {
    const uint32_t v[KF_BUILD_COUNTERS] = {n_box, n_chi2, n_comp, n_steps, n_upd, n_fb};
#pragma unroll
    for (int i = 0; i < KF_BUILD_COUNTERS; ++i)
      if (v[i]) atomicAdd(&p.counters[i], static_cast<unsigned long long>(v[i]));
  }
}

__global__ void __launch_bounds__(256) build_serial_kernel(BuildP p) {
  build_serial_tile(p, static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6));
}

// forward weights of the window network, staged once per block (learned-window kernels only)
template <bool LW>
struct MlpLds {
  __device__ static const unsigned char* stage(const unsigned char*) { return nullptr; }
};
template <>
struct MlpLds<true> {
  __device__ static const unsigned char* stage(const unsigned char* packed) {
    __shared__ __align__(16) unsigned char w[kfm::kFwdBytes];
    kfm::stage_forward(packed, w);
    return w;
  }
};

template <int G, typename T, bool LW>
__device__ __forceinline__ void tiled_body(const BuildP& p) {
  const unsigned char* wl = MlpLds<LW>::stage(p.mlp);
  // Workgroups are dealt to the accelerator dies round robin (block b on die b % kXcds).  Blocks are renumbered so
  // that each die takes runs of kXcdRun consecutive blocks: neighbouring tiles (neighbouring directions of one
  // event, whose windows share hit records) then run on the same die and share its L2.  The last incomplete
  // group of kXcds * kXcdRun blocks keeps its numbering.
  int64_t b = blockIdx.x;
  const int64_t grp = static_cast<int64_t>(kXcds) * kXcdRun;
  if (b < static_cast<int64_t>(gridDim.x) / grp * grp) {
    const int64_t r = b % grp;
    b = b - r + (r % kXcds) * kXcdRun + r / kXcds;
  }
  const int64_t tile = b * (blockDim.x >> 6) + (threadIdx.x >> 6);
  build_tile<G, T, LW>(p, tile, wl);
}

template <int G, typename T, bool LW>
__device__ __forceinline__ void persistent_body(const BuildP& p, int64_t n_tiles) {
  const unsigned char* wl = MlpLds<LW>::stage(p.mlp);
  const int lane = threadIdx.x & 63;
  // Each die has a counter and takes the tile sequence in runs of kXcdRun tiles, run r of die c being tiles
  // [(r kXcds + c) kXcdRun, ... + kXcdRun), the runs the tiled launch deals to it: every die starts on the dense
  // events (the sequence is ordered densest first) and works on neighbouring directions at a time, which share
  // hit records in its L2.  Workgroups are dealt to the dies round robin, so a block serves its own die's runs
  // first and then helps with the other dies' in turn.  A die's tiles increase with its counter, so the first
  // index past the end means its runs are exhausted.
  // (one loop with a single call site of the tile body, so that the body is inlined once)
  const int home = static_cast<int>(blockIdx.x % kXcds);
  int k = 0, c = home;
#pragma unroll 1
  for (;;) {
    int32_t j = 0;
    if (lane == 0) j = atomicAdd(&p.queue[c], 1);
    j = __builtin_amdgcn_readfirstlane(j);
    const int64_t tile = ((static_cast<int64_t>(j) / kXcdRun) * kXcds + c) * kXcdRun + (j % kXcdRun);
    if (tile < n_tiles) {
      // the arguments are addressed through the counter value (j >> 31 is 0), so that their loads stay inside
      // the iteration instead of being held in registers across the loop
      build_tile<G, T, LW>((&p)[j >> 31], tile, wl);
      continue;
    }
    if (++k == kXcds) break;  // every die's runs are exhausted
    c = (home + k) % kXcds;
  }
}

// Entry kernels.  The single-precision tiled and persistent builds are compiled for three waves per SIMD (at
// most 168 registers): the build is bound by the latency of its dependent LDS and memory chains, which more
// resident waves hide.  The persistent loop addresses the arguments through its tile number, so that their
// scalar loads are issued inside each tile rather than held in registers across the loop.
template <int G, bool LW>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) build_tiled_kernel(BuildP p) {
  tiled_body<G, float, LW>(p);
}

template <int G, bool LW>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
build_persistent_kernel(BuildP p, int64_t n_tiles) {
  persistent_body<G, float, LW>(p, n_tiles);
}

template <int G, bool LW>
__global__ void __launch_bounds__(256) build_tiled_kernel_f64(BuildP p) {
  tiled_body<G, double, LW>(p);
}

template <int G, bool LW>
__global__ void __launch_bounds__(256) build_persistent_kernel_f64(BuildP p, int64_t n_tiles) {
  persistent_body<G, double, LW>(p, n_tiles);
}

// ---------------------------------------------------------------------------
// seed ordering: seeds of an event grouped by the direction of their position
// (kSeedPhi x kSeedEta cells), so that a wave's windows fall on neighbouring
// bins and share cached hit records.  Results do not depend on the order.
// ---------------------------------------------------------------------------
constexpr int kSeedPhi = 64, kSeedEta = 32, kSeedCells = kSeedPhi * kSeedEta;

__device__ __forceinline__ int seed_event_of(const int64_t* seed_offsets, int n_events, int64_t s) {
  int lo = 0, hi = n_events;  // seed_offsets[lo] <= s < seed_offsets[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (seed_offsets[mid] <= s) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int seed_cell(const float* __restrict__ st, int64_t ld, int64_t s) {
  const float x = st[s], y = st[ld + s], z = st[2 * ld + s];
  const float r2 = x * x + y * y;
  const float phi = atan2f(y, x);
  const float eta = asinh_hw(z * __builtin_amdgcn_rsqf(r2));  // a cell of the tile order: any rounding will do
  if (!(r2 > 0.f) || !isfinite(phi) || !isfinite(eta)) return 0;
  int ip = static_cast<int>((phi + 3.14159265f) * (kSeedPhi / 6.2831853f));
  int ie = static_cast<int>((eta + 2.f) * (kSeedEta / 4.f));
  ip = ip < 0 ? 0 : (ip > kSeedPhi - 1 ? kSeedPhi - 1 : ip);
  ie = ie < 0 ? 0 : (ie > kSeedEta - 1 ? kSeedEta - 1 : ie);
  return ip * kSeedEta + ie;
}

__global__ void __launch_bounds__(256) seed_count_kernel(int64_t n_seeds, int32_t n_events,
                                                         const int64_t* __restrict__ seed_offsets,
                                                         const float* __restrict__ st, int64_t ld,
                                                         int32_t* __restrict__ cells) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= n_seeds) return;
  const int e = seed_event_of(seed_offsets, n_events, s);
  atomicAdd(&cells[static_cast<int64_t>(e) * kSeedCells + seed_cell(st, ld, s)], 1);
}

// Where each event's seeds start in the tile order: events with more seeds (denser events, whose tiles cost
// more) first, ties by index, so that the expensive tiles start early and the cheap ones fill in behind them.
// One block; beyond kOrderMax events the events keep index order.
__global__ void __launch_bounds__(1024) event_base_kernel(int32_t n_events, const int64_t* __restrict__ seed_offsets,
                                                          int64_t* __restrict__ base) {
  __shared__ int32_t cnt[kOrderMax];
  if (n_events > kOrderMax) {
    for (int e = threadIdx.x; e < n_events; e += blockDim.x) base[e] = seed_offsets[e];
    return;
  }
  for (int e = threadIdx.x; e < n_events; e += blockDim.x)
    cnt[e] = static_cast<int32_t>(seed_offsets[e + 1] - seed_offsets[e]);
  __syncthreads();
  for (int e = threadIdx.x; e < n_events; e += blockDim.x) {
    const int32_t v = cnt[e];
    int64_t b = seed_offsets[0];
    for (int f = 0; f < n_events; ++f) {
      const int32_t w = cnt[f];
      b += (w > v || (w == v && f < e)) ? w : 0;
    }
    base[e] = b;
  }
}

// one block per event: exclusive scan of its cell counts, offset by where the event's seeds start
__global__ void __launch_bounds__(1024) seed_scan_kernel(const int64_t* __restrict__ base,
                                                         int32_t* __restrict__ cells) {
  __shared__ int32_t part[1024];
  const int e = blockIdx.x;
  int32_t* c = cells + static_cast<int64_t>(e) * kSeedCells;
  constexpr int per = kSeedCells / 1024;
  const int t = threadIdx.x;
  int32_t v[per];
  int32_t sum = 0;
#pragma unroll
  for (int k = 0; k < per; ++k) {
    v[k] = c[t * per + k];
    sum += v[k];
  }
  part[t] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int32_t y = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += y;
    __syncthreads();
  }
  int32_t run = static_cast<int32_t>(base[e]) + part[t] - sum;
#pragma unroll
  for (int k = 0; k < per; ++k) {
    c[t * per + k] = run;
    run += v[k];
  }
}

__global__ void __launch_bounds__(256) seed_scatter_kernel(int64_t n_seeds, int32_t n_events,
                                                           const int64_t* __restrict__ seed_offsets,
                                                           const float* __restrict__ st, int64_t ld,
                                                           int32_t* __restrict__ cells, int32_t* __restrict__ order) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= n_seeds) return;
  const int e = seed_event_of(seed_offsets, n_events, s);
  const int32_t at = atomicAdd(&cells[static_cast<int64_t>(e) * kSeedCells + seed_cell(st, ld, s)], 1);
  order[at] = static_cast<int32_t>(s);
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// lanes per seed: the candidates of a seed sit in G consecutive lanes (G = 6 keeps 60 of 64 lanes busy for N = 5, 6)
int lanes_for(int n) { return n <= 1 ? 1 : n <= 2 ? 2 : n <= 4 ? 4 : n <= 6 ? 6 : 8; }

struct Launch {
  bool persistent, f64, learned;
  unsigned grid, block;
  hipStream_t stream;
  int64_t n_tiles;
  int n_back;  // layers with a back-pointer (n_layers - first_layer)
};

template <int G, typename T, bool LW>
void launch_build(const Launch& c, const BuildP& p) {
  const size_t lds = (c.block / 64) * (sizeof(ScanLds<T, LW>) + (kBackLds<LW> ? c.n_back * 64 * sizeof(int32_t) : 0));
  if constexpr (std::is_same<T, float>::value) {
    if (c.persistent)
      build_persistent_kernel<G, LW><<<c.grid, c.block, lds, c.stream>>>(p, c.n_tiles);
    else
      build_tiled_kernel<G, LW><<<c.grid, c.block, lds, c.stream>>>(p);
  } else {
    if (c.persistent)
      build_persistent_kernel_f64<G, LW><<<c.grid, c.block, lds, c.stream>>>(p, c.n_tiles);
    else
      build_tiled_kernel_f64<G, LW><<<c.grid, c.block, lds, c.stream>>>(p);
  }
}

template <int G>
void launch_g(const Launch& c, const BuildP& p) {
  if (c.f64) {
    if (c.learned) launch_build<G, double, true>(c, p); else launch_build<G, double, false>(c, p);
  } else {
    if (c.learned) launch_build<G, float, true>(c, p); else launch_build<G, float, false>(c, p);
  }
}

void launch_any(int G, const Launch& c, const BuildP& p) {
  switch (G) {
    case 1: launch_g<1>(c, p); break;
    case 2: launch_g<2>(c, p); break;
    case 4: launch_g<4>(c, p); break;
    case 6: launch_g<6>(c, p); break;
    default: launch_g<8>(c, p); break;
  }
}

}  // namespace

using kfh::set_error;

extern "C" {

// per-hit bin ids, then the launch order of the (event, layer) pairs (room for the largest layer count)
static size_t bin_ids_bytes(int64_t ldh) { return (static_cast<size_t>(ldh > 0 ? ldh : 0) * 4u + 255) & ~size_t(255); }
size_t kf_bin_hits_workspace_size(int64_t ldh, int64_t n_events) {
  return bin_ids_bytes(ldh) + static_cast<size_t>(n_events > 0 ? n_events : 0) * KF_MAX_LAYERS * 4u;
}

int32_t kf_bin_hits(kf_ctx* ctx, const kf_bin_args* a) {
  if (int32_t rc = kfh::enter(ctx)) return rc;
  if (!a) return set_error(KF_ERR_INVALID_ARG, "null args");
  if (!ctx->has_geometry) return set_error(KF_ERR_GEOMETRY, "no geometry set");
  if (a->n_events < 0 || a->ldh < 0) return set_error(KF_ERR_INVALID_ARG, "bad sizes");
  if (a->n_phi < 1 || a->n_eta < 1 || static_cast<int64_t>(a->n_phi) * a->n_eta > kMaxBinsFine)
    return set_error(KF_ERR_INVALID_ARG, "need 1 <= n_phi * n_eta <= %d", kMaxBinsFine);
  if (a->ldh >= (int64_t(1) << 31)) return set_error(KF_ERR_INVALID_ARG, "too many hits for int32 slots");
  if (a->n_events == 0) return KF_OK;
  if (!a->layer_offsets || !a->hit_pos || !a->hit_cov || !a->bin_offsets || !a->perm || !a->binned ||
      !a->layer_vmax)
    return set_error(KF_ERR_INVALID_ARG, "null array");
  if (!a->workspace || a->workspace_bytes < kf_bin_hits_workspace_size(a->ldh, a->n_events))
    return set_error(KF_ERR_WORKSPACE, "workspace of %zu bytes needed", kf_bin_hits_workspace_size(a->ldh, a->n_events));
  const int L = ctx->geom.n_layers;
  const int64_t n_el = a->n_events * L;
  if (n_el > INT32_MAX) return set_error(KF_ERR_INVALID_ARG, "too many (event, layer) pairs");
  const int nb = a->n_phi * a->n_eta;
  hipStream_t sm = kfh::stream_of(a->stream);
  int32_t* el_order = nullptr;  // index order beyond kOrderMax pairs
  if (n_el <= kOrderMax) {
    el_order = reinterpret_cast<int32_t*>(static_cast<char*>(a->workspace) + bin_ids_bytes(a->ldh));
    el_order_kernel<<<static_cast<unsigned>((n_el + kOrderThreads - 1) / kOrderThreads), kOrderThreads, 0, sm>>>(
        static_cast<int32_t>(n_el), a->layer_offsets, el_order);
    if (int32_t rc = kfh::check_hip(hipGetLastError(), "el_order_kernel launch")) return rc;
  }
  if (nb <= kMaxBins) {
    const size_t lds_bytes = static_cast<size_t>(kBinWaves + 1) * nb * sizeof(int32_t);
    if (int32_t rc = kfh::check_hip(hipFuncSetAttribute(reinterpret_cast<const void*>(bin_kernel),
                                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                                        static_cast<int>((kBinWaves + 1) * kMaxBins * sizeof(int32_t))),
                                    "hipFuncSetAttribute(bin_kernel)"))
      return rc;
    bin_kernel<<<static_cast<unsigned>(n_el), kBinThreads, lds_bytes, sm>>>(
        L, a->layer_offsets, a->hit_pos, a->hit_cov, a->ldh, a->n_phi, a->n_eta, ctx->dgeom,
        static_cast<int32_t*>(a->workspace), a->bin_offsets, a->perm, a->binned, a->layer_vmax, el_order);
    return kfh::check_hip(hipGetLastError(), "bin_kernel launch");
  }
  if (int32_t rc = kfh::check_hip(hipFuncSetAttribute(reinterpret_cast<const void*>(bin_fine_kernel),
                                                      hipFuncAttributeMaxDynamicSharedMemorySize,
                                                      static_cast<int>(kMaxBinsFine * sizeof(int32_t))),
                                  "hipFuncSetAttribute(bin_fine_kernel)"))
    return rc;
  bin_fine_kernel<<<static_cast<unsigned>(n_el), kBinThreads, static_cast<size_t>(nb) * sizeof(int32_t), sm>>>(
      L, a->layer_offsets, a->hit_pos, a->hit_cov, a->ldh, a->n_phi, a->n_eta, ctx->dgeom,
      static_cast<int32_t*>(a->workspace), a->bin_offsets, a->perm, a->binned, a->layer_vmax, el_order);
  return kfh::check_hip(hipGetLastError(), "bin_fine_kernel launch");
}

namespace {
constexpr size_t kQueueBytes = 256;
size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
// serial-candidate build: the two candidate buffers, one slot per tile position (tiles of 64 seeds)
size_t serial_buf_bytes(const kf_build_cfg* cfg, int64_t n_seeds) {
  const int64_t ld = (n_seeds + 63) / 64 * 64;
  const int n = cfg->max_cands >= 1 && cfg->max_cands <= 8 ? cfg->max_cands : 8;
  return align256(static_cast<size_t>(2) * kSerialWords * n * ld * sizeof(float));
}
size_t cells_bytes(int64_t n_events) { return align256(static_cast<size_t>(n_events) * kSeedCells * 4); }
}  // namespace

size_t kf_build_workspace_size(const kf_build_cfg* cfg, int64_t n_events, int64_t n_seeds) {
  if (!cfg || n_events < 0 || n_seeds < 0) return 0;
  size_t b = kQueueBytes;  // persistent work queue (kept in every layout)
  if (cfg->seed_order)
    b += cells_bytes(n_events) + align256(static_cast<size_t>(n_seeds) * 4) + align256(static_cast<size_t>(n_events) * 8);
  if (cfg->mode == KF_BUILD_SERIAL) return b + serial_buf_bytes(cfg, n_seeds);
  return (cfg->mode == KF_BUILD_PERSISTENT || cfg->seed_order) ? b : 0;
}

}  // extern "C"

namespace {

// Static scratch of kf_build_noalloc: the work queue, direction cells and seed order that kf_build keeps in the
// caller's workspace.  Each device the library runs on holds one copy until the process ends; kernels receive
// its device address (kf_ctx::scratch, from hipGetSymbolAddress), never this host-side name.
constexpr size_t kScratchBytes = KF_BUILD_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes == (size_t(16) << 20), "scratch size");
__device__ __align__(256) unsigned char scratch[kScratchBytes];

int32_t build_impl(kf_ctx* ctx, const kf_build_cfg* cfg, const kf_build_args* a, void* workspace,
                   size_t workspace_bytes);

}  // namespace

int32_t kfh::scratch_init(kf_ctx* ctx) {
  void* ptr = nullptr;
  if (int32_t rc = check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"))
    return rc;
  ctx->scratch = ptr;
  ctx->scratch_bytes = kScratchBytes;
  return KF_OK;
}

extern "C" {

int32_t kf_build(kf_ctx* ctx, const kf_build_cfg* cfg, const kf_build_args* a) {
  if (int32_t rc = kfh::enter(ctx)) return rc;
  if (!a) return set_error(KF_ERR_INVALID_ARG, "null args");
  return build_impl(ctx, cfg, a, a->workspace, a->workspace_bytes);
}

int32_t kf_build_noalloc(kf_ctx* ctx, const kf_build_cfg* cfg, const kf_build_args* a) {
  if (int32_t rc = kfh::enter(ctx)) return rc;
  if (!cfg || !a) return set_error(KF_ERR_INVALID_ARG, "null args");
  if (!ctx->scratch) return set_error(KF_ERR_DEVICE, "static scratch not initialised for device %d", ctx->device);
  const size_t need = kf_build_workspace_size(cfg, a->n_events, a->n_seeds);
  if (need > ctx->scratch_bytes)
    return set_error(KF_ERR_WORKSPACE, "kf_build_noalloc: this problem needs %zu bytes of scratch, the static maximum "
                     "is %zu (use kf_build with a workspace)", need, ctx->scratch_bytes);
  return build_impl(ctx, cfg, a, ctx->scratch, ctx->scratch_bytes);
}

}  // extern "C"

namespace {

int32_t build_impl(kf_ctx* ctx, const kf_build_cfg* cfg, const kf_build_args* a, void* workspace,
                   size_t workspace_bytes) {
  if (!cfg || !a) return set_error(KF_ERR_INVALID_ARG, "null args");
  if (!ctx->has_geometry) return set_error(KF_ERR_GEOMETRY, "no geometry set");
  const int L = ctx->geom.n_layers;
  if (cfg->max_cands < 1 || cfg->max_cands > 8) return set_error(KF_ERR_INVALID_ARG, "max_cands must be 1..8");
  if (!(cfg->chi2_cut > 0.f)) return set_error(KF_ERR_INVALID_ARG, "chi2_cut must be > 0");
  if (cfg->n_phi < 1 || cfg->n_eta < 1 || static_cast<int64_t>(cfg->n_phi) * cfg->n_eta > kMaxBinsFine)
    return set_error(KF_ERR_INVALID_ARG, "bad bin counts");
  if (!(cfg->window_margin >= 0.f)) return set_error(KF_ERR_INVALID_ARG, "window_margin must be >= 0");
  if (cfg->mode != KF_BUILD_TILED && cfg->mode != KF_BUILD_PERSISTENT && cfg->mode != KF_BUILD_SERIAL)
    return set_error(KF_ERR_INVALID_ARG, "unknown mode %d", cfg->mode);
  if (cfg->mode == KF_BUILD_SERIAL && (cfg->window_mode != KF_WINDOW_PLAIN || cfg->precision != KF_PREC_F32))
    return set_error(KF_ERR_UNSUPPORTED, "the serial-candidate build supports the plain window in single precision");
  if (cfg->window_mode != KF_WINDOW_PLAIN && cfg->window_mode != KF_WINDOW_LEARNED)
    return set_error(KF_ERR_INVALID_ARG, "unknown window mode %d", cfg->window_mode);
  if (cfg->window_mode == KF_WINDOW_LEARNED) {
    if (!(cfg->learned_nsigma > 0.f) || !std::isfinite(cfg->learned_nsigma))
      return set_error(KF_ERR_INVALID_ARG, "learned_nsigma must be > 0");
    if (!a->mlp_packed) return set_error(KF_ERR_INVALID_ARG, "learned window without mlp_packed");
  }
  if (cfg->precision != KF_PREC_F32 && cfg->precision != KF_PREC_F64)
    return set_error(KF_ERR_INVALID_ARG, "unknown precision %d", cfg->precision);
  if (a->n_events < 0 || a->n_seeds < 0 || a->ld_seed < a->n_seeds)
    return set_error(KF_ERR_INVALID_ARG, "bad sizes");
  if (a->first_layer < 3 || a->first_layer > L) return set_error(KF_ERR_INVALID_ARG, "first_layer must be in [3, L]");
  if (a->n_seeds == 0) return KF_OK;
  if (a->n_events < 1 || a->n_events > INT32_MAX) return set_error(KF_ERR_INVALID_ARG, "bad n_events");
  if (!a->seed_offsets || !a->seed_state || !a->seed_cov || !a->seed_charge || !a->seed_hits || !a->layer_offsets ||
      !a->bin_offsets || !a->binned || !a->layer_vmax || !a->n_cands || !a->cand_hits || !a->cand_chi2 ||
      !a->cand_nhits || !a->cand_status)
    return set_error(KF_ERR_INVALID_ARG, "null array");
  if ((a->best_state == nullptr) != (a->best_cov == nullptr))
    return set_error(KF_ERR_INVALID_ARG, "best_state and best_cov go together");
  if (a->n_seeds * static_cast<int64_t>(cfg->max_cands) * L > INT64_MAX / 8)
    return set_error(KF_ERR_INVALID_ARG, "too many seeds");
  BuildP p;
  p.n_seeds = a->n_seeds;
  p.ld_seed = a->ld_seed;
  p.n_events = static_cast<int32_t>(a->n_events);
  p.first_layer = a->first_layer;
  p.max_cands = cfg->max_cands;
  p.n_phi = cfg->n_phi;
  p.n_eta = cfg->n_eta;
  p.chi2_cut = cfg->chi2_cut;
  p.margin = cfg->window_margin;
  p.seed_offsets = a->seed_offsets;
  p.seed_state = a->seed_state;
  p.seed_cov = a->seed_cov;
  p.seed_charge = a->seed_charge;
  p.seed_hits = a->seed_hits;
  p.layer_offsets = a->layer_offsets;
  p.bin_offsets = a->bin_offsets;
  p.binned = a->binned;
  p.layer_vmax = a->layer_vmax;
  p.n_cands = a->n_cands;
  p.cand_hits = a->cand_hits;
  p.cand_chi2 = a->cand_chi2;
  p.cand_nhits = a->cand_nhits;
  p.cand_status = a->cand_status;
  p.best_state = a->best_state;
  p.best_cov = a->best_cov;
  p.counters = reinterpret_cast<unsigned long long*>(a->counters);
  p.queue = nullptr;
  p.cand_buf = nullptr;
  p.buf_ld = 0;
  p.mlp = cfg->window_mode == KF_WINDOW_LEARNED ? static_cast<const unsigned char*>(a->mlp_packed) : nullptr;
  p.nsigma = cfg->learned_nsigma;
  p.g = ctx->dgeom;
  const int G = lanes_for(cfg->max_cands);
  const int64_t spw = 64 / G;
  const int64_t n_tiles = (a->n_seeds + spw - 1) / spw;
  const int wpb = cfg->waves_per_block > 0 ? cfg->waves_per_block : 4;
  if (wpb > 4) return set_error(KF_ERR_INVALID_ARG, "waves_per_block must be 1..4");
  hipStream_t stream = kfh::stream_of(a->stream);
  const size_t need = kf_build_workspace_size(cfg, a->n_events, a->n_seeds);
  if (need > 0 && (!workspace || workspace_bytes < need))
    return set_error(KF_ERR_WORKSPACE, "this configuration needs kf_build_workspace_size() = %zu bytes of workspace",
                     need);
  p.order = nullptr;
  if (cfg->seed_order) {
    if (a->n_seeds > INT32_MAX) return set_error(KF_ERR_INVALID_ARG, "seed_order needs n_seeds < 2^31");
    unsigned char* w = static_cast<unsigned char*>(workspace);
    int32_t* cells = reinterpret_cast<int32_t*>(w + kQueueBytes);
    int32_t* order = reinterpret_cast<int32_t*>(w + kQueueBytes + cells_bytes(a->n_events));
    const int64_t nc = a->n_events * kSeedCells;
    fill_i32_kernel<<<kfh::grid_for(nc, 256), 256, 0, stream>>>(cells, nc, 0);
    seed_count_kernel<<<kfh::grid_for(a->n_seeds, 256), 256, 0, stream>>>(
        a->n_seeds, static_cast<int32_t>(a->n_events), a->seed_offsets, a->seed_state, a->ld_seed, cells);
    int64_t* base = reinterpret_cast<int64_t*>(w + kQueueBytes + cells_bytes(a->n_events) +
                                               align256(static_cast<size_t>(a->n_seeds) * 4));
    event_base_kernel<<<1, 1024, 0, stream>>>(static_cast<int32_t>(a->n_events), a->seed_offsets, base);
    seed_scan_kernel<<<static_cast<unsigned>(a->n_events), 1024, 0, stream>>>(base, cells);
    seed_scatter_kernel<<<kfh::grid_for(a->n_seeds, 256), 256, 0, stream>>>(
        a->n_seeds, static_cast<int32_t>(a->n_events), a->seed_offsets, a->seed_state, a->ld_seed, cells, order);
    if (int32_t rc = kfh::check_hip(hipGetLastError(), "seed ordering launch")) return rc;
    p.order = order;
  }
  if (cfg->mode == KF_BUILD_SERIAL) {
    const int64_t tiles64 = (a->n_seeds + 63) / 64;
    p.buf_ld = tiles64 * 64;
    p.cand_buf = reinterpret_cast<float*>(static_cast<unsigned char*>(workspace) + need - serial_buf_bytes(cfg, a->n_seeds));
    const size_t lds = static_cast<size_t>(wpb) * sizeof(ScanLds<float, false>);
    build_serial_kernel<<<static_cast<unsigned>((tiles64 + wpb - 1) / wpb), 64u * wpb, lds, stream>>>(p);
    return kfh::check_hip(hipGetLastError(), "build_serial_kernel launch");
  }
  const bool f64 = cfg->precision == KF_PREC_F64;
  Launch lc;
  lc.f64 = f64;
  lc.learned = p.mlp != nullptr;
  lc.stream = stream;
  lc.n_tiles = n_tiles;
  lc.n_back = L - a->first_layer;
  lc.block = 64u * wpb;
  if (cfg->mode == KF_BUILD_TILED) {
    lc.persistent = false;
    lc.grid = static_cast<unsigned>((n_tiles + wpb - 1) / wpb);
    launch_any(G, lc, p);
    return kfh::check_hip(hipGetLastError(), "build_tiled_kernel launch");
  }
  p.queue = static_cast<int32_t*>(workspace);
  fill_i32_kernel<<<1, 64, 0, stream>>>(p.queue, kXcds, 0);
  const int bpc = cfg->blocks_per_cu > 0 ? cfg->blocks_per_cu : 2;
  lc.persistent = true;
  lc.grid = static_cast<unsigned>(ctx->num_cus * bpc);
  launch_any(G, lc, p);
  return kfh::check_hip(hipGetLastError(), "build_persistent_kernel launch");
}

}  // namespace
