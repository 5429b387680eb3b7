// kf_host_build.hip -- binning and building from host memory with the
// transfers overlapped: events in chunks, input copies / kernels / output
// copies on their own streams linked by events (the kernels of consecutive
// chunks alternate between two streams, so that one chunk's launch tail
// overlaps the next chunk's kernels).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "kf_internal.hpp"

using kfh::set_error;

namespace {

// p[i] -= p[0] for 0 < i < n (offsets of a chunk rebased to its first entry; p[0] itself is cleared by
// rebase_first_kernel afterwards, so every block reads the same base)
__global__ void rebase_i64_kernel(int64_t* __restrict__ p, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i > 0 && i < n) p[i] -= p[0];
}

__global__ void rebase_first_kernel(int64_t* __restrict__ p) { p[0] = 0; }

// p[i] += delta for p[i] >= 0 (global <-> chunk hit indices; -1 = no hit stays)
__global__ void shift_hits_kernel(int32_t* __restrict__ p, int64_t n, int64_t delta) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    const int32_t v = p[i];
    if (v >= 0) p[i] = static_cast<int32_t>(v + delta);
  }
}

struct Chunk {
  int64_t e0, e1, s0, s1, h0, h1;
};

struct Layout {
  std::vector<Chunk> chunks;
  int64_t cap_e = 0, cap_s = 0, cap_h = 0;
  // byte offsets inside one slot, then the shared parts
  size_t pos, cov, lofs, sofs, sst, scv, sq, shit, o_nc, o_hits, o_chi2, o_nh, o_st, o_bs, o_bc, slot_bytes;
  size_t bo, perm, binned, vmax, bin_ws, build_ws, scratch_bytes, total;  // scratch: one set per kernel stream
};

constexpr int kRunStreams = 2;

size_t al(size_t b) { return (b + 255) & ~size_t(255); }

int32_t plan(const kf_ctx* ctx, const kf_build_cfg* cfg, const kf_build_host_args* a, Layout& y) {
  const int L = ctx->geom.n_layers;
  if (a->n_events < 1 || a->n_seeds < 1 || a->n_hits < 0) return set_error(KF_ERR_INVALID_ARG, "bad sizes");
  if (!a->layer_offsets || !a->seed_offsets) return set_error(KF_ERR_INVALID_ARG, "null offsets");
  if (a->n_chunks < 1 || a->n_chunks > a->n_events) return set_error(KF_ERR_INVALID_ARG, "n_chunks must be 1..n_events");
  if (a->n_slots < 1 || a->n_slots > 4) return set_error(KF_ERR_INVALID_ARG, "n_slots must be 1..4");
  const int64_t E = a->n_events;
  if (a->seed_offsets[0] != 0 || a->seed_offsets[E] != a->n_seeds)
    return set_error(KF_ERR_INVALID_ARG, "seed_offsets must run from 0 to n_seeds");
  if (a->layer_offsets[0] != 0 || a->layer_offsets[E * L] != a->n_hits)
    return set_error(KF_ERR_INVALID_ARG, "layer_offsets must run from 0 to n_hits");
  for (int64_t e = 0; e < E; ++e)
    if (a->seed_offsets[e + 1] < a->seed_offsets[e]) return set_error(KF_ERR_INVALID_ARG, "seed_offsets descend");
  for (int64_t i = 0; i < E * L; ++i) {
    const int64_t d = a->layer_offsets[i + 1] - a->layer_offsets[i];
    if (d < 0) return set_error(KF_ERR_INVALID_ARG, "layer_offsets descend");
    if (d >= (int64_t(1) << 24) - 1) return set_error(KF_ERR_INVALID_ARG, "an (event, layer) holds 2^24 - 1 or more hits");
  }
  // consecutive events, cut where the running seed count passes k / n_chunks of the total
  y.chunks.clear();
  int64_t e0 = 0;
  for (int k = 1; k <= a->n_chunks && e0 < E; ++k) {
    int64_t e1 = e0 + 1;
    const int64_t target = (a->n_seeds * k) / a->n_chunks;
    const int64_t left = a->n_chunks - k;  // chunks still to fill need an event each
    while (e1 < E - left && a->seed_offsets[e1] < target) ++e1;
    if (k == a->n_chunks) e1 = E;
    Chunk c{e0, e1, a->seed_offsets[e0], a->seed_offsets[e1], a->layer_offsets[e0 * L], a->layer_offsets[e1 * L]};
    y.chunks.push_back(c);
    y.cap_e = std::max(y.cap_e, e1 - e0);
    y.cap_s = std::max(y.cap_s, c.s1 - c.s0);
    y.cap_h = std::max(y.cap_h, c.h1 - c.h0);
    e0 = e1;
  }
  if (y.cap_h >= (int64_t(1) << 31)) return set_error(KF_ERR_INVALID_ARG, "a chunk holds 2^31 or more hits");
  const int64_t N = cfg->max_cands, S = std::max<int64_t>(y.cap_s, 1), H = std::max<int64_t>(y.cap_h, 1);
  const int64_t EL = y.cap_e * L;
  size_t o = 0;
  auto put = [&](size_t bytes) { const size_t at = o; o += al(bytes); return at; };
  y.pos = put(3 * H * 4);
  y.cov = put(6 * H * 4);
  y.lofs = put((EL + 1) * 8);
  y.sofs = put((y.cap_e + 1) * 8);
  y.sst = put(6 * S * 4);
  y.scv = put(21 * S * 4);
  y.sq = put(S);
  y.shit = put(3 * S * 4);
  y.o_nc = put(S * 4);
  y.o_hits = put(static_cast<size_t>(L) * S * N * 4);
  y.o_chi2 = put(S * N * 4);
  y.o_nh = put(S * N * 4);
  y.o_st = put(S * N * 4);
  y.o_bs = put(6 * S * 4);
  y.o_bc = put(21 * S * 4);
  y.slot_bytes = o;
  o = 0;
  const int64_t nb = static_cast<int64_t>(cfg->n_phi) * cfg->n_eta;
  y.bo = put(EL * (nb + 1) * 4);
  y.perm = put(H * 4);
  y.binned = put(H * KF_BINNED_FLOATS * 4);
  y.vmax = put(EL * 2 * 4);
  y.bin_ws = put(kf_bin_hits_workspace_size(H, y.cap_e));
  y.build_ws = put(kf_build_workspace_size(cfg, y.cap_e, S));
  y.scratch_bytes = o;
  y.total = y.slot_bytes * a->n_slots + y.scratch_bytes * kRunStreams;
  return KF_OK;
}

unsigned grid(int64_t n) { return static_cast<unsigned>((n + 255) / 256); }

// `rows` row copies of `width` bytes between arrays with row pitches dpitch / spitch: one plain asynchronous
// copy per row (each a contiguous transfer of the copy engine)
hipError_t copy_rows(void* dst, size_t dpitch, const void* src, size_t spitch, size_t width, size_t rows,
                     hipMemcpyKind kind, hipStream_t s) {
  for (size_t r = 0; r < rows; ++r) {
    const hipError_t e = hipMemcpyAsync(static_cast<char*>(dst) + r * dpitch,
                                        static_cast<const char*>(src) + r * spitch, width, kind, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

size_t kf_build_host_workspace_size(kf_ctx* ctx, const kf_build_cfg* cfg, const kf_build_host_args* a) {
  if (!ctx || !cfg || !a || !ctx->has_geometry) return 0;
  Layout y;
  if (plan(ctx, cfg, a, y) != KF_OK) return 0;
  return y.total;
}

int32_t kf_build_host(kf_ctx* ctx, const kf_build_cfg* cfg, const kf_build_host_args* a) {
  if (int32_t rc = kfh::enter(ctx)) return rc;
  if (!cfg || !a) return set_error(KF_ERR_INVALID_ARG, "null args");
  if (!ctx->has_geometry) return set_error(KF_ERR_GEOMETRY, "no geometry set");
  if (!a->hit_pos || !a->hit_cov || !a->seed_state || !a->seed_cov || !a->seed_charge || !a->seed_hits ||
      !a->n_cands || !a->cand_hits || !a->cand_chi2 || !a->cand_nhits || !a->cand_status)
    return set_error(KF_ERR_INVALID_ARG, "null array");
  if ((a->best_state == nullptr) != (a->best_cov == nullptr))
    return set_error(KF_ERR_INVALID_ARG, "best_state and best_cov go together");
  if (cfg->max_cands < 1 || cfg->max_cands > 8) return set_error(KF_ERR_INVALID_ARG, "max_cands must be 1..8");
  if (a->first_layer < 3 || a->first_layer > ctx->geom.n_layers)
    return set_error(KF_ERR_INVALID_ARG, "first_layer must be in [3, L]");
  Layout y;
  if (int32_t rc = plan(ctx, cfg, a, y)) return rc;
  if (!a->workspace || a->workspace_bytes < y.total)
    return set_error(KF_ERR_WORKSPACE, "kf_build_host needs kf_build_host_workspace_size() = %zu bytes", y.total);
  if (int32_t rc = kfh::pipe_streams(ctx, 3 * static_cast<int>(y.chunks.size()) + 1)) return rc;
  const int L = ctx->geom.n_layers;
  const int64_t N = cfg->max_cands;
  const int64_t S = a->n_seeds, H = a->n_hits;
  hipStream_t caller = kfh::stream_of(a->stream);
  hipStream_t s_in = ctx->pipe[0], s_out = ctx->pipe[1];
  hipEvent_t* ev = ctx->pipe_events.data();  // [0] start, then per chunk: inputs copied, kernels done, outputs copied
  const int K = static_cast<int>(y.chunks.size());
  auto ev_in = [&](int k) { return ev[1 + 3 * k]; };
  auto ev_run = [&](int k) { return ev[2 + 3 * k]; };
  auto ev_out = [&](int k) { return ev[3 + 3 * k]; };
  unsigned char* ws = static_cast<unsigned char*>(a->workspace);
  auto chk = [](hipError_t e, const char* what) { return kfh::check_hip(e, what); };
#define KF_TRY(x, what) \
  do {                  \
    if (int32_t rc_ = chk((x), what)) return rc_; \
  } while (0)
  KF_TRY(hipEventRecord(ev[0], caller), "hipEventRecord");
  for (int i = 0; i < 2 + kRunStreams; ++i) KF_TRY(hipStreamWaitEvent(ctx->pipe[i], ev[0], 0), "hipStreamWaitEvent");
  const hipMemcpyKind h2d = hipMemcpyHostToDevice, d2h = hipMemcpyDeviceToHost;
  for (int k = 0; k < K; ++k) {
    const Chunk& c = y.chunks[k];
    const int64_t Ec = c.e1 - c.e0, Sc = c.s1 - c.s0, Hc = c.h1 - c.h0;
    unsigned char* sl = ws + y.slot_bytes * (k % a->n_slots);
    unsigned char* sc = ws + y.slot_bytes * a->n_slots + y.scratch_bytes * (k % kRunStreams);
    hipStream_t s_run = ctx->pipe[2 + k % kRunStreams];
    float* d_pos = reinterpret_cast<float*>(sl + y.pos);
    float* d_cov = reinterpret_cast<float*>(sl + y.cov);
    int64_t* d_lofs = reinterpret_cast<int64_t*>(sl + y.lofs);
    int64_t* d_sofs = reinterpret_cast<int64_t*>(sl + y.sofs);
    float* d_sst = reinterpret_cast<float*>(sl + y.sst);
    float* d_scv = reinterpret_cast<float*>(sl + y.scv);
    int8_t* d_sq = reinterpret_cast<int8_t*>(sl + y.sq);
    int32_t* d_shit = reinterpret_cast<int32_t*>(sl + y.shit);
    // ---- input copies (the slot is free once its previous chunk's kernels are done)
    if (k >= a->n_slots) KF_TRY(hipStreamWaitEvent(s_in, ev_run(k - a->n_slots), 0), "hipStreamWaitEvent");
    if (Hc > 0) {
      KF_TRY(copy_rows(d_pos, Hc * 4, a->hit_pos + c.h0, H * 4, Hc * 4, 3, h2d, s_in), "copy hit_pos");
      KF_TRY(copy_rows(d_cov, Hc * 4, a->hit_cov + c.h0, H * 4, Hc * 4, 6, h2d, s_in), "copy hit_cov");
    }
    KF_TRY(hipMemcpyAsync(d_lofs, a->layer_offsets + c.e0 * L, (Ec * L + 1) * 8, h2d, s_in), "copy layer_offsets");
    KF_TRY(hipMemcpyAsync(d_sofs, a->seed_offsets + c.e0, (Ec + 1) * 8, h2d, s_in), "copy seed_offsets");
    if (Sc > 0) {
      KF_TRY(copy_rows(d_sst, Sc * 4, a->seed_state + c.s0, S * 4, Sc * 4, 6, h2d, s_in), "copy seed_state");
      KF_TRY(copy_rows(d_scv, Sc * 4, a->seed_cov + c.s0, S * 4, Sc * 4, 21, h2d, s_in), "copy seed_cov");
      KF_TRY(hipMemcpyAsync(d_sq, a->seed_charge + c.s0, Sc, h2d, s_in), "copy seed_charge");
      KF_TRY(copy_rows(d_shit, Sc * 4, a->seed_hits + c.s0, S * 4, Sc * 4, 3, h2d, s_in), "copy seed_hits");
    }
    KF_TRY(hipEventRecord(ev_in(k), s_in), "hipEventRecord");
    // ---- kernels: rebase the chunk's offsets and seed hits, bin, build, shift the hit indices back to global
    KF_TRY(hipStreamWaitEvent(s_run, ev_in(k), 0), "hipStreamWaitEvent");
    // this slot's outputs of the chunk before are on their way to the host
    if (k >= a->n_slots) KF_TRY(hipStreamWaitEvent(s_run, ev_out(k - a->n_slots), 0), "hipStreamWaitEvent");
    rebase_i64_kernel<<<grid(Ec + 1), 256, 0, s_run>>>(d_sofs, Ec + 1);
    rebase_first_kernel<<<1, 1, 0, s_run>>>(d_sofs);
    rebase_i64_kernel<<<grid(Ec * L + 1), 256, 0, s_run>>>(d_lofs, Ec * L + 1);
    rebase_first_kernel<<<1, 1, 0, s_run>>>(d_lofs);
    if (Sc > 0) shift_hits_kernel<<<grid(3 * Sc), 256, 0, s_run>>>(d_shit, 3 * Sc, -c.h0);
    KF_TRY(hipGetLastError(), "rebase kernels");
    if (Sc > 0) {
      kf_bin_args b{};
      b.n_events = Ec;
      b.layer_offsets = d_lofs;
      b.hit_pos = d_pos;
      b.hit_cov = d_cov;
      b.ldh = Hc;
      b.n_phi = cfg->n_phi;
      b.n_eta = cfg->n_eta;
      b.bin_offsets = reinterpret_cast<int32_t*>(sc + y.bo);
      b.perm = reinterpret_cast<int32_t*>(sc + y.perm);
      b.binned = reinterpret_cast<float*>(sc + y.binned);
      b.layer_vmax = reinterpret_cast<float*>(sc + y.vmax);
      b.workspace = sc + y.bin_ws;
      b.workspace_bytes = kf_bin_hits_workspace_size(Hc, Ec);
      b.stream = s_run;
      if (int32_t rc = kf_bin_hits(ctx, &b)) return rc;
      kf_build_args g{};
      g.n_events = Ec;
      g.n_seeds = Sc;
      g.ld_seed = Sc;
      g.first_layer = a->first_layer;
      g.seed_offsets = d_sofs;
      g.seed_state = d_sst;
      g.seed_cov = d_scv;
      g.seed_charge = d_sq;
      g.seed_hits = d_shit;
      g.layer_offsets = d_lofs;
      g.bin_offsets = b.bin_offsets;
      g.binned = b.binned;
      g.layer_vmax = b.layer_vmax;
      g.n_cands = reinterpret_cast<int32_t*>(sl + y.o_nc);
      g.cand_hits = reinterpret_cast<int32_t*>(sl + y.o_hits);
      g.cand_chi2 = reinterpret_cast<float*>(sl + y.o_chi2);
      g.cand_nhits = reinterpret_cast<int32_t*>(sl + y.o_nh);
      g.cand_status = reinterpret_cast<int32_t*>(sl + y.o_st);
      g.best_state = a->best_state ? reinterpret_cast<float*>(sl + y.o_bs) : nullptr;
      g.best_cov = a->best_state ? reinterpret_cast<float*>(sl + y.o_bc) : nullptr;
      g.counters = a->counters;
      g.workspace = sc + y.build_ws;
      g.workspace_bytes = kf_build_workspace_size(cfg, Ec, Sc);
      g.stream = s_run;
      g.mlp_packed = a->mlp_packed;
      if (int32_t rc = kf_build(ctx, cfg, &g)) return rc;
      shift_hits_kernel<<<grid(L * Sc * N), 256, 0, s_run>>>(g.cand_hits, L * Sc * N, c.h0);
      KF_TRY(hipGetLastError(), "shift_hits_kernel");
    }
    KF_TRY(hipEventRecord(ev_run(k), s_run), "hipEventRecord");
    // ---- output copies into the host arrays at the chunk's seeds
    KF_TRY(hipStreamWaitEvent(s_out, ev_run(k), 0), "hipStreamWaitEvent");
    if (Sc > 0) {
      KF_TRY(hipMemcpyAsync(a->n_cands + c.s0, sl + y.o_nc, Sc * 4, d2h, s_out), "copy n_cands");
      KF_TRY(copy_rows(a->cand_hits + c.s0 * N, S * N * 4, sl + y.o_hits, Sc * N * 4, Sc * N * 4, L, d2h, s_out),
             "copy cand_hits");
      KF_TRY(hipMemcpyAsync(a->cand_chi2 + c.s0 * N, sl + y.o_chi2, Sc * N * 4, d2h, s_out), "copy cand_chi2");
      KF_TRY(hipMemcpyAsync(a->cand_nhits + c.s0 * N, sl + y.o_nh, Sc * N * 4, d2h, s_out), "copy cand_nhits");
      KF_TRY(hipMemcpyAsync(a->cand_status + c.s0 * N, sl + y.o_st, Sc * N * 4, d2h, s_out), "copy cand_status");
      if (a->best_state) {
        KF_TRY(copy_rows(a->best_state + c.s0, S * 4, sl + y.o_bs, Sc * 4, Sc * 4, 6, d2h, s_out),
               "copy best_state");
        KF_TRY(copy_rows(a->best_cov + c.s0, S * 4, sl + y.o_bc, Sc * 4, Sc * 4, 21, d2h, s_out),
               "copy best_cov");
      }
    }
    KF_TRY(hipEventRecord(ev_out(k), s_out), "hipEventRecord");
  }
  // the caller's stream continues after every copy back (the output stream runs them in chunk order)
  KF_TRY(hipStreamWaitEvent(caller, ev_out(K - 1), 0), "hipStreamWaitEvent");
#undef KF_TRY
  return KF_OK;
}

}  // extern "C"
