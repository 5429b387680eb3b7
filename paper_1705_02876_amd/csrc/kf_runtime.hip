// kf_runtime.cpp -- host runtime around the kernels: HIP graph capture of
// whole call sequences and the build-launch autotuner with its file cache.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "kf_internal.hpp"

using kfh::set_error;

struct kf_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = 0;
};

namespace {

// Cache key of a tuned build launch: device architecture, the digest of the kernel sources, and the problem's
// class (candidates, precision, window, power-of-two bucket of the seed count, bin grid).  Entries taken on
// another device or with other kernels never match.
std::string tune_key(const kf_ctx* ctx, const kf_build_cfg* cfg, int64_t n_seeds) {
  int bucket = 0;
  while ((int64_t(1) << (bucket + 1)) <= n_seeds && bucket < 62) ++bucket;
  char buf[160];
  std::snprintf(buf, sizeof buf, "%s_%s_N%d_p%d_w%d_s2^%d_phi%d_eta%d", ctx->arch, KF_SOURCE_DIGEST, cfg->max_cands,
                cfg->precision, cfg->window_mode, bucket, cfg->n_phi, cfg->n_eta);
  return buf;
}

}  // namespace

int32_t kfh::pipe_streams(kf_ctx* ctx, int n_events) {
  for (int i = 0; i < 4; ++i)
    if (!ctx->pipe[i])  // default priority, not synchronising with the null stream
      if (int32_t rc = check_hip(hipStreamCreateWithFlags(&ctx->pipe[i], hipStreamNonBlocking), "hipStreamCreate"))
        return rc;
  while (static_cast<int>(ctx->pipe_events.size()) < n_events) {
    hipEvent_t e = nullptr;
    if (int32_t rc = check_hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate")) return rc;
    ctx->pipe_events.push_back(e);
  }
  return KF_OK;
}

void kfh::ctx_release(kf_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  for (int i = 0; i < 4; ++i)
    if (ctx->pipe[i]) {
      (void)hipStreamSynchronize(ctx->pipe[i]);
      (void)hipStreamDestroy(ctx->pipe[i]);
      ctx->pipe[i] = nullptr;
    }
  for (hipEvent_t e : ctx->pipe_events) (void)hipEventDestroy(e);
  ctx->pipe_events.clear();
}

std::string kfh::fit_tune_key(const kf_ctx* ctx, uint32_t flags, int64_t n) {
  int bucket = 0;
  while ((int64_t(1) << (bucket + 1)) <= n && bucket < 62) ++bucket;
  char buf[160];
  std::snprintf(buf, sizeof buf, "%s_%s_fit_f%u_n2^%d", ctx->arch, KF_SOURCE_DIGEST,
                static_cast<unsigned>(flags & (KF_FIT_FP64 | KF_FIT_EMIT_RESIDUALS)), bucket);
  return buf;
}

extern "C" {

int32_t kf_graph_begin(kf_ctx* ctx, void* stream) {
  if (int32_t rc = kfh::enter(ctx)) return rc;
  if (!stream) return set_error(KF_ERR_INVALID_ARG, "graph capture needs a created (non-default) stream");
  return kfh::check_hip(hipStreamBeginCapture(kfh::stream_of(stream), hipStreamCaptureModeThreadLocal),
                        "hipStreamBeginCapture");
}

int32_t kf_graph_end(kf_ctx* ctx, void* stream, kf_graph** out) {
  if (int32_t rc = kfh::enter(ctx)) return rc;
  if (!stream || !out) return set_error(KF_ERR_INVALID_ARG, "null stream or output");
  *out = nullptr;
  hipGraph_t g = nullptr;
  if (int32_t rc = kfh::check_hip(hipStreamEndCapture(kfh::stream_of(stream), &g), "hipStreamEndCapture")) return rc;
  hipGraphExec_t ex = nullptr;
  if (int32_t rc = kfh::check_hip(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "hipGraphInstantiate")) {
    (void)hipGraphDestroy(g);
    return rc;
  }
  kf_graph* k = new kf_graph();
  k->graph = g;
  k->exec = ex;
  k->device = ctx->device;
  *out = k;
  return KF_OK;
}

int32_t kf_graph_launch(kf_graph* g, void* stream) {
  if (!g || !g->exec) return set_error(KF_ERR_INVALID_ARG, "null graph");
  if (int32_t rc = kfh::check_hip(hipSetDevice(g->device), "hipSetDevice")) return rc;
  return kfh::check_hip(hipGraphLaunch(g->exec, kfh::stream_of(stream)), "hipGraphLaunch");
}

void kf_graph_destroy(kf_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

int32_t kf_build_autotune(kf_ctx* ctx, kf_build_cfg* cfg, const kf_build_args* args, int32_t reps, float* best_ms) {
  if (int32_t rc = kfh::enter(ctx)) return rc;
  if (!cfg || !args) return set_error(KF_ERR_INVALID_ARG, "null argument");
  if (reps < 1 || reps > 1000) return set_error(KF_ERR_INVALID_ARG, "reps must be 1..1000");
  const std::string key = tune_key(ctx, cfg, args->n_seeds);
  auto it = ctx->tuned.find(key);
  if (it != ctx->tuned.end()) {
    cfg->mode = it->second.mode;
    cfg->waves_per_block = it->second.waves_per_block;
    cfg->blocks_per_cu = it->second.blocks_per_cu;
    if (best_ms) *best_ms = it->second.ms;
    return KF_OK;
  }
  if (args->n_seeds == 0) return KF_OK;
  kf_build_args a = *args;
  a.counters = nullptr;  // tuning runs do not count work
  hipStream_t s = kfh::stream_of(a.stream);
  hipEvent_t e0, e1;
  if (int32_t rc = kfh::check_hip(hipEventCreate(&e0), "hipEventCreate")) return rc;
  if (int32_t rc = kfh::check_hip(hipEventCreate(&e1), "hipEventCreate")) {
    (void)hipEventDestroy(e0);
    return rc;
  }
  kf_tuned best;
  best.ms = INFINITY;
  kf_build_cfg pc = *cfg;
  pc.mode = KF_BUILD_PERSISTENT;
  const bool can_persist = a.workspace && a.workspace_bytes >= kf_build_workspace_size(&pc, a.n_events, a.n_seeds);
  kf_build_cfg sc = *cfg;
  sc.mode = KF_BUILD_SERIAL;
  const bool can_serial = cfg->window_mode == KF_WINDOW_PLAIN && cfg->precision == KF_PREC_F32 && a.workspace &&
                          a.workspace_bytes >= kf_build_workspace_size(&sc, a.n_events, a.n_seeds);
  const int wpbs[3] = {1, 2, 4};
  const int bpcs[7] = {1, 2, 3, 4, 8, 12, 14};  // 12 and 14 one-wave blocks fill a CU as the tiled launch does
  int32_t rc = KF_OK;
  for (int mode = KF_BUILD_TILED; mode <= KF_BUILD_SERIAL && rc == KF_OK; ++mode) {
    if (mode == KF_BUILD_PERSISTENT && !can_persist) continue;
    if (mode == KF_BUILD_SERIAL && !can_serial) continue;
    for (int wi = 0; wi < 3 && rc == KF_OK; ++wi)
      for (int bi = 0; bi < (mode == KF_BUILD_PERSISTENT ? 7 : 1) && rc == KF_OK; ++bi) {
        kf_build_cfg c = *cfg;
        c.mode = mode;
        c.waves_per_block = wpbs[wi];
        c.blocks_per_cu = bpcs[bi];
        if ((rc = kf_build(ctx, &c, &a)) != KF_OK) break;  // warm-up and validation
        if ((rc = kfh::check_hip(hipEventRecord(e0, s), "hipEventRecord")) != KF_OK) break;
        for (int r = 0; r < reps && rc == KF_OK; ++r) rc = kf_build(ctx, &c, &a);
        if (rc != KF_OK) break;
        if ((rc = kfh::check_hip(hipEventRecord(e1, s), "hipEventRecord")) != KF_OK) break;
        if ((rc = kfh::check_hip(hipEventSynchronize(e1), "hipEventSynchronize")) != KF_OK) break;
        float ms = 0.f;
        if ((rc = kfh::check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime")) != KF_OK) break;
        ms /= static_cast<float>(reps);
        if (ms < best.ms) {
          best.mode = c.mode;
          best.waves_per_block = c.waves_per_block;
          best.blocks_per_cu = c.blocks_per_cu;
          best.ms = ms;
        }
      }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != KF_OK) return rc;
  ctx->tuned[key] = best;
  cfg->mode = best.mode;
  cfg->waves_per_block = best.waves_per_block;
  cfg->blocks_per_cu = best.blocks_per_cu;
  if (best_ms) *best_ms = best.ms;
  return KF_OK;
}

int32_t kf_fit_autotune(kf_ctx* ctx, const kf_fit_args* args, int32_t reps, int32_t* best_block, float* best_ms) {
  if (int32_t rc = kfh::enter(ctx)) return rc;
  if (!args) return set_error(KF_ERR_INVALID_ARG, "null argument");
  if (reps < 1 || reps > 1000) return set_error(KF_ERR_INVALID_ARG, "reps must be 1..1000");
  const std::string key = kfh::fit_tune_key(ctx, args->flags, args->n);
  auto it = ctx->fit_tuned.find(key);
  if (it != ctx->fit_tuned.end()) {
    if (best_block) *best_block = 64 * it->second.waves_per_block;
    if (best_ms) *best_ms = it->second.ms;
    return KF_OK;
  }
  if (args->n == 0) {
    if (best_block) *best_block = 256;
    if (best_ms) *best_ms = 0.f;
    return KF_OK;
  }
  hipStream_t s = kfh::stream_of(args->stream);
  hipEvent_t e0, e1;
  if (int32_t rc = kfh::check_hip(hipEventCreate(&e0), "hipEventCreate")) return rc;
  if (int32_t rc = kfh::check_hip(hipEventCreate(&e1), "hipEventCreate")) {
    (void)hipEventDestroy(e0);
    return rc;
  }
  kf_tuned best;
  best.ms = INFINITY;
  int32_t rc = KF_OK;
  const int waves[3] = {1, 2, 4};  // 64, 128, 256 threads (the kernels' launch bound is 256)
  for (int wi = 0; wi < 3 && rc == KF_OK; ++wi) {
    kf_tuned t;
    t.waves_per_block = waves[wi];
    ctx->fit_tuned[key] = t;  // kf_fit launches with the candidate block size while it is timed
    if ((rc = kf_fit(ctx, args)) != KF_OK) break;  // warm-up and validation
    if ((rc = kfh::check_hip(hipEventRecord(e0, s), "hipEventRecord")) != KF_OK) break;
    for (int r = 0; r < reps && rc == KF_OK; ++r) rc = kf_fit(ctx, args);
    if (rc != KF_OK) break;
    if ((rc = kfh::check_hip(hipEventRecord(e1, s), "hipEventRecord")) != KF_OK) break;
    if ((rc = kfh::check_hip(hipEventSynchronize(e1), "hipEventSynchronize")) != KF_OK) break;
    float ms = 0.f;
    if ((rc = kfh::check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime")) != KF_OK) break;
    ms /= static_cast<float>(reps);
    if (ms < best.ms) {
      best.waves_per_block = waves[wi];
      best.ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != KF_OK) {
    ctx->fit_tuned.erase(key);
    return rc;
  }
  ctx->fit_tuned[key] = best;
  if (best_block) *best_block = 64 * best.waves_per_block;
  if (best_ms) *best_ms = best.ms;
  return KF_OK;
}

int32_t kf_autotune_save(kf_ctx* ctx, const char* path) {
  if (!ctx || !path) return set_error(KF_ERR_INVALID_ARG, "null argument");
  std::FILE* f = std::fopen(path, "w");
  if (!f) return set_error(KF_ERR_INVALID_ARG, "cannot write %s", path);
  for (const auto& kv : ctx->tuned)
    std::fprintf(f, "{\"key\": \"%s\", \"mode\": %d, \"waves_per_block\": %d, \"blocks_per_cu\": %d, \"ms\": %.6g}\n",
                 kv.first.c_str(), kv.second.mode, kv.second.waves_per_block, kv.second.blocks_per_cu,
                 static_cast<double>(kv.second.ms));
  for (const auto& kv : ctx->fit_tuned)
    std::fprintf(f, "{\"key\": \"%s\", \"fit_block\": %d, \"ms\": %.6g}\n", kv.first.c_str(),
                 64 * kv.second.waves_per_block, static_cast<double>(kv.second.ms));
  const bool ok = std::fclose(f) == 0;
  return ok ? KF_OK : set_error(KF_ERR_INVALID_ARG, "error writing %s", path);
}

int32_t kf_autotune_load(kf_ctx* ctx, const char* path) {
  if (!ctx || !path) return set_error(KF_ERR_INVALID_ARG, "null argument");
  std::FILE* f = std::fopen(path, "r");
  if (!f) return set_error(KF_ERR_INVALID_ARG, "cannot read %s", path);
  char line[512];
  int32_t rc = KF_OK;
  while (std::fgets(line, sizeof line, f)) {
    char key[161];
    kf_tuned t;
    double ms = 0.0;
    int block = 0;
    if (std::sscanf(line, " {\"key\": \"%160[^\"]\", \"fit_block\": %d, \"ms\": %lf", key, &block, &ms) == 3) {
      if (block != 64 && block != 128 && block != 256) {
        rc = set_error(KF_ERR_INVALID_ARG, "malformed fit autotune entry in %s", path);
        break;
      }
      t.waves_per_block = block / 64;
      t.ms = static_cast<float>(ms);
      ctx->fit_tuned[key] = t;
      continue;
    }
    if (std::sscanf(line, " {\"key\": \"%160[^\"]\", \"mode\": %d, \"waves_per_block\": %d, \"blocks_per_cu\": %d, \"ms\": %lf",
                    key, &t.mode, &t.waves_per_block, &t.blocks_per_cu, &ms) != 5 ||
        (t.mode != KF_BUILD_TILED && t.mode != KF_BUILD_PERSISTENT && t.mode != KF_BUILD_SERIAL) ||
        t.waves_per_block < 1 ||
        t.waves_per_block > 4 || t.blocks_per_cu < 0 || t.blocks_per_cu > 64) {
      rc = set_error(KF_ERR_INVALID_ARG, "malformed autotune entry in %s", path);
      break;
    }
    t.ms = static_cast<float>(ms);
    ctx->tuned[key] = t;
  }
  std::fclose(f);
  return rc;
}

}  // extern "C"
