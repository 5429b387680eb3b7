// kf_internal.hpp -- host-side context and helpers shared by the library's
// translation units (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "../../include/kfmi.h"
#include "kf_device.hpp"

// digest of the kernel sources this library was built from (set by the build); keys the autotune cache
#ifndef KF_SOURCE_DIGEST
#define KF_SOURCE_DIGEST "unknown"
#endif

// one autotuned build launch configuration
struct kf_tuned {
  int32_t mode = 0, waves_per_block = 0, blocks_per_cu = 0;
  float ms = 0.f;
};

struct kf_ctx {
  int device = 0;
  bool has_geometry = false;
  kf_geometry geom{};
  kfd::Geom dgeom{};
  int num_cus = 0;
  char arch[64] = {0};                    // gcnArchName of the device (keys the autotune cache)
  std::map<std::string, kf_tuned> tuned;  // autotune cache, key from kf_build_autotune
  std::map<std::string, kf_tuned> fit_tuned;  // fit launches: waves_per_block holds the block size in waves
  void* scratch = nullptr;                    // device address of this device's static build scratch
  size_t scratch_bytes = 0;
  hipStream_t pipe[4] = {nullptr, nullptr, nullptr, nullptr};  // kf_build_host: input copies, output copies, and
                                                               // two kernel streams
  std::vector<hipEvent_t> pipe_events;                 // kf_build_host: start, then three per chunk
};

namespace kfh {

int32_t set_error(int32_t code, const char* fmt, ...);

inline int32_t check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) return set_error(KF_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
  return KF_OK;
}

// Make ctx's device current for this host thread.
int32_t enter(kf_ctx* ctx);

inline hipStream_t stream_of(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Creates kf_build_host's four streams (once) and at least n_events timing-free events in ctx.
int32_t pipe_streams(kf_ctx* ctx, int n_events);

// Releases the streams and events a context created.
void ctx_release(kf_ctx* ctx);

// Looks up the device address of the static build scratch on ctx's (current) device.
int32_t scratch_init(kf_ctx* ctx);

// Cache key of a tuned fit launch (device architecture, source digest, precision flag, bucket of the track count).
std::string fit_tune_key(const kf_ctx* ctx, uint32_t flags, int64_t n);

inline unsigned grid_for(int64_t n, int block) { return static_cast<unsigned>((n + block - 1) / block); }

}  // namespace kfh
