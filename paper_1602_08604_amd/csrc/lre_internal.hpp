// lre_internal.hpp -- host-side pieces shared by the translation units of liblre.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

struct lre_ctx {
  int device;
  uint32_t* flags;              // device word: FLAG_* bits raised by the kernels
  hipEvent_t stage_events[4];   // optional profiling events (lre_set_stage_events)
  int n_stage_events;
  void* blas = nullptr;         // rocBLAS handle of lre_project, created on first use
  char* scratch = nullptr;      // this device's address of the static scratch array
                                // (lre_estimate_noalloc), resolved by lre_create
  int scratch_status = 0;       // hipError_t of that lookup
};

namespace lre_detail {

// Releases the rocBLAS handle of a context (lre_project.hip).
void destroy_blas(void* handle);

inline void record_stage(lre_ctx* ctx, int k, hipStream_t st) {
  if (k < ctx->n_stage_events && ctx->stage_events[k]) (void)hipEventRecord(ctx->stage_events[k], st);
}

// Makes `dev` current for the guard's lifetime.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

inline bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

}  // namespace lre_detail
