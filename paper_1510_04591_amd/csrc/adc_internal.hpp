// Host-side internals of the ADC library.
#pragma once
#include <vector>

#include "kernels.hpp"

enum Slot {
  SLOT_WS = 0,     // solver workspace (vectors, second eigenvector buffer, operands)
  SLOT_DESC,       // per-level descriptors
  SLOT_FLAG,       // small flags
  SLOT_QC,         // standalone Cauchy matrix
  SLOT_HSS,        // HSS workspace of the solver
  SLOT_HSS2,       // HSS work arrays of the solver (second arena)
  SLOT_BATCH,      // batched solver workspace
  SLOT_BATCH_DESC, // batched solver descriptors
  SLOT_MLP,        // MLP scratch
  NSLOT
};

struct MlpState;

struct adc_ctx_s {
  struct Buf {
    void* ptr = nullptr;
    size_t bytes = 0;
  };
  int device = 0;
  hipStream_t stream = nullptr;
  Buf bufs[NSLOT];
  void* host_stage = nullptr;
  size_t host_stage_bytes = 0;
  MlpState* mlp = nullptr;
  void* batch_cache = nullptr;  // graph cache of the batched solver
  adc_status buffer(int slot, size_t bytes, void** p);
  adc_status stage(size_t bytes, void** p);
  void release();
};

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
  }
};

// bump allocator over one device region
struct Arena {
  char* base = nullptr;
  size_t off = 0;
  size_t cap = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += count * sizeof(T);
    return p;
  }
};

adc_status check_finite(adc_ctx c, const double* x, int64_t n, bool* ok);
int pick_waves(int64_t K);
void mlp_release(adc_ctx c);

__global__ void k_check_finite(const double* __restrict__ x, int64_t n, int* __restrict__ flag);
__global__ void k_set_int(int* p, int v);
__global__ void k_tear(const double* __restrict__ diag, const double* __restrict__ off,
                       const int64_t* __restrict__ splits, int nsplit, double* __restrict__ a, int64_t n);
adc_status validate_opts_ext(const adc_opts& o);
