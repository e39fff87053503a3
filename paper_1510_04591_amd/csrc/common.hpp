// Shared device/host definitions of the gfx950 ADC library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include "adc.h"

#define ADC_EPS 2.220446049250313e-16

typedef double dbl4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- host side
#define HIP_OK(expr)                                  \
  do {                                                \
    hipError_t _e = (expr);                           \
    if (_e != hipSuccess) return ADC_ERR_HIP;         \
  } while (0)

#define ADC_TRY(expr)                                 \
  do {                                                \
    adc_status _s = (expr);                           \
    if (_s != ADC_OK) return _s;                      \
  } while (0)

// ---------------------------------------------------------------- device side

// d_i - lam_j by the accurate differences of Remark 1 (eq. d-lambda):
//   (d_i - d_j) - gam_j       for i <= j
//   (d_i - d_{j+1}) + mu_j    for i >  j
// dj1 is d_{j+1} (unused when i <= j).
__device__ __forceinline__ double d_minus_lam(int i, int j, double di, double dj, double dj1,
                                              double gj, double mj) {
  return (i <= j) ? ((di - dj) - gj) : ((di - dj1) + mj);
}

// Global-memory views of pointers: loads and stores through them compile to
// global instructions.  Through a generic pointer (one read from a structure,
// say) they are generic (flat) instructions, which also count as LDS
// operations, so that every wait for an LDS read would also wait for all
// global loads in flight.
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) const double gcdouble;
typedef __attribute__((address_space(1))) const int32_t gcint;
__device__ __forceinline__ gdouble* gmem(double* p) { return (gdouble*)p; }
__device__ __forceinline__ gcdouble* gmem(const double* p) { return (gcdouble*)p; }
__device__ __forceinline__ gcint* gmem(const int32_t* p) { return (gcint*)p; }

// The index of the calling wave in its workgroup, as a wave-uniform value:
// loop bounds derived from it stay in scalar registers, so that operands
// indexed by them are read with scalar loads (threadIdx.x >> 6 alone is
// taken as divergent by the compiler).
__device__ __forceinline__ int wave_index() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

__device__ __forceinline__ double wave_sum(double x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

__device__ __forceinline__ double wave_max(double x) {
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
  return x;
}

__device__ __forceinline__ int wave_sum_i(int x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}
