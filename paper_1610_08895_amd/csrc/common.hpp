// Internal helpers shared by the library's translation units: error reporting,
// HIP call checking and small device utilities.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "ri.h"

namespace ri {

// Thread-local last-error message, returned by ri_last_error().
void set_error_msg(const char* fmt, ...);
const char* error_msg();

inline int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  set_error_msg("%s", buf);
  return code;
}

#define RI_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return ::ri::fail(RI_EHIP, "%s:%d %s: %s", __FILE__, __LINE__, #call,           \
                        hipGetErrorString(e_));                                       \
  } while (0)

#define RI_LAUNCH_CHECK() RI_HIP(hipGetLastError())

#define RI_TRY(expr)              \
  do {                            \
    int rc_ = (expr);             \
    if (rc_ != RI_OK) return rc_; \
  } while (0)

// Device allocation that reports RI_ENOMEM.
template <class T>
int dev_alloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) return RI_OK;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(RI_ENOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T),
                hipGetErrorString(e));
  }
  return RI_OK;
}

template <class T>
void dev_free(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

inline bool is_pow2(long long v) { return v > 0 && (v & (v - 1)) == 0; }
inline int ilog2(long long v) {
  int r = 0;
  while ((1LL << r) < v) ++r;
  return r;
}

// Number of compute units of the current device (cached per process).
int device_cus();

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// Wavefront-level FP64 sum (64 lanes), result valid in every lane.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace ri
