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

// Lane moves of the sums below, as DPP modifiers of a VALU move (no LDS traffic).  Rows
// of 16 lanes outside ROWS keep 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ float lane_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, false));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double lane_move(double v) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
  const unsigned lo = __builtin_amdgcn_update_dpp(0, int(b), CTRL, ROWS, 0xf, false);
  const unsigned hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}
__device__ __forceinline__ float lane63(float v) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63)); }
__device__ __forceinline__ double lane63(double v) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
  const unsigned lo = __builtin_amdgcn_readlane(int(b), 63), hi = __builtin_amdgcn_readlane(int(b >> 32), 63);
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// Sum over the 64 lanes of a wavefront whose lanes are all active; the result is returned
// to every lane.  Pairs and quads through quad permutes, eights and rows of 16 through the
// half-row and row mirrors; then lane 15 of rows 0 and 2 (their row sums) is added into
// rows 1 and 3, and lane 31 (rows 0 + 1) into rows 2 and 3, which leaves the total in lane
// 63.  The order of the additions is fixed, so the sum is deterministic.
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
  v += lane_move<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
  v += lane_move<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
  v += lane_move<0x141, 0xf>(v);  // row_half_mirror
  v += lane_move<0x140, 0xf>(v);  // row_mirror
  v += lane_move<0x142, 0xa>(v);  // row_bcast:15
  v += lane_move<0x143, 0xc>(v);  // row_bcast:31
  return lane63(v);
}

// Maximum over the 64 lanes of a wavefront (all active, values >= 0), the same lane moves.
__device__ __forceinline__ float wave_max(float v) {
  v = fmaxf(v, lane_move<0xb1, 0xf>(v));
  v = fmaxf(v, lane_move<0x4e, 0xf>(v));
  v = fmaxf(v, lane_move<0x141, 0xf>(v));
  v = fmaxf(v, lane_move<0x140, 0xf>(v));
  v = fmaxf(v, lane_move<0x142, 0xa>(v));
  v = fmaxf(v, lane_move<0x143, 0xc>(v));
  return lane63(v);
}

}  // namespace ri
