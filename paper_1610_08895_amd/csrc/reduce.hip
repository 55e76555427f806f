// Fill kernels and FP64 wavefront-reduction l2 norms (power iterations, diagnostics).
// The sum of squares is deterministic: fixed-size per-workgroup partials, then one
// workgroup sums them in a fixed order.
#include "plan.hpp"

namespace ri {

namespace {

constexpr int RT = 256;
constexpr int RPART = SUMSQ_SCRATCH - 1;  // partial sums (first pass workgroups)

__global__ void k_zero_f32(float* __restrict__ p, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    p[i] = 0.f;
}

__global__ __launch_bounds__(RT) void k_sumsq_part(const float* __restrict__ x, size_t n, double* __restrict__ part) {
  __shared__ double red[RT / 64];
  double acc = 0.0;
  for (size_t i = blockIdx.x * size_t(RT) + threadIdx.x; i < n; i += size_t(gridDim.x) * RT) {
    const double v = x[i];
    acc += v * v;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < RT / 64; ++k) t += red[k];
    part[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(RT) void k_sum_parts(const double* __restrict__ part, int np, double* __restrict__ out) {
  __shared__ double red[RT / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += RT) acc += part[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < RT / 64; ++k) t += red[k];
    *out = t;
  }
}

__global__ void k_scale_rsqrt(float* __restrict__ x, size_t n, const double* __restrict__ sq) {
  const double s = *sq;
  const float f = s > 0.0 ? float(1.0 / sqrt(s)) : 0.f;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    x[i] *= f;
}

unsigned blocks_for(size_t n) {
  const size_t b = (n + RT - 1) / RT;
  return unsigned(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

int zero_f32(float* p, size_t n, hipStream_t s) {
  if (n == 0) return RI_OK;
  hipLaunchKernelGGL(k_zero_f32, dim3(blocks_for(n)), dim3(RT), 0, s, p, n);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

int zero_c64(float2* p, size_t n, hipStream_t s) { return zero_f32(reinterpret_cast<float*>(p), 2 * n, s); }

// out points at SUMSQ_SCRATCH doubles: the result goes to out[0], the partials to out[1..].
int sumsq_f32(const float* x, size_t n, double* out, hipStream_t s) {
  double* part = out + 1;
  hipLaunchKernelGGL(k_sumsq_part, dim3(RPART), dim3(RT), 0, s, x, n, part);
  RI_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(RT), 0, s, part, RPART, out);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

int scale_by_rsqrt(float* x, size_t n, const double* sq, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_rsqrt, dim3(blocks_for(n)), dim3(RT), 0, s, x, n, sq);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

}  // namespace ri
