// Block selection on the device: step 3 of Algorithm 1 (block i is active with
// probability p_i, independently, Sec. III-B) and the adaptive probabilities of Sec. IV
// (Eq. 13 energies c_i, Eq. 14 water-filling), so that an iteration replayed from a
// captured graph draws its own active set and no host round trip separates two steps.
//
// One workgroup does everything: d is at most a few thousand, and Eq. 14 needs global
// sums over all blocks.  Sums are formed in a fixed order (a strided per-thread loop,
// the wavefront sum of common.hpp, then the wavefront partials in order), so results are
// reproducible run to run.  Eq. 14 is solved by successive saturation, the method of the
// host entry point ri_probs: from a = 0, saturate every unsaturated block with
// w_i + a > p_max - p_min and recompute a so the unsaturated blocks absorb the remaining
// mass evenly; a never decreases, so at most d rounds are needed.
#include "common.hpp"

namespace ri {
namespace {

constexpr int ST = 256;  // threads of the selection workgroup
constexpr int SW = ST / 64;
constexpr int SCHED_MAX_D = 4096;

__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < SW; ++k) s += red[k];
  return s;
}

__device__ __forceinline__ double energy(double sq, double eps) {
  const double over = sqrt(sq) - eps;  // Eq. 13 from the squared residual norm
  return over > 0.0 ? (over * over) / (eps * eps) : 0.0;
}

__global__ __launch_bounds__(ST) void k_schedule(ri_sched a, int flags) {
  __shared__ double w[SCHED_MAX_D];
  __shared__ unsigned char sat[SCHED_MAX_D];
  __shared__ double red[SW];
  const int d = a.d;
  const int64_t t = *a.counter;
  if ((flags & RI_SCHED_UPDATE) && t > 0)
    for (int i = threadIdx.x; i < d; i += ST)
      if (a.mask[i]) a.c[i] = energy(a.stats_step[2 * i + 1], a.eps[i]);
  if (flags & RI_SCHED_REFRESH)
    for (int i = threadIdx.x; i < d; i += ST) a.c[i] = energy(a.stats_x[2 * i + 1], a.eps[i]);
  if (!(flags & RI_SCHED_DRAW)) return;

  // probabilities p_i into w[]
  if (flags & RI_SCHED_ADAPTIVE) {
    double part = 0.0;
    for (int i = threadIdx.x; i < d; i += ST) part += a.c[i];
    const double total = block_sum(part, red);
    if (total == 0.0) {
      for (int i = threadIdx.x; i < d; i += ST) w[i] = a.n_nodes / d;
    } else {
      const double R = a.n_nodes - d * a.p_min, cap = a.p_max - a.p_min;
      for (int i = threadIdx.x; i < d; i += ST) {
        w[i] = R * a.c[i] / total;
        sat[i] = 0;
      }
      __syncthreads();
      double aa = 0.0;
      for (int round = 0; round <= d; ++round) {
        double grew = 0.0;
        for (int i = threadIdx.x; i < d; i += ST)
          if (!sat[i] && w[i] + aa > cap) {
            sat[i] = 1;
            grew = 1.0;
          }
        if (block_sum(grew, red) == 0.0) break;
        double nf = 0.0, fm = 0.0;
        for (int i = threadIdx.x; i < d; i += ST)
          if (!sat[i]) {
            nf += 1.0;
            fm += w[i];
          }
        const double nfree = block_sum(nf, red);
        const double free_mass = block_sum(fm, red);
        if (nfree == 0.0) {
          aa = cap;
          break;
        }
        aa = (R - (d - nfree) * cap - free_mass) / nfree;
        if (aa < 0.0) aa = 0.0;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < d; i += ST) w[i] = a.p_min + (w[i] + aa < cap ? w[i] + aa : cap);
    }
  } else {
    for (int i = threadIdx.x; i < d; i += ST) w[i] = a.p_fixed != nullptr ? a.p_fixed[i] : 1.0;
  }
  __syncthreads();

  // step 3: the active set of iteration t from row t mod T
  const int64_t row = t % a.T;
  for (int i = threadIdx.x; i < d; i += ST) {
    const size_t k = size_t(row) * d + i;
    const uint8_t m = a.masks != nullptr ? a.masks[k] : uint8_t(a.u[k] < w[i]);
    a.mask[i] = m;
    if (a.p_log != nullptr) a.p_log[k] = w[i];
    if (a.mask_log != nullptr) a.mask_log[k] = m;
  }
  __syncthreads();  // every thread has read the counter
  if (threadIdx.x == 0) *a.counter = t + 1;
}

}  // namespace
}  // namespace ri

using ri::fail;

extern "C" int ri_sched_step(const ri_sched* a, int flags, hipStream_t stream) {
  if (!a) return fail(RI_EINVAL, "ri_sched is NULL");
  if (a->d < 1 || a->d > ri::SCHED_MAX_D) return fail(RI_EINVAL, "d = %d outside [1, %d]", a->d, ri::SCHED_MAX_D);
  if (flags & ~(RI_SCHED_UPDATE | RI_SCHED_REFRESH | RI_SCHED_ADAPTIVE | RI_SCHED_DRAW))
    return fail(RI_EINVAL, "unknown flags 0x%x", flags);
  if (!a->counter || !a->mask) return fail(RI_EINVAL, "counter and mask are required");
  const bool adaptive = flags & RI_SCHED_ADAPTIVE, update = flags & RI_SCHED_UPDATE,
             refresh = flags & RI_SCHED_REFRESH, draw = flags & RI_SCHED_DRAW;
  if ((adaptive || update || refresh) && !a->c) return fail(RI_EINVAL, "c is required");
  if ((update || refresh) && !a->eps) return fail(RI_EINVAL, "eps is required");
  if (update && !a->stats_step) return fail(RI_EINVAL, "stats_step is required");
  if (refresh && !a->stats_x) return fail(RI_EINVAL, "stats_x is required");
  if (draw) {
    if (a->T < 1) return fail(RI_EINVAL, "T must be >= 1");
    if (!a->masks && !a->u) return fail(RI_EINVAL, "u or masks is required to draw");
  }
  if (adaptive) {
    const double nd = a->n_nodes / a->d;
    if (!(a->p_min > 0 && a->p_min <= nd && nd <= a->p_max && a->p_max <= 1.0))
      return fail(RI_EINVAL, "need 0 < p_min <= n/d <= p_max <= 1 (p_min %g, n/d %g, p_max %g)", a->p_min, nd,
                  a->p_max);
  }
  hipLaunchKernelGGL(ri::k_schedule, dim3(1), dim3(ri::ST), 0, stream, *a, flags);
  RI_LAUNCH_CHECK();
  return RI_OK;
}
