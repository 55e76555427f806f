// Kernels of the reverse (vector-Jacobian) sweep of one Algorithm 1 iteration with the
// active set fixed.  Complex values are pairs of reals and every inner product is real.
//
// Steps 17-18, x' = max(z, 0) with z = x - tau (sigma s~ + varsigma g), x~' = 2 x' - x:
//   zbar = (xbar' + 2 xtbar') [x' > 0],  xbar = zbar - xtbar',
//   dL/dtau -= <zbar, sigma s~ + varsigma g>,  dL/dsigma -= tau <zbar, s~>.
// Step 13, s' = clip(a, -alpha, alpha), a = s + Psi^dagger x~ (the clip is min/max, so
// |s'| < alpha exactly where |a| < alpha):  abar = (sbar' - tau sigma Psi^dagger zbar)[|s'| < alpha].
// Step 8, v_i' = r_i max(0, 1 - eps_i / ||r_i||), r_i = v_i + G_i b_i - y_i, for active
// blocks, with u_i = vbar_i' - tau varsigma (Phi zbar)_i:
//   rbar_i = (1 - eps_i/||r_i||) u_i + eps_i r_i (r_i^T u_i) / ||r_i||^3 if ||r_i|| > eps_i, else 0;
// inactive blocks keep v_i, so their vbar_i = u_i.  FP64 reductions run in a fixed order.
#include "vjp.hpp"

namespace ri {

namespace {

constexpr int VT = 256;          // threads per workgroup
constexpr int BALL_CHUNK = 4096;  // visibilities per workgroup of the per-block passes

__global__ __launch_bounds__(VT) void k_vjp_primal(int n, const float* __restrict__ x_new,
                                                   float* __restrict__ xbar, const float* __restrict__ xtbar,
                                                   float* __restrict__ zbar) {
  for (int k = blockIdx.x * VT + threadIdx.x; k < n; k += gridDim.x * VT) {
    const float xt = xtbar[k];
    const float z = x_new[k] > 0.f ? xbar[k] + 2.f * xt : 0.f;
    zbar[k] = z;
    xbar[k] = z - xt;
  }
}

// part[2 b], part[2 b + 1]: this workgroup's <zbar, sigma st + varsigma g> and <zbar, st>
__global__ __launch_bounds__(VT) void k_dot2(int n, const float* __restrict__ zbar, const float* __restrict__ st,
                                             const float* __restrict__ g, double sigma, double varsigma,
                                             double* __restrict__ part) {
  __shared__ double red[2][VT / 64];
  double a = 0.0, b = 0.0;
  for (int k = blockIdx.x * VT + threadIdx.x; k < n; k += gridDim.x * VT) {
    const double z = zbar[k], s = st[k];
    a += z * (sigma * s + varsigma * double(g[k]));
    b += z * s;
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x / 64] = a;
    red[1][threadIdx.x / 64] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int w = 0; w < VT / 64; ++w) {
      s0 += red[0][w];
      s1 += red[1][w];
    }
    part[2 * blockIdx.x] = s0;
    part[2 * blockIdx.x + 1] = s1;
  }
}

__global__ void k_dot2_final(const double* __restrict__ part, int nparts, double tau, double* __restrict__ pgrad) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int b = 0; b < nparts; ++b) {
      s0 += part[2 * b];
      s1 += part[2 * b + 1];
    }
    pgrad[0] -= s0;
    pgrad[1] -= tau * s1;
  }
}

__global__ __launch_bounds__(VT) void k_vjp_clip(size_t count, const float* __restrict__ s_new, float alpha,
                                                 const float* __restrict__ wts, const float* __restrict__ w, float c,
                                                 float* __restrict__ sbar) {
  for (size_t k = size_t(blockIdx.x) * VT + threadIdx.x; k < count; k += size_t(gridDim.x) * VT) {
    const float bound = wts != nullptr ? alpha * wts[k] : alpha;  // the forward clip's bound
    sbar[k] = fabsf(s_new[k]) < bound ? sbar[k] + c * w[k] : 0.f;
  }
}

__global__ __launch_bounds__(VT) void k_axpy(int n, float a, const float* __restrict__ x, float* __restrict__ y) {
  for (int k = blockIdx.x * VT + threadIdx.x; k < n; k += gridDim.x * VT) y[k] += a * x[k];
}

// part[i * nch + ch] = sum over chunk ch of block i of r^T u, u = vbar + c phiz
__global__ __launch_bounds__(VT) void k_ball_dot(const int64_t* __restrict__ off, const uint8_t* __restrict__ mask,
                                                 const float2* __restrict__ vbar, const float2* __restrict__ phiz,
                                                 float c, const float2* __restrict__ r, int nch,
                                                 double* __restrict__ part) {
  __shared__ double red[VT / 64];
  const int i = blockIdx.y, ch = blockIdx.x;
  if (mask[i] == 0) return;
  const int64_t lo = off[i] + int64_t(ch) * BALL_CHUNK, hi = min(off[i + 1], lo + BALL_CHUNK);
  double acc = 0.0;
  for (int64_t m = lo + threadIdx.x; m < hi; m += VT) {
    const float2 vb = vbar[m], pz = phiz[m], rr = r[m];
    const double ux = double(vb.x) + double(c) * pz.x, uy = double(vb.y) + double(c) * pz.y;
    acc += double(rr.x) * ux + double(rr.y) * uy;
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < VT / 64; ++w) s += red[w];
    part[size_t(i) * nch + ch] = s;
  }
}

// per block: coef[2i] (weight of u), coef[2i+1] (weight of r)
__global__ void k_ball_coef(int d, const int64_t* __restrict__ off, const uint8_t* __restrict__ mask,
                            const double* __restrict__ stats, const double* __restrict__ eps,
                            const double* __restrict__ part, int nch, double* __restrict__ coef) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d; i += gridDim.x * blockDim.x) {
    if (mask[i] == 0) {
      coef[2 * i] = 1.0;
      coef[2 * i + 1] = 0.0;
      continue;
    }
    const double nr = sqrt(stats[2 * i]), ep = eps[i];
    if (!(nr > ep)) {
      coef[2 * i] = 0.0;
      coef[2 * i + 1] = 0.0;
      continue;
    }
    const int nc = int((off[i + 1] - off[i] + BALL_CHUNK - 1) / BALL_CHUNK);
    double ru = 0.0;
    for (int ch = 0; ch < nc; ++ch) ru += part[size_t(i) * nch + ch];
    coef[2 * i] = 1.0 - ep / nr;
    coef[2 * i + 1] = ep * ru / (nr * nr * nr);
  }
}

__global__ __launch_bounds__(VT) void k_ball_apply(const int64_t* __restrict__ off, const uint8_t* __restrict__ mask,
                                                   float2* __restrict__ vbar, const float2* __restrict__ phiz, float c,
                                                   const float2* __restrict__ r, const double* __restrict__ coef) {
  const int i = blockIdx.y, ch = blockIdx.x;
  const int64_t lo = off[i] + int64_t(ch) * BALL_CHUNK, hi = min(off[i + 1], lo + BALL_CHUNK);
  const float a = float(coef[2 * i]), b = float(coef[2 * i + 1]);
  const bool active = mask[i] != 0;
  for (int64_t m = lo + threadIdx.x; m < hi; m += VT) {
    const float2 vb = vbar[m], pz = phiz[m];
    const float2 u = make_float2(vb.x + c * pz.x, vb.y + c * pz.y);
    float2 out = make_float2(a * u.x, a * u.y);
    if (active) {
      const float2 rr = r[m];
      out.x += b * rr.x;
      out.y += b * rr.y;
    }
    vbar[m] = out;
  }
}

unsigned blocks_for(size_t n) { return unsigned(std::min<size_t>((n + VT - 1) / VT, 4096)); }

}  // namespace

int vjp_primal(int n, const float* x_new, float* xbar, const float* xtbar, float* zbar, hipStream_t s) {
  hipLaunchKernelGGL(k_vjp_primal, dim3(blocks_for(n)), dim3(VT), 0, s, n, x_new, xbar, xtbar, zbar);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

int vjp_param_grads(int n, const float* zbar, const float* st, const float* g, double tau, double sigma,
                    double varsigma, double* part, int nparts, double* pgrad, hipStream_t s) {
  hipLaunchKernelGGL(k_dot2, dim3(nparts), dim3(VT), 0, s, n, zbar, st, g, sigma, varsigma, part);
  RI_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_dot2_final, dim3(1), dim3(64), 0, s, part, nparts, tau, pgrad);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

int vjp_clip(size_t count, const float* s_new, float alpha, const float* wts, const float* w, float c, float* sbar,
             hipStream_t s) {
  hipLaunchKernelGGL(k_vjp_clip, dim3(blocks_for(count)), dim3(VT), 0, s, count, s_new, alpha, wts, w, c, sbar);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

int axpy(int n, float a, const float* x, float* y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy, dim3(blocks_for(n)), dim3(VT), 0, s, n, a, x, y);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

int ball_chunks(const Plan& p) {
  int64_t mx = 1;
  for (int i = 0; i < p.d; ++i) mx = std::max<int64_t>(mx, p.block_off_host[i + 1] - p.block_off_host[i]);
  return int((mx + BALL_CHUNK - 1) / BALL_CHUNK);
}

int vjp_ball(const Plan& p, const uint8_t* mask, float2* vbar, const float2* phiz, float c, const float2* r,
             const double* stats, const double* eps, double* part, double* coef, hipStream_t s) {
  const int nch = ball_chunks(p);
  const dim3 g(nch, p.d);
  hipLaunchKernelGGL(k_ball_dot, g, dim3(VT), 0, s, p.block_off, mask, vbar, phiz, c, r, nch, part);
  RI_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_ball_coef, dim3((p.d + 255) / 256), dim3(256), 0, s, p.d, p.block_off, mask, stats, eps, part,
                     nch, coef);
  RI_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_ball_apply, g, dim3(VT), 0, s, p.block_off, mask, vbar, phiz, c, r, coef);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

}  // namespace ri
