// Launchers of the reverse-sweep kernels (vjp.hip); the sweep itself is ri_pd_step_vjp.
#pragma once

#include <algorithm>

#include "plan.hpp"

namespace ri {

// zbar = (xbar + 2 xtbar) [x_new > 0]; xbar <- zbar - xtbar   (n floats)
int vjp_primal(int n, const float* x_new, float* xbar, const float* xtbar, float* zbar, hipStream_t s);
// pgrad[0] -= <zbar, sigma st + varsigma g>, pgrad[1] -= tau <zbar, st> (FP64, fixed order;
// part: 2 * nparts doubles of scratch)
int vjp_param_grads(int n, const float* zbar, const float* st, const float* g, double tau, double sigma,
                    double varsigma, double* part, int nparts, double* pgrad, hipStream_t s);
// sbar <- (sbar + c w) [|s_new| < bound], bound = alpha, or alpha * wts[k] with weights
int vjp_clip(size_t count, const float* s_new, float alpha, const float* wts, const float* w, float c, float* sbar,
             hipStream_t s);
// y += a x
int axpy(int n, float a, const float* x, float* y, hipStream_t s);
// Per-block FP64 partials needed by vjp_ball: d * ball_chunks(p) doubles.
int ball_chunks(const Plan& p);
// vbar <- step-8 VJP of u = vbar + c phiz per block (see vjp.hip); part: d * ball_chunks,
// coef: 2 d doubles of scratch.
// r: v_old + G b - y of the step (RI_PD_E after it).
int vjp_ball(const Plan& p, const uint8_t* mask, float2* vbar, const float2* phiz, float c, const float2* r,
             const double* stats, const double* eps, double* part, double* coef, hipStream_t s);

}  // namespace ri
