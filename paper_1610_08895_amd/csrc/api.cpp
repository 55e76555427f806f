// Library-wide entry points: error reporting, versions, and the host-side probability
// rules of Sec. IV (Eqs. 13 and 14).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "common.hpp"

namespace ri {

namespace {
thread_local std::string g_err;
int g_cus = 0;
}  // namespace

void set_error_msg(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

const char* error_msg() { return g_err.c_str(); }

int device_cus() {
  if (g_cus > 0) return g_cus;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
    g_cus = cus;
  else
    g_cus = 256;
  return g_cus;
}

}  // namespace ri

using ri::fail;

extern "C" {

const char* ri_last_error(void) { return ri::error_msg(); }

int ri_version(void) { return 10000; }

int ri_hip_runtime_version(int* out) {
  if (!out) return fail(RI_EINVAL, "out is NULL");
  RI_HIP(hipRuntimeGetVersion(out));
  return RI_OK;
}

int ri_residual_energy(const double* resid_norm, const double* eps, int d, double* c_out) {
  if (!resid_norm || !eps || !c_out || d < 1) return fail(RI_EINVAL, "bad argument");
  for (int i = 0; i < d; ++i) {
    if (!(eps[i] > 0)) return fail(RI_EINVAL, "eps[%d] must be positive", i);
    const double over = resid_norm[i] - eps[i];
    c_out[i] = over > 0 ? (over * over) / (eps[i] * eps[i]) : 0.0;
  }
  return RI_OK;
}

// Eq. 14 by successive saturation: start from a = 0; whenever some unsaturated block would
// exceed p_max - p_min at the current a, saturate it and recompute a so that the
// unsaturated blocks absorb the remaining mass evenly.  a never decreases between rounds,
// so a block once saturated stays saturated, and at most d rounds are needed.
int ri_probs(const double* c, int d, double n_nodes, double p_min, double p_max, double* p_out,
             double* a_out) {
  if (!c || !p_out || d < 1) return fail(RI_EINVAL, "bad argument");
  if (!(p_min > 0 && p_min <= n_nodes / d && n_nodes / d <= p_max && p_max <= 1.0))
    return fail(RI_EINVAL, "need 0 < p_min <= n/d <= p_max <= 1 (p_min %g, n/d %g, p_max %g)", p_min,
                n_nodes / d, p_max);
  double total = 0.0;
  for (int i = 0; i < d; ++i) {
    if (!(c[i] >= 0) || !std::isfinite(c[i])) return fail(RI_EINVAL, "c[%d] must be finite and >= 0", i);
    total += c[i];
  }
  if (total == 0.0) {
    for (int i = 0; i < d; ++i) p_out[i] = n_nodes / d;
    if (a_out) *a_out = 0.0;
    return RI_OK;
  }
  const double R = n_nodes - d * p_min, cap = p_max - p_min;
  std::vector<double> w(d);
  std::vector<char> sat(d, 0);
  for (int i = 0; i < d; ++i) w[i] = R * c[i] / total;
  double a = 0.0;
  for (int round = 0; round <= d; ++round) {
    bool grew = false;
    for (int i = 0; i < d; ++i)
      if (!sat[i] && w[i] + a > cap) {
        sat[i] = 1;
        grew = true;
      }
    if (!grew) break;
    int nfree = 0;
    double free_mass = 0.0;
    for (int i = 0; i < d; ++i)
      if (!sat[i]) {
        ++nfree;
        free_mass += w[i];
      }
    if (nfree == 0) {
      a = cap;
      break;
    }
    const double nsat = double(d - nfree);
    a = (R - nsat * cap - free_mass) / nfree;
    if (a < 0.0) a = 0.0;
  }
  for (int i = 0; i < d; ++i) p_out[i] = p_min + (w[i] + a < cap ? w[i] + a : cap);
  if (a_out) *a_out = a;
  return RI_OK;
}

}  // extern "C"
