// Host-side FP64 numerics that set up the device tables: the Kaiser-Bessel
// interpolation kernel (its weights as per-tap polynomials, its Fourier transform for
// the pre-compensation S of Eq. 3), twiddle factors, and the Daubechies filters of the
// SARA dictionary.  Everything is derived here from the mathematical definitions.
#include "host_math.hpp"

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace ri {

// Modified Bessel function of the first kind, order 0, from its power series
// I0(x) = sum_k ((x/2)^k / k!)^2.  All terms are positive, so the partial sums lose no
// precision; the series is summed until a term no longer changes the total.
double bessel_i0(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 500; ++k) {
    term *= q / (double(k) * double(k));
    const double next = sum + term;
    if (next == sum) break;
    sum = next;
  }
  return sum;
}

double kb_weight(double t, int J, double beta) {
  const double a = 1.0 - (2.0 * t / J) * (2.0 * t / J);
  if (a < 0.0) return 0.0;
  return bessel_i0(beta * std::sqrt(a)) / bessel_i0(beta);
}

// Fourier transform of the Kaiser-Bessel window over |t| <= J/2:
// J sinh(z) / (z I0(beta)), z = sqrt(beta^2 - (pi J f)^2), for pi J |f| < beta.
double kb_hat(double f, int J, double beta) {
  const double z = std::sqrt(beta * beta - (M_PI * J * f) * (M_PI * J * f));
  return J * std::sinh(z) / (z * bessel_i0(beta));
}

// Tap j (0 <= j < J/2) sits at distance t = f + J/2 - 1 - j from the visibility, f in
// [0, 1) the fractional grid coordinate.  With x = 2f - 1 the weight is fitted by a
// degree-D polynomial P_j(x) via Chebyshev interpolation; the mirrored tap J-1-j has
// weight P_j(-x) because the kernel is even.
int kb_fit_taps(int J, double beta, int D, std::vector<double>& mono, double* max_err) {
  const int half = J / 2;
  mono.assign(size_t(half) * (D + 1), 0.0);
  // monomial coefficients of T_0..T_D
  std::vector<std::vector<double>> T(D + 1, std::vector<double>(D + 1, 0.0));
  T[0][0] = 1.0;
  if (D >= 1) T[1][1] = 1.0;
  for (int k = 1; k < D; ++k)
    for (int p = 0; p <= D; ++p)
      T[k + 1][p] = (p > 0 ? 2.0 * T[k][p - 1] : 0.0) - T[k - 1][p];
  double worst = 0.0;
  for (int j = 0; j < half; ++j) {
    std::vector<double> fx(D + 1), c(D + 1, 0.0);
    std::vector<double> nodes(D + 1);
    for (int i = 0; i <= D; ++i) {
      nodes[i] = std::cos(M_PI * (i + 0.5) / (D + 1));
      const double f = 0.5 * (nodes[i] + 1.0);
      fx[i] = kb_weight(f + half - 1 - j, J, beta);
    }
    for (int k = 0; k <= D; ++k) {
      double s = 0.0;
      for (int i = 0; i <= D; ++i) s += fx[i] * std::cos(M_PI * k * (i + 0.5) / (D + 1));
      c[k] = (k == 0 ? 1.0 : 2.0) * s / (D + 1);
    }
    double* m = &mono[size_t(j) * (D + 1)];
    for (int k = 0; k <= D; ++k)
      for (int p = 0; p <= D; ++p) m[p] += c[k] * T[k][p];
    for (int s = 0; s <= 2000; ++s) {
      const double x = -1.0 + 2.0 * s / 2000.0;
      double acc = 0.0;
      for (int p = D; p >= 0; --p) acc = acc * x + m[p];
      const double ref = kb_weight(0.5 * (x + 1.0) + half - 1 - j, J, beta);
      worst = std::max(worst, std::fabs(acc - ref));
    }
  }
  if (max_err) *max_err = worst;
  return 0;
}

// ---- Daubechies filters ----------------------------------------------------------------
// |H(w)|^2 = 2 cos^{2N}(w/2) P(sin^2(w/2)), P(y) = sum_{k<N} C(N-1+k, k) y^k.  Each root
// y_k of P gives a pair of zeros z, 1/z of z^2 - (2 - 4 y_k) z + 1; keeping the zero inside
// the unit circle gives the minimum-phase factor
// H(z) = c (1 + z^-1)^N prod_k (1 - z_k z^-1), normalised to sum h = sqrt 2.

static double binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Roots of sum_k a[k] y^k (degree deg >= 1) by the Durand-Kerner (Weierstrass)
// simultaneous iteration, followed by Newton polishing.
static std::vector<std::complex<double>> poly_roots(const std::vector<double>& a) {
  using C = std::complex<double>;
  const int deg = int(a.size()) - 1;
  std::vector<C> r(deg);
  const C seed(0.4, 0.9);
  C p = 1.0;
  for (int i = 0; i < deg; ++i) {
    r[i] = p;
    p *= seed;
  }
  auto eval = [&](C y) {
    C acc = 0.0;
    for (int k = deg; k >= 0; --k) acc = acc * y + a[k] / a[deg];
    return acc;
  };
  for (int it = 0; it < 2000; ++it) {
    double change = 0.0;
    for (int i = 0; i < deg; ++i) {
      C den = 1.0;
      for (int j = 0; j < deg; ++j)
        if (j != i) den *= (r[i] - r[j]);
      const C step = eval(r[i]) / den;
      r[i] -= step;
      change = std::max(change, std::abs(step));
    }
    if (change < 1e-16) break;
  }
  for (auto& y : r) {
    for (int it = 0; it < 3; ++it) {
      C f = 0.0, df = 0.0;
      for (int k = deg; k >= 0; --k) {
        df = df * y + f;
        f = f * y + a[k];
      }
      if (std::abs(df) > 0) y -= f / df;
    }
  }
  return r;
}

int daubechies_lowpass(int N, std::vector<double>& h, double* orth_err) {
  using C = std::complex<double>;
  std::vector<C> poly{1.0};
  auto mul = [&](C c0, C c1) {  // poly *= (c0 + c1 w), w = z^-1
    std::vector<C> out(poly.size() + 1, 0.0);
    for (size_t i = 0; i < poly.size(); ++i) {
      out[i] += c0 * poly[i];
      out[i + 1] += c1 * poly[i];
    }
    poly.swap(out);
  };
  for (int i = 0; i < N; ++i) mul(1.0, 1.0);
  if (N > 1) {
    std::vector<double> P(N);
    for (int k = 0; k < N; ++k) P[k] = binom(N - 1 + k, k);
    for (const C& y : poly_roots(P)) {
      const C b = 2.0 - 4.0 * y;             // z + 1/z = b
      const C disc = std::sqrt(b * b - 4.0);
      C z = 0.5 * (b + disc);
      if (std::abs(z) > 1.0) z = 0.5 * (b - disc);
      mul(1.0, -z);
    }
  }
  h.assign(2 * N, 0.0);
  double sum = 0.0;
  for (int i = 0; i < 2 * N; ++i) sum += (h[i] = poly[i].real());
  for (auto& v : h) v *= std::sqrt(2.0) / sum;
  double err = 0.0;
  for (int l = 0; l < N; ++l) {
    double s = 0.0;
    for (int k = 0; k + 2 * l < 2 * N; ++k) s += h[k] * h[k + 2 * l];
    err = std::max(err, std::fabs(s - (l == 0 ? 1.0 : 0.0)));
  }
  if (orth_err) *orth_err = err;
  return 0;
}

}  // namespace ri
