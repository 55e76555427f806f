// FP64 host numerics used to build the device tables (see host_math.cpp).
#pragma once
#include <vector>

namespace ri {

double bessel_i0(double x);
double kb_weight(double t, int J, double beta);
double kb_hat(double f, int J, double beta);
// Per-tap monomial coefficients (J/2 rows of D+1, increasing powers of x = 2f - 1).
int kb_fit_taps(int J, double beta, int D, std::vector<double>& mono, double* max_err);
// Minimum-phase Daubechies lowpass with N vanishing moments, sum h = sqrt 2.
int daubechies_lowpass(int N, std::vector<double>& h, double* orth_err);

}  // namespace ri
