// Internal state of the SARA sparsity dictionary (Sec. III): Dirac plus Daubechies bases.
#pragma once

#include "common.hpp"

namespace ri {

constexpr int MAX_WAVELETS = 8;
constexpr int MAX_TAPS = 16;  // db8

// Filters of the wavelet bases, by wavelet slot.  On the device they live in one buffer,
// FILT_STRIDE floats per slot (lowpass h in [0, 16), highpass g in [16, 32)), read through
// a pointer with uniform indices (scalar loads).
constexpr int FILT_STRIDE = 2 * MAX_TAPS;
struct SaraFilters {
  float h[MAX_WAVELETS][MAX_TAPS];
  float g[MAX_WAVELETS][MAX_TAPS];
  int len[MAX_WAVELETS];
};

struct Sara {
  int n = 0, levels = 0;
  int dirac = 0;  // 1 if basis 0 is the Dirac basis
  int nw = 0;     // number of wavelet bases
  int b = 0;      // dirac + nw
  SaraFilters filt{};
  float* dfilt = nullptr;  // nw * FILT_STRIDE
  int* dlen = nullptr;     // nw
  size_t tmp_stride = 0;        // floats of LL scratch per wavelet
  size_t tmp_off[8] = {0};      // offset of LL_l (l = 1..levels-1) inside a wavelet's scratch
  float* tmp = nullptr;         // nw * tmp_stride
  float* coef_tmp = nullptr;    // b * n * n, power iterations
  float* vec_tmp = nullptr;     // n * n, power iterations
  double* dsum = nullptr;
};

// s = Psi^dagger x, or with clip: s = clip(s + Psi^dagger x, -alpha, alpha) (step 13 Moreau form);
// with weights wts (b*n*n, the layout of s) the bound of coefficient k is alpha * wts[k].
int psi_adj_apply(const Sara& S, const float* x, float* s, bool clip, float alpha, hipStream_t st,
                  const float* wts = nullptr);
// x = Psi s.
int psi_apply(const Sara& S, const float* s, float* x, hipStream_t st);


}  // namespace ri
