// Pruned 2D FFTs of the measurement operator: b~ = F Z S x (Algorithm 1 step 4) and its
// adjoint Re S Z^dagger F^dagger (step 17), on the K x K grid, K = 2n.
//
// Pixel (r, c) has centred coordinates l = (r - n/2, c - n/2) and lands on grid index
// q = l mod K, so only n of the K inputs per axis are nonzero: q in [0, n/2) maps back to
// pixel q + n/2 and q in [K - n/2, K) to pixel q - K + n/2.  The forward transform runs a
// row pass over the n nonzero image rows (K-point FFTs of zero-padded, S-scaled rows) into
// an n x K buffer, then a column pass over all K columns that reads only the n nonzero
// rows and writes the full grid.  The adjoint runs the column pass first, keeping only
// the n output rows that map back to pixels, then a row pass keeping n of K outputs and
// the real part, scaled by S.
#include "fft.hpp"
#include "plan.hpp"

namespace ri {

namespace {

__device__ __forceinline__ int pix_of(int q, int n, int K) {
  // grid index -> pixel index, or -1 outside the image support
  return q < n / 2 ? q + n / 2 : (q >= K - n / 2 ? q - K + n / 2 : -1);
}

template <int K>
struct RowCfg {
  static constexpr int W = (K / 2 < 2048 / K ? K / 2 : (2048 / K > 1 ? 2048 / K : 1));
  static constexpr int NT = K == 32 ? 64 : (K == 4096 ? 512 : 256);
};
template <int K>
struct ColCfg {
  static constexpr int W = K <= 1024 ? 16 : 16384 / K;
  static constexpr int NT = K <= 512 ? 256 : 512;
};

// Column panel of workgroup b of nb: consecutive blocks go round-robin to the eight XCDs,
// so neighbouring panels, which share 128-byte rows of the grid, are given to blocks on
// the same XCD (and its L2) when nb is a multiple of 8.
__device__ __forceinline__ int panel_of(int b, int nb) {
  return nb % 8 == 0 ? (b % 8) * (nb / 8) + b / 8 : b;
}

// Twiddles are staged in LDS when the panel and the table fit in 144 KiB together.
template <int K, int W>
struct TwLds {
  static constexpr bool fits = (K * W + K) * 8 <= 144 * 1024;
  static constexpr int size = fits ? K : 1;
};

template <int K, int W, int NT>
__global__ __launch_bounds__(NT) void k_fwd_rows(const float* __restrict__ x, const float* __restrict__ S,
                                                 float2* __restrict__ rows, const float2* __restrict__ tw) {
  constexpr int n = K / 2;
  __shared__ float2 lds[K * W];
  __shared__ float2 twl[TwLds<K, W>::size];
  const int r0 = blockIdx.x * W;
  auto load = [&](int w, int q) -> float2 {
    const int c = pix_of(q, n, K);
    if (c < 0) return make_float2(0.f, 0.f);
    const int r = r0 + w;
    return make_float2(x[size_t(r) * n + c] * (S[r] * S[c]), 0.f);
  };
  auto store = [&](int w, int k, float2 v) { rows[size_t(r0 + w) * K + k] = v; };
  FftPanel<K, W, NT, -1, false>::template run<TwLds<K, W>::fits>(lds, tw, twl, load, store);
}

template <int K, int W, int NT>
__global__ __launch_bounds__(NT) void k_fwd_cols(const float2* __restrict__ rows, float2* __restrict__ grid,
                                                 const float2* __restrict__ tw) {
  constexpr int n = K / 2;
  __shared__ float2 lds[K * W];
  __shared__ float2 twl[TwLds<K, W>::size];
  const int c0 = panel_of(blockIdx.x, gridDim.x) * W;
  auto load = [&](int w, int q) -> float2 {
    const int r = pix_of(q, n, K);
    if (r < 0) return make_float2(0.f, 0.f);
    return rows[size_t(r) * K + c0 + w];
  };
  auto store = [&](int w, int k, float2 v) { grid[size_t(k) * K + c0 + w] = v; };
  FftPanel<K, W, NT, -1, true>::template run<TwLds<K, W>::fits>(lds, tw, twl, load, store);
}

template <int K, int W, int NT>
__global__ __launch_bounds__(NT) void k_adj_cols(const float2* __restrict__ grid, float2* __restrict__ rows,
                                                 const float2* __restrict__ tw) {
  constexpr int n = K / 2;
  __shared__ float2 lds[K * W];
  __shared__ float2 twl[TwLds<K, W>::size];
  const int c0 = panel_of(blockIdx.x, gridDim.x) * W;
  auto load = [&](int w, int k) -> float2 { return grid[size_t(k) * K + c0 + w]; };
  // the data branch's kernels issue ahead of the sparsity branch's waves sharing their SIMDs
  __builtin_amdgcn_s_setprio(3);
  auto store = [&](int w, int q, float2 v) {
    const int r = pix_of(q, n, K);
    if (r >= 0) rows[size_t(r) * K + c0 + w] = v;
  };
  FftPanel<K, W, NT, +1, true>::template run<TwLds<K, W>::fits>(lds, tw, twl, load, store);
}

// UPD: the output g = Re S (...) feeds steps 17-18 (PrimalUpdate) instead of being stored.
template <int K, int W, int NT, bool UPD>
__global__ __launch_bounds__(NT) void k_adj_rows(const float2* __restrict__ rows, const float* __restrict__ S,
                                                 float* __restrict__ x, const float2* __restrict__ tw,
                                                 PrimalUpdate u) {
  constexpr int n = K / 2;
  __shared__ float2 lds[K * W];
  __shared__ float2 twl[TwLds<K, W>::size];
  const int r0 = blockIdx.x * W;
  // With one row per workgroup, K / 8 threads and a radix-8 last pass, thread t stores the
  // outputs t + i K / 8, i < 8, of which i = 0, 1, 6, 7 are pixels: their x and s~ are
  // loaded before the transform, so the update does not wait for them at the end.
  constexpr bool PREF = UPD && W == 1 && NT == K / 8 && FftPanel<K, W, NT, +1, false>::RB == 8;
  float xp[4] = {0.f, 0.f, 0.f, 0.f}, sp[4] = {0.f, 0.f, 0.f, 0.f};
  if constexpr (PREF) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = threadIdx.x + (i < 2 ? i : i + 4) * (K / 8);
      const size_t o = size_t(r0) * n + pix_of(q, n, K);
      xp[i] = u.x[o];
      sp[i] = u.st[o];
    }
  }
  auto load = [&](int w, int k) -> float2 { return rows[size_t(r0 + w) * K + k]; };
  auto store = [&](int w, int q, float2 v) {
    const int c = pix_of(q, n, K);
    if (c >= 0) {
      const int r = r0 + w;
      const size_t o = size_t(r) * n + c;
      const float g = v.x * (S[r] * S[c]);
      if (UPD) {
        float xo, so;
        if constexpr (PREF) {
          const int i = q < K / 8 ? 0 : (q < K / 4 ? 1 : (q < 7 * K / 8 ? 2 : 3));
          xo = i == 0 ? xp[0] : (i == 1 ? xp[1] : (i == 2 ? xp[2] : xp[3]));
          so = i == 0 ? sp[0] : (i == 1 ? sp[1] : (i == 2 ? sp[2] : sp[3]));
        } else {
          xo = u.x[o];
          so = u.st[o];
        }
        const float xn = fmaxf(0.f, xo - u.tau * (u.sigma * so + u.varsigma * g));
        u.x[o] = xn;
        u.xt[o] = 2.f * xn - xo;
      } else {
        x[o] = g;
      }
    }
  };
  FftPanel<K, W, NT, +1, false>::template run<TwLds<K, W>::fits>(lds, tw, twl, load, store);
}

template <int K>
int fwd_rows_impl(const Plan& p, const float* x, float2*, hipStream_t s) {
  using RC = RowCfg<K>;
  hipLaunchKernelGGL((k_fwd_rows<K, RC::W, RC::NT>), dim3(K / 2 / RC::W), dim3(RC::NT), 0, s, x, p.scale,
                     p.rowbuf, p.twiddle);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

template <int K>
int fwd_cols_impl(const Plan& p, const float*, float2* grid, hipStream_t s) {
  using CC = ColCfg<K>;
  hipLaunchKernelGGL((k_fwd_cols<K, CC::W, CC::NT>), dim3(K / CC::W), dim3(CC::NT), 0, s, p.rowbuf, grid,
                     p.twiddle);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

template <int K>
int adj_cols_impl(const Plan& p, const float2* grid, float*, hipStream_t s) {
  using CC = ColCfg<K>;
  hipLaunchKernelGGL((k_adj_cols<K, CC::W, CC::NT>), dim3(K / CC::W), dim3(CC::NT), 0, s, grid, p.rowbuf,
                     p.twiddle);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

template <int K>
int adj_rows_impl(const Plan& p, const float2*, float* x, hipStream_t s) {
  using RC = RowCfg<K>;
  hipLaunchKernelGGL((k_adj_rows<K, RC::W, RC::NT, false>), dim3(K / 2 / RC::W), dim3(RC::NT), 0, s, p.rowbuf,
                     p.scale, x, p.twiddle, PrimalUpdate{});
  RI_LAUNCH_CHECK();
  return RI_OK;
}

template <int K>
int adj_rows_update_impl(const Plan& p, const PrimalUpdate& u, hipStream_t s) {
  using RC = RowCfg<K>;
  hipLaunchKernelGGL((k_adj_rows<K, RC::W, RC::NT, true>), dim3(K / 2 / RC::W), dim3(RC::NT), 0, s, p.rowbuf,
                     p.scale, nullptr, p.twiddle, u);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

}  // namespace

#define RI_FFT_DISPATCH(FN, ...)                                          \
  switch (p.K) {                                                          \
    case 32: return FN<32>(__VA_ARGS__);                                  \
    case 64: return FN<64>(__VA_ARGS__);                                  \
    case 128: return FN<128>(__VA_ARGS__);                                \
    case 256: return FN<256>(__VA_ARGS__);                                \
    case 512: return FN<512>(__VA_ARGS__);                                \
    case 1024: return FN<1024>(__VA_ARGS__);                              \
    case 2048: return FN<2048>(__VA_ARGS__);                              \
    case 4096: return FN<4096>(__VA_ARGS__);                              \
    default: return fail(RI_EINVAL, "unsupported FFT size K=%d", p.K);    \
  }

int fft_forward_rows(const Plan& p, const float* x, hipStream_t s) {
  RI_FFT_DISPATCH(fwd_rows_impl, p, x, nullptr, s)
}

int fft_forward_cols(const Plan& p, float2* grid, hipStream_t s) {
  RI_FFT_DISPATCH(fwd_cols_impl, p, nullptr, grid, s)
}

int fft_adjoint_cols(const Plan& p, const float2* grid, hipStream_t s) {
  RI_FFT_DISPATCH(adj_cols_impl, p, grid, nullptr, s)
}

int fft_adjoint_rows(const Plan& p, float* x, hipStream_t s) {
  RI_FFT_DISPATCH(adj_rows_impl, p, nullptr, x, s)
}

int fft_adjoint_rows_update(const Plan& p, const PrimalUpdate& u, hipStream_t s) {
  RI_FFT_DISPATCH(adj_rows_update_impl, p, u, s)
}

int fft_forward(const Plan& p, const float* x, float2* grid, hipStream_t s) {
  RI_TRY(fft_forward_rows(p, x, s));
  return fft_forward_cols(p, grid, s);
}

int fft_adjoint(const Plan& p, const float2* grid, float* x, hipStream_t s) {
  RI_TRY(fft_adjoint_cols(p, grid, s));
  return fft_adjoint_rows(p, x, s);
}

}  // namespace ri
