// SARA dictionary: Psi^dagger (analysis, Algorithm 1 step 13) and Psi (synthesis,
// step 14) for the Dirac basis plus Daubechies wavelets, as periodic separable 2D filter
// banks.  One analysis level of an m x m input, per axis:
//   a[k] = sum_j h[j] x[(2k + j) mod m],   d[k] = sum_j g[j] x[(2k + j) mod m],
// x (columns) first, then y (rows), written in Mallat layout; synthesis is the transpose.
//
// Each workgroup owns an output tile and stages the input it needs in LDS together with
// its periodic halo (filter length - 2 samples), then runs the row and the column filters
// from LDS; the filter length is a compile-time constant per basis.  Synthesis computes
// output pairs (2q, 2q + 1) from the same coefficients a[q - u], d[q - u].  Analysis of
// level 1 reads x~ once per wavelet from L2; the dual update of step 13,
// s = clip(s + Psi^dagger x~, -alpha, alpha), is applied as each coefficient is produced,
// with the old coefficients loaded before the input is staged; for the weighted l1 prior of
// reweighted SARA the bound is alpha w_k, with the weights w laid out like s.  The last
// synthesis level sums all bases in registers.
#include <cmath>
#include <new>
#include <vector>

#include "host_math.hpp"
#include "handles.hpp"
#include "sara.hpp"

namespace ri {
namespace {

constexpr int ST = 256;  // threads per workgroup
constexpr int TO = 16;   // analysis: outputs per subband per axis per workgroup
constexpr int TS = 32;   // synthesis: outputs per axis per workgroup

__device__ __forceinline__ float clampf(float v, float a) { return fminf(fmaxf(v, -a), a); }

// Tile (tx, ty) of this workgroup in a gridDim.x x gridDim.y tile grid.  Consecutive
// workgroups go round-robin to the eight XCDs, so with a row-major order neighbouring tiles,
// whose staged regions overlap, would sit on different XCDs; when the row count is a
// multiple of 8, each XCD takes a band of whole tile rows instead, and the overlaps are
// fetched once into its L2.
__device__ __forceinline__ void band_tile(int& tx, int& ty) {
  const int nx = gridDim.x, ny = gridDim.y;
  if (ny % 8 != 0) {
    tx = blockIdx.x;
    ty = blockIdx.y;
    return;
  }
  const int b = blockIdx.x + nx * blockIdx.y, i = b / 8;
  ty = (b % 8) * (ny / 8) + i / nx;
  tx = i - (i / nx) * nx;
}

struct DwtArgs {
  const float* x;  // level-1 input (n x n)
  float* tmp;
  size_t tmp_stride, in_off, out_off;
  float* s;
  int n, m, level, levels, dirac, nw;
  int clip;
  float alpha;
  const float* wts;  // per-coefficient weights of the clip bound (layout of s), or null
};

// bound of the clip at coefficient k of s: alpha, or alpha w_k (the same FP32 product
// wherever it is formed, so a clipped value equals the bound exactly)
__device__ __forceinline__ float clip_bound(const DwtArgs& A, size_t k) {
  return A.wts != nullptr ? A.alpha * A.wts[k] : A.alpha;
}

__device__ __forceinline__ void put_coef(const DwtArgs& A, size_t k, float v) {
  A.s[k] = A.clip ? clampf(A.s[k] + v, clip_bound(A, k)) : v;
}

// One analysis level for wavelet w with filters of (compile-time) length L on an output
// tile (i0, j0) of each subband.  Sizes are powers of two, so indices wrap with masks.
template <int L>
__device__ __forceinline__ void analysis_tile(const DwtArgs& A, const float* __restrict__ hw, int w, int i0,
                                              int j0, float* in, float* lo, float* hi) {
  const float* __restrict__ gw = hw + MAX_TAPS;
  constexpr int RE = 2 * TO + L - 2;       // input rows / columns the tile reads
  constexpr int RW = 2 * TO + MAX_TAPS - 2; // LDS row stride
  const int n = A.n, m = A.m, mo = A.m / 2, mm = A.m - 1;
  const float* src = A.level == 1 ? A.x : A.tmp + w * A.tmp_stride + A.in_off;
  float* sb = A.s + size_t(w + A.dirac) * n * n;
  // the coefficients this thread updates (one output position per thread: TO * TO == ST),
  // loaded now so that their latency overlaps the staging and the filters
  static_assert(TO * TO == ST, "one output position per thread");
  const int pi = threadIdx.x / TO, pj = threadIdx.x - (threadIdx.x / TO) * TO;
  const int qi = i0 + pi, qj = j0 + pj;
  const bool mine = qi < mo && qj < mo;
  float old[4] = {0.f, 0.f, 0.f, 0.f}, bnd[4] = {A.alpha, A.alpha, A.alpha, A.alpha};
  const size_t sbo = size_t(w + A.dirac) * n * n;
  const size_t ko[4] = {size_t(qi) * n + qj, size_t(qi) * n + mo + qj, size_t(mo + qi) * n + qj,
                        size_t(mo + qi) * n + mo + qj};
  if (A.clip && mine) {
    if (A.level == A.levels) old[0] = sb[ko[0]];
    old[1] = sb[ko[1]];
    old[2] = sb[ko[2]];
    old[3] = sb[ko[3]];
    if (A.wts != nullptr)
#pragma unroll
      for (int c = 0; c < 4; ++c) bnd[c] = clip_bound(A, sbo + ko[c]);
  }
  for (int idx = threadIdx.x; idx < RE * RE; idx += ST) {
    const int ly = idx / RE, lx = idx - ly * RE;
    in[ly * RW + lx] = src[size_t((2 * i0 + ly) & mm) * m + ((2 * j0 + lx) & mm)];
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < RE * TO; idx += ST) {
    const int rho = idx / TO, j = idx - rho * TO;
    const float* row = &in[rho * RW + 2 * j];
    float a = 0.f, d = 0.f;
#pragma unroll
    for (int t = 0; t < L; ++t) {
      a = fmaf(hw[t], row[t], a);
      d = fmaf(gw[t], row[t], d);
    }
    lo[rho * TO + j] = a;
    hi[rho * TO + j] = d;
  }
  __syncthreads();
  if (!mine) return;
  float ll = 0.f, lh = 0.f, hl = 0.f, hh = 0.f;
#pragma unroll
  for (int t = 0; t < L; ++t) {
    const float l = lo[(2 * pi + t) * TO + pj], h = hi[(2 * pi + t) * TO + pj];
    ll = fmaf(hw[t], l, ll);
    lh = fmaf(hw[t], h, lh);
    hl = fmaf(gw[t], l, hl);
    hh = fmaf(gw[t], h, hh);
  }
  auto put = [&](int c, float v) { sb[ko[c]] = A.clip ? clampf(old[c] + v, bnd[c]) : v; };
  if (A.level < A.levels) A.tmp[w * A.tmp_stride + A.out_off + size_t(qi) * mo + qj] = ll;
  else put(0, ll);
  put(1, lh);
  put(2, hl);
  put(3, hh);
}

#define RI_SWITCH_L(LEN, CALL)          \
  switch (LEN) {                        \
    case 2: CALL(2); break;             \
    case 4: CALL(4); break;             \
    case 6: CALL(6); break;             \
    case 8: CALL(8); break;             \
    case 10: CALL(10); break;           \
    case 12: CALL(12); break;           \
    case 14: CALL(14); break;           \
    default: CALL(16); break;           \
  }

__global__ __launch_bounds__(ST) void k_dwt_level(DwtArgs A, const float* __restrict__ filt,
                                                  const int* __restrict__ flen) {
  constexpr int RW = 2 * TO + MAX_TAPS - 2;
  __shared__ float in[RW * RW];
  __shared__ float lo[RW * TO], hi[RW * TO];
  const int n = A.n;
  int tx, ty;
  band_tile(tx, ty);
  const int i0 = ty * TO, j0 = tx * TO;
  const int z = blockIdx.z;
  if (z == A.nw) {  // Dirac basis at level 1: coefficient = pixel
    for (int idx = threadIdx.x; idx < 4 * TO * TO; idx += ST) {
      const int r = 2 * i0 + idx / (2 * TO), c = 2 * j0 + idx % (2 * TO);
      if (r < n && c < n) put_coef(A, size_t(r) * n + c, A.x[size_t(r) * n + c]);
    }
    return;
  }
#define RI_ANALYSIS(LL) analysis_tile<LL>(A, filt + z * FILT_STRIDE, z, i0, j0, in, lo, hi)
  RI_SWITCH_L(flen[z], RI_ANALYSIS)
#undef RI_ANALYSIS
}

struct IdwtArgs {
  const float* s;
  float* tmp;
  size_t tmp_stride, ll_off, out_off;
  int n, m, level, levels, dirac, nw;
  float* x;  // top level only: the image Psi s
};

constexpr int RS = TS / 2 + MAX_TAPS / 2;  // LDS stride of a staged subband region

// Coefficients of one synthesis tile: output tile (p0, q0) of wavelet w (half filter
// length H) reads rows / columns [p0 / 2 - H, p0 / 2 + TS / 2) and [q0 / 2 - H, ...) of
// each of its four subbands (periodic).  A thread holds elements idx = threadIdx.x + e * ST
// of the RL x RL region, RL = TS / 2 + H, at (idx / RL, idx % RL).
constexpr int STAGE_PER = (RS * RS + ST - 1) / ST;
struct Stage {
  float v[4][STAGE_PER];
};

__device__ __forceinline__ void fetch_stage(const IdwtArgs& A, int w, int H, int p0, int q0, Stage& r) {
  const int RL = TS / 2 + H;
  const int n = A.n, mo = A.m / 2, mk = A.m / 2 - 1;
  const int kr = p0 / 2 - H, kc = q0 / 2 - H;
  const float* sw = A.s + size_t(w + A.dirac) * n * n;
  const bool ll_coef = A.level == A.levels;
  const float* ll = ll_coef ? sw : A.tmp + w * A.tmp_stride + A.ll_off;
  const int ll_stride = ll_coef ? n : mo;
#pragma unroll
  for (int e = 0; e < STAGE_PER; ++e) {
    const int idx = threadIdx.x + e * ST;
    if (idx >= RL * RL) break;
    const int ky = idx / RL, kx = idx - ky * RL;
    const int gy = (kr + ky) & mk, gx = (kc + kx) & mk;
    r.v[0][e] = ll[size_t(gy) * ll_stride + gx];
    r.v[1][e] = sw[size_t(gy) * n + mo + gx];       // low-y, high-x
    r.v[2][e] = sw[size_t(mo + gy) * n + gx];       // high-y, low-x
    r.v[3][e] = sw[size_t(mo + gy) * n + mo + gx];  // high-y, high-x
  }
}

__device__ __forceinline__ void deposit_stage(int H, const Stage& r, float (*sb)[RS * RS]) {
  const int RL = TS / 2 + H;
#pragma unroll
  for (int e = 0; e < STAGE_PER; ++e) {
    const int idx = threadIdx.x + e * ST;
    if (idx >= RL * RL) break;
    const int ky = idx / RL, kx = idx - ky * RL;
#pragma unroll
    for (int c = 0; c < 4; ++c) sb[c][ky * RS + kx] = r.v[c][e];
  }
}

// One synthesis level for one wavelet (filters of length L) on a tile whose coefficients
// are staged in sb: out[2q + r] = sum_u h[2u + r] a[q - u] + g[2u + r] d[q - u] along each
// axis (the transpose of the analysis), columns (y) first into lo / hi, then rows (x).
// Returns through `emit(k, pl, q, v_even, v_odd)` the output pairs (p0 + pl, q0 + 2q +
// {0, 1}).  Requires sb complete (a barrier after staging); ends after the barrier
// between its two passes, so sb may be overwritten once it returns.
template <int L, class Emit>
__device__ __forceinline__ void synthesis_staged(const float* __restrict__ hw, const float (*sb)[RS * RS],
                                                 float* lo, float* hi, Emit& emit) {
  const float* __restrict__ gw = hw + MAX_TAPS;
  constexpr int H = L / 2;
  constexpr int RL = TS / 2 + H;
  for (int idx = threadIdx.x; idx < (TS / 2) * RL; idx += ST) {
    const int qy = idx / RL, jl = idx - qy * RL;
    float le = 0.f, lo_ = 0.f, he = 0.f, ho = 0.f;
#pragma unroll
    for (int u = 0; u < H; ++u) {
      const int k = (qy + H - u) * RS + jl;
      const float a0 = sb[0][k], a1 = sb[1][k], a2 = sb[2][k], a3 = sb[3][k];
      le = fmaf(hw[2 * u], a0, fmaf(gw[2 * u], a2, le));
      lo_ = fmaf(hw[2 * u + 1], a0, fmaf(gw[2 * u + 1], a2, lo_));
      he = fmaf(hw[2 * u], a1, fmaf(gw[2 * u], a3, he));
      ho = fmaf(hw[2 * u + 1], a1, fmaf(gw[2 * u + 1], a3, ho));
    }
    lo[(2 * qy) * RS + jl] = le;
    lo[(2 * qy + 1) * RS + jl] = lo_;
    hi[(2 * qy) * RS + jl] = he;
    hi[(2 * qy + 1) * RS + jl] = ho;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < TS * TS / 2 / ST; ++k) {
    const int idx = threadIdx.x + k * ST;
    const int pl = idx / (TS / 2), qx = idx - pl * (TS / 2);
    float ve = 0.f, vo = 0.f;
#pragma unroll
    for (int u = 0; u < H; ++u) {
      const float a = lo[pl * RS + qx + H - u], d = hi[pl * RS + qx + H - u];
      ve = fmaf(hw[2 * u], a, fmaf(gw[2 * u], d, ve));
      vo = fmaf(hw[2 * u + 1], a, fmaf(gw[2 * u + 1], d, vo));
    }
    emit(k, pl, qx, ve, vo);
  }
}

__global__ __launch_bounds__(ST) void k_idwt_level(IdwtArgs A, const float* __restrict__ filt,
                                                   const int* __restrict__ flen) {
  __shared__ float sb[4][RS * RS];
  __shared__ float lo[TS * RS], hi[TS * RS];
  const int w = blockIdx.z;
  int tx, ty;
  band_tile(tx, ty);
  const int p0 = ty * TS, q0 = tx * TS, m = A.m;
  float* out = A.tmp + w * A.tmp_stride + A.out_off;
  auto emit = [&](int, int pl, int qx, float ve, float vo) {
    const int p = p0 + pl, q = q0 + 2 * qx;
    if (p < m && q < m) {
      out[size_t(p) * m + q] = ve;
      out[size_t(p) * m + q + 1] = vo;
    }
  };
  const int L = flen[w];
  Stage r;
  fetch_stage(A, w, L / 2, p0, q0, r);
  deposit_stage(L / 2, r, sb);
  __syncthreads();
#define RI_SYNTH(LL) synthesis_staged<LL>(filt + w * FILT_STRIDE, sb, lo, hi, emit)
  RI_SWITCH_L(L, RI_SYNTH)
#undef RI_SYNTH
}

// Last level: each workgroup sums all wavelets' syntheses of its tile in registers.  The
// coefficients of wavelet w + 1 are loaded into registers while wavelet w is computed and
// moved to LDS after its column pass, so the loads overlap the arithmetic.
__global__ __launch_bounds__(ST) void k_idwt_top(IdwtArgs A, const float* __restrict__ filt,
                                                 const int* __restrict__ flen) {
  constexpr int PER = TS * TS / 2 / ST;  // output pairs per thread
  __shared__ float sb[4][RS * RS];
  __shared__ float lo[TS * RS], hi[TS * RS];
  int tx, ty;
  band_tile(tx, ty);
  const int p0 = ty * TS, q0 = tx * TS, n = A.n;
  float acc_e[PER], acc_o[PER], dir[PER][2];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    acc_e[k] = acc_o[k] = 0.f;
    const int idx = threadIdx.x + k * ST;
    const int p = p0 + idx / (TS / 2), q = q0 + 2 * (idx % (TS / 2));
    const bool in = A.dirac && p < n && q < n;
    dir[k][0] = in ? A.s[size_t(p) * n + q] : 0.f;
    dir[k][1] = in ? A.s[size_t(p) * n + q + 1] : 0.f;
  }
  auto emit = [&](int k, int, int, float ve, float vo) {
    acc_e[k] += ve;
    acc_o[k] += vo;
  };
  if (A.nw > 0) {
    Stage r;
    fetch_stage(A, 0, flen[0] / 2, p0, q0, r);
    deposit_stage(flen[0] / 2, r, sb);
    __syncthreads();
    for (int w = 0; w < A.nw; ++w) {
      const int L = flen[w];
      const bool more = w + 1 < A.nw;
      const int Hn = more ? flen[w + 1] / 2 : 0;
      if (more) fetch_stage(A, w + 1, Hn, p0, q0, r);
#define RI_SYNTH(LL) synthesis_staged<LL>(filt + w * FILT_STRIDE, sb, lo, hi, emit)
      RI_SWITCH_L(L, RI_SYNTH)
#undef RI_SYNTH
      if (more) deposit_stage(Hn, r, sb);
      __syncthreads();
    }
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int idx = threadIdx.x + k * ST;
    const int p = p0 + idx / (TS / 2), q = q0 + 2 * (idx % (TS / 2));
    if (p >= n || q >= n) continue;
    A.x[size_t(p) * n + q] = acc_e[k] + dir[k][0];
    A.x[size_t(p) * n + q + 1] = acc_o[k] + dir[k][1];
  }
}

unsigned tiles(int outputs, int t) { return unsigned((outputs + t - 1) / t); }

int analysis(const Sara& S, const float* x, float* s, bool clip, float alpha, const float* wts, hipStream_t st) {
  for (int lev = 1; lev <= S.levels; ++lev) {
    const int m = S.n >> (lev - 1), mo = m / 2;
    DwtArgs A{x, S.tmp, S.tmp_stride, lev >= 2 ? S.tmp_off[lev - 1] : 0, lev < S.levels ? S.tmp_off[lev] : 0,
              s, S.n, m, lev, S.levels, S.dirac, S.nw, clip ? 1 : 0, alpha, wts};
    const int z = S.nw + ((lev == 1 && S.dirac) ? 1 : 0);
    if (z == 0) continue;
    hipLaunchKernelGGL(k_dwt_level, dim3(tiles(mo, TO), tiles(mo, TO), z), dim3(ST), 0, st, A, S.dfilt,
                       S.dlen);
    RI_LAUNCH_CHECK();
  }
  return RI_OK;
}

int synthesis_lower(const Sara& S, const float* s, hipStream_t st) {
  for (int lev = S.levels; lev >= 2; --lev) {
    const int m = S.n >> (lev - 1);
    IdwtArgs A{s, S.tmp, S.tmp_stride, lev < S.levels ? S.tmp_off[lev] : 0, S.tmp_off[lev - 1], S.n, m, lev,
               S.levels, S.dirac, S.nw, nullptr};
    if (S.nw == 0) break;
    hipLaunchKernelGGL(k_idwt_level, dim3(tiles(m, TS), tiles(m, TS), S.nw), dim3(ST), 0, st, A, S.dfilt,
                       S.dlen);
    RI_LAUNCH_CHECK();
  }
  return RI_OK;
}

int synthesis_top(const Sara& S, const float* s, float* x, hipStream_t st) {
  IdwtArgs A{s, S.tmp, S.tmp_stride, S.levels > 1 ? S.tmp_off[1] : 0, 0, S.n, S.n, 1, S.levels, S.dirac, S.nw, x};
  const dim3 g(tiles(S.n, TS), tiles(S.n, TS));
  hipLaunchKernelGGL(k_idwt_top, g, dim3(ST), 0, st, A, S.dfilt, S.dlen);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

void destroy_sara(Sara& S) {
  dev_free(S.tmp);
  dev_free(S.coef_tmp);
  dev_free(S.vec_tmp);
  dev_free(S.dsum);
  dev_free(S.dfilt);
  dev_free(S.dlen);
}

int create_sara(Sara& S, int n, int levels, uint32_t bases) {
  if (bases == 0) bases = 0x1FF;
  if (bases & ~0x1FFu) return fail(RI_EINVAL, "bases bitmask 0x%x has bits above db8", bases);
  if (levels < 1 || levels > 6) return fail(RI_EINVAL, "levels=%d must be in [1, 6]", levels);
  if (!is_pow2(n) || n > 4096 || n < (1 << levels) || n < 4)
    return fail(RI_EINVAL, "n=%d must be a power of two in [max(4, 2^levels), 4096] (levels=%d)", n, levels);
  S.n = n;
  S.levels = levels;
  S.dirac = (bases & 1u) ? 1 : 0;
  S.nw = 0;
  for (int N = 1; N <= 8; ++N) {
    if (!(bases & (1u << N))) continue;
    std::vector<double> h;
    double err = 1.0;
    daubechies_lowpass(N, h, &err);
    if (!(err < 1e-12)) return fail(RI_EINVAL, "db%d filter orthonormality error %.3g", N, err);
    const int w = S.nw++;
    S.filt.len[w] = 2 * N;
    for (int j = 0; j < 2 * N; ++j) {
      S.filt.h[w][j] = float(h[j]);
      S.filt.g[w][j] = float(((j & 1) ? -1.0 : 1.0) * h[2 * N - 1 - j]);
    }
  }
  S.b = S.dirac + S.nw;
  S.tmp_stride = 0;
  for (int l = 1; l < levels; ++l) {
    S.tmp_off[l] = S.tmp_stride;
    S.tmp_stride += size_t(n >> l) * (n >> l);
  }
  RI_TRY(dev_alloc(&S.tmp, size_t(S.nw) * S.tmp_stride));
  RI_TRY(dev_alloc(&S.coef_tmp, size_t(S.b) * n * n));
  RI_TRY(dev_alloc(&S.vec_tmp, size_t(n) * n));
  RI_TRY(dev_alloc(&S.dsum, SUMSQ_SCRATCH));
  if (S.nw > 0) {
    std::vector<float> f(size_t(S.nw) * FILT_STRIDE, 0.f);
    for (int w = 0; w < S.nw; ++w)
      for (int j = 0; j < MAX_TAPS; ++j) {
        f[size_t(w) * FILT_STRIDE + j] = S.filt.h[w][j];
        f[size_t(w) * FILT_STRIDE + MAX_TAPS + j] = S.filt.g[w][j];
      }
    RI_TRY(dev_alloc(&S.dfilt, f.size()));
    RI_TRY(dev_alloc(&S.dlen, size_t(S.nw)));
    RI_HIP(hipMemcpy(S.dfilt, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
    RI_HIP(hipMemcpy(S.dlen, S.filt.len, S.nw * sizeof(int), hipMemcpyHostToDevice));
  }
  return RI_OK;
}

}  // namespace

int psi_adj_apply(const Sara& S, const float* x, float* s, bool clip, float alpha, hipStream_t st,
                  const float* wts) {
  return analysis(S, x, s, clip, alpha, wts, st);
}

int psi_apply(const Sara& S, const float* s, float* x, hipStream_t st) {
  RI_TRY(synthesis_lower(S, s, st));
  return synthesis_top(S, s, x, st);
}

}  // namespace ri

using ri::fail;

extern "C" {

int ri_sara_create(ri_sara* out, int n, int levels, uint32_t bases, hipStream_t stream) {
  (void)stream;
  if (!out) return fail(RI_EINVAL, "out is NULL");
  *out = nullptr;
  ri_sara h = new (std::nothrow) ri_sara_s;
  if (!h) return fail(RI_ENOMEM, "host allocation failed");
  const int rc = ri::create_sara(h->s, n, levels, bases);
  if (rc != RI_OK) {
    ri::destroy_sara(h->s);
    delete h;
    return rc;
  }
  *out = h;
  return RI_OK;
}

void ri_sara_destroy(ri_sara sara) {
  if (!sara) return;
  ri::destroy_sara(sara->s);
  delete sara;
}

int ri_sara_bases(ri_sara sara, int* b) {
  if (!sara || !b) return fail(RI_EINVAL, "NULL argument");
  *b = sara->s.b;
  return RI_OK;
}

int ri_psi(ri_sara sara, const float* s, float* x, hipStream_t stream) {
  if (!sara || !s || !x) return fail(RI_EINVAL, "NULL argument");
  return ri::psi_apply(sara->s, s, x, stream);
}

int ri_psi_adj(ri_sara sara, const float* x, float* s, hipStream_t stream) {
  if (!sara || !s || !x) return fail(RI_EINVAL, "NULL argument");
  return ri::psi_adj_apply(sara->s, x, s, false, 0.f, stream);
}

int ri_psi_norm(ri_sara sara, float* x0, int max_it, double rtol, double* norm_host, int* iters_host,
                hipStream_t stream) {
  if (!sara || !x0 || !norm_host || max_it < 1) return fail(RI_EINVAL, "bad argument");
  ri::Sara& S = sara->s;
  const size_t N = size_t(S.n) * S.n;
  float* cur = x0;
  float* nxt = S.vec_tmp;
  double lam = 0.0, lam_prev = 0.0, sq = 0.0;
  int it;
  RI_TRY(ri::sumsq_f32(cur, N, S.dsum, stream));
  RI_TRY(ri::scale_by_rsqrt(cur, N, S.dsum, stream));
  for (it = 1; it <= max_it; ++it) {
    RI_TRY(ri::psi_adj_apply(S, cur, S.coef_tmp, false, 0.f, stream));
    RI_TRY(ri::psi_apply(S, S.coef_tmp, nxt, stream));
    RI_TRY(ri::sumsq_f32(nxt, N, S.dsum, stream));
    RI_HIP(hipMemcpyAsync(&sq, S.dsum, sizeof(double), hipMemcpyDeviceToHost, stream));
    RI_HIP(hipStreamSynchronize(stream));
    lam = std::sqrt(sq);
    RI_TRY(ri::scale_by_rsqrt(nxt, N, S.dsum, stream));
    std::swap(cur, nxt);
    if (lam == 0.0 || std::fabs(lam - lam_prev) <= rtol * lam) break;
    lam_prev = lam;
  }
  if (cur != x0) RI_HIP(hipMemcpyAsync(x0, cur, N * sizeof(float), hipMemcpyDeviceToDevice, stream));
  RI_HIP(hipStreamSynchronize(stream));
  *norm_host = std::sqrt(lam);
  if (iters_host) *iters_host = it > max_it ? max_it : it;
  return RI_OK;
}

}  // extern "C"
