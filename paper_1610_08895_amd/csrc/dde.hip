// Direction-dependent effects in the interpolation G (Eq. 1's D(l, u), folded into G's
// kernels as Sec. II describes): the DDE of visibility m is band limited on the
// oversampled grid, D_m(l) = sum_{p,q} d_m[q, p] exp(-2 pi i (p l_x + q l_y) / K), so its
// row of G is the jd x jd kernel d_m convolved with the Kaiser-Bessel kernel (the plain
// kernel at a frequency shifted by (p, q) whole cells is the same 8 weights on shifted
// cells):
//
//   W_m[ty][tx] = sum_{p,q} d_m[q, p] w_y[ty - h - q] w_x[tx - h - p],   0 <= tx, ty < S,
//
// on the S = J + 2h cells per axis starting at floor(kappa) - J/2 + 1 - h.  The weights are
// built once per plan (k_dde_weights) and stored tap-major, w[t * M + m], so the 64 lanes of
// a wavefront, which take 64 consecutive visibilities, read 512 contiguous bytes per tap:
// with S^2 complex weights per visibility (1152 bytes at S = 12) against 24 bytes of
// coordinates and data, these operators are bound by streaming the weights from HBM.
//
// Degridding stages a tile plus the kernel's reach in LDS, as the plain kernel does, and
// forms y_m = sum_t W_m[t] b[cell_m + t].  Gridding (the adjoint, conjugate weights) is
// owner-computes per tile: one workgroup accumulates every active item of its tile exactly
// in fixed point with 64-bit LDS integer atomics (per item a power-of-two scale from the
// bound sum_m max_t(|Re W| + |Im W|) (|Re v| + |Im v|)), folds each item into FP32
// registers, and writes the tile's whole region (tile plus reach) to a per-tile patch; a
// merge pass then adds, for every grid cell, the patches of the up to nine tiles whose
// regions cover it, in a fixed order.  Results are deterministic.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "handles.hpp"

namespace ri {
namespace {

constexpr int DT = 256;                 // threads per workgroup
constexpr int DNV = MAX_BIN / DT;       // visibilities per thread per item
constexpr int MAX_H = 3;                // jd <= 7

template <int T, int H>
struct DdeGeom {
  static constexpr int S = KB_J + 2 * H;      // taps per axis
  static constexpr int R0 = KB_J / 2 - 1 + H;  // reach before the tile
  static constexpr int TW = T + S - 1;         // region: tile plus reach
  static constexpr int TP = TW + 1;            // LDS pitch
};

// One thread per visibility: W = d * (w_y (x) w_x) by separable convolution, and its bound.
template <int H>
__global__ __launch_bounds__(DT) void k_dde_weights(int64_t M, const uint2* __restrict__ coord,
                                                    const float2* __restrict__ d, KBPoly P,
                                                    float2* __restrict__ w, float* __restrict__ wmax) {
  constexpr int JD = 2 * H + 1, S = KB_J + 2 * H;
  for (int64_t m = blockIdx.x * int64_t(DT) + threadIdx.x; m < M; m += int64_t(gridDim.x) * DT) {
    float wx[KB_J], wy[KB_J];
    int cx, cy;
    kb_weights(coord[m].x, P, wx, cx);
    kb_weights(coord[m].y, P, wy, cy);
    const float2* dm = d + m * JD * JD;
    float mx = 0.f;
    // every loop has a compile-time trip count and is unrolled, so all register indices are
    // constants: W[ty][tx] = sum_{q,p} d[q][p] w_y[ty - q] w_x[tx - p] (shifts q - H, p - H)
#pragma unroll
    for (int ty = 0; ty < S; ++ty) {
      float2 row[S];
#pragma unroll
      for (int tx = 0; tx < S; ++tx) row[tx] = make_float2(0.f, 0.f);
#pragma unroll
      for (int q = 0; q < JD; ++q) {
        const int jy = ty - q;  // the Kaiser-Bessel row of this term
        if (jy < 0 || jy >= KB_J) continue;
        const float a = wy[jy];
#pragma unroll
        for (int pp = 0; pp < JD; ++pp) {
          const float2 dq = dm[q * JD + pp];
          const float2 c = make_float2(a * dq.x, a * dq.y);
#pragma unroll
          for (int jx = 0; jx < KB_J; ++jx) {
            const int tx = jx + pp;  // < S
            row[tx].x = fmaf(c.x, wx[jx], row[tx].x);
            row[tx].y = fmaf(c.y, wx[jx], row[tx].y);
          }
        }
      }
#pragma unroll
      for (int tx = 0; tx < S; ++tx) {
        w[size_t(ty * S + tx) * M + m] = row[tx];
        mx = fmaxf(mx, fabsf(row[tx].x) + fabsf(row[tx].y));
      }
    }
    wmax[m] = mx;
  }
}

enum { DD_APPLY = 0, DD_RESIDUAL = 1 };

// Degridding over units {tile, first, end} of items; MODE as k_degrid in gridding.hip
// (residual: r = v + G b - y into out and FP64 partial norms of r and of G b - y per wavefront).
template <int T, int H, int MODE>
__global__ __launch_bounds__(DT) void k_degrid_dde(const int4* __restrict__ units, int nunits,
                                                   const Item* __restrict__ items, const uint8_t* __restrict__ mask,
                                                   const uint2* __restrict__ coord, const float2* __restrict__ w,
                                                   int64_t M, const float2* __restrict__ grid, int K, int tpa,
                                                   float2* __restrict__ out, const float2* __restrict__ y,
                                                   const float2* __restrict__ v, double* __restrict__ part) {
  using G = DdeGeom<T, H>;
  constexpr int S = G::S, TW = G::TW, TP = G::TP, R0 = G::R0;
  constexpr int NWV = DT / 64;
  __shared__ float2 tile[TW * TP];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
    const int4 un = units[u];
    bool any = mask == nullptr && un.y < un.z;  // empty units fill gaps of the XCD order
    for (int q = un.y; q < un.z && !any; ++q) any = mask[items[q].x] != 0;
    if (!any) continue;
    const int ty = un.x / tpa, tx = un.x - (un.x / tpa) * tpa;
    const int gy0 = ty * T - R0, gx0 = tx * T - R0;
    for (int idx = threadIdx.x; idx < TW * TW; idx += DT) {
      const int ly = idx / TW, lx = idx - ly * TW;
      tile[ly * TP + lx] = grid[size_t((gy0 + ly) & (K - 1)) * K + ((gx0 + lx) & (K - 1))];
    }
    __syncthreads();
    for (int q = un.y; q < un.z; ++q) {
      const Item it = items[q];
      if (mask != nullptr && mask[it.x] == 0) continue;
      double sr = 0.0, se = 0.0;
      for (int k = 0; k < DNV; ++k) {
        const int s = threadIdx.x + k * DT;
        if (s >= it.w) break;
        const int64_t m = it.z + s;
        const uint2 c = coord[m];
        // region row / column of the first tap: cell - 3 - h - (tile origin - R0)
        const int ly0 = int(c.y >> FRAC_BITS) - ty * T, lx0 = int(c.x >> FRAC_BITS) - tx * T;
        const float2* base = &tile[ly0 * TP + lx0];
        const float2* wm = w + m;
        float2 acc = make_float2(0.f, 0.f);
        for (int a = 0; a < S; ++a) {
          float2 wr[S];
#pragma unroll
          for (int b = 0; b < S; ++b) wr[b] = wm[size_t(a * S + b) * M];
#pragma unroll
          for (int b = 0; b < S; ++b) {
            const float2 g = base[a * TP + b];
            acc.x = fmaf(wr[b].x, g.x, fmaf(-wr[b].y, g.y, acc.x));
            acc.y = fmaf(wr[b].x, g.y, fmaf(wr[b].y, g.x, acc.y));
          }
        }
        if (MODE == DD_APPLY) {
          out[m] = acc;
        } else {
          const float2 yy = y[m], vv = v[m];
          const float2 e = make_float2(acc.x - yy.x, acc.y - yy.y);
          const float2 r = make_float2(vv.x + e.x, vv.y + e.y);
          if (out != nullptr) out[m] = r;
          sr += double(r.x) * r.x + double(r.y) * r.y;
          se += double(e.x) * e.x + double(e.y) * e.y;
        }
      }
      if (MODE == DD_RESIDUAL) {
        sr = wave_sum(sr);
        se = wave_sum(se);
        if (lane == 0) {
          part[(size_t(it.y) * NWV + wv) * 2] = sr;
          part[(size_t(it.y) * NWV + wv) * 2 + 1] = se;
        }
      }
    }
    __syncthreads();
  }
}

// Gridding with conjugate DDE weights over whole-tile units.  PROJECT: the values are the
// step-8 dual changes (v_new = r shrink_i stored, v_new - v_old gridded), else y.
// The tile's region goes to its patch (stored, or added with ADDP).
template <int T, int H, bool PROJECT, bool ADDP>
__global__ __launch_bounds__(DT) void k_grid_dde(const int4* __restrict__ units, int nunits,
                                                 const Item* __restrict__ items, const uint8_t* __restrict__ mask,
                                                 const uint2* __restrict__ coord, const float2* __restrict__ w,
                                                 const float* __restrict__ wmax, int64_t M,
                                                 const float2* __restrict__ y, const float2* __restrict__ e,
                                                 float2* __restrict__ v, const float* __restrict__ shrink,
                                                 float2* __restrict__ patch, int tpa) {
  using G = DdeGeom<T, H>;
  constexpr int S = G::S, TW = G::TW, TP = G::TP;
  constexpr int NWV = DT / 64;
  constexpr int NC = (TW * TW + DT - 1) / DT;
  __shared__ unsigned long long acci[TW * TP];
  __shared__ float red[NWV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k = threadIdx.x; k < TW * TP; k += DT) acci[k] = 0ull;
  __syncthreads();
  for (int u = blockIdx.x; u < nunits; u += gridDim.x) {
    const int4 un = units[u];
    const int ty = un.x / tpa, tx = un.x - (un.x / tpa) * tpa;
    float2 acc[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[j] = make_float2(0.f, 0.f);
    for (int q = un.y; q < un.z; ++q) {
      const Item it = items[q];
      if (mask != nullptr && mask[it.x] == 0) continue;
      float2 val[DNV];
      float babs = 0.f;
#pragma unroll
      for (int k = 0; k < DNV; ++k) {
        const int s = threadIdx.x + k * DT;
        val[k] = make_float2(0.f, 0.f);
        if (s < it.w) {
          const int64_t m = it.z + s;
          if (PROJECT) {
            const float sh = shrink[it.x];
            const float2 vo = v[m], rr = e[m];  // r = v_old + G b - y from the degridding
            const float2 vn = make_float2(rr.x * sh, rr.y * sh);
            v[m] = vn;
            val[k] = make_float2(vn.x - vo.x, vn.y - vo.y);
          } else {
            val[k] = y[m];
          }
          babs += wmax[m] * (fabsf(val[k].x) + fabsf(val[k].y));
        }
      }
      babs = wave_sum(babs);
      if (lane == 0) red[wv] = babs;
      __syncthreads();
      float bound = 0.f;
#pragma unroll
      for (int k = 0; k < NWV; ++k) bound += red[k];
      if (bound > 0.f) {
        // 2^E with bound * 2^E <= 2^30: no cell's sum of either part can leave 31 bits
        int ex = 0;
        frexpf(bound * 1.0001f, &ex);
        const float scale = ldexpf(1.f, 30 - ex);
#pragma unroll
        for (int k = 0; k < DNV; ++k) {
          const int s = threadIdx.x + k * DT;
          if (s >= it.w) continue;
          const int64_t m = it.z + s;
          const uint2 c = coord[m];
          const int ly0 = int(c.y >> FRAC_BITS) - ty * T, lx0 = int(c.x >> FRAC_BITS) - tx * T;
          unsigned long long* base = &acci[ly0 * TP + lx0];
          const float vr = val[k].x * scale, vi = val[k].y * scale;
          const float2* wm = w + m;
          for (int a = 0; a < S; ++a) {
            float2 wr[S];
#pragma unroll
            for (int b = 0; b < S; ++b) wr[b] = wm[size_t(a * S + b) * M];
#pragma unroll
            for (int b = 0; b < S; ++b) {
              // conj(W) v = (Wr Vr + Wi Vi) + i (Wr Vi - Wi Vr), rounded to nearest
              const long long ir = static_cast<int>(floorf(fmaf(wr[b].x, vr, fmaf(wr[b].y, vi, 0.5f))));
              const long long ii = static_cast<int>(floorf(fmaf(wr[b].x, vi, fmaf(-wr[b].y, vr, 0.5f))));
              atomicAdd(base + a * TP + b, static_cast<unsigned long long>(ii * 4294967296LL + ir));
            }
          }
        }
        __syncthreads();
        const float inv = ldexpf(1.f, ex - 30);
#pragma unroll
        for (int j = 0; j < NC; ++j) {
          const int c = threadIdx.x + j * DT;
          if (c < TW * TW) {
            unsigned long long* cell = &acci[c + c / TW];
            const unsigned long long w64 = *cell;
            if (w64) {
              *cell = 0ull;
              const int ir = static_cast<int>(static_cast<unsigned>(w64));
              const int ii = static_cast<int>(static_cast<unsigned>(
                  (w64 - static_cast<unsigned long long>(static_cast<long long>(ir))) >> 32));
              acc[j].x += float(ir) * inv;
              acc[j].y += float(ii) * inv;
            }
          }
        }
      }
      __syncthreads();
    }
    float2* pt = patch + size_t(un.x) * TW * TW;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const int c = threadIdx.x + j * DT;
      if (c >= TW * TW) continue;
      if (ADDP) {
        if (acc[j].x != 0.f || acc[j].y != 0.f) {
          const float2 o = pt[c];
          pt[c] = make_float2(o.x + acc[j].x, o.y + acc[j].y);
        }
      } else {
        pt[c] = acc[j];
      }
    }
  }
}

// grid cell (=, or += with ADD) the sum of the patches of the tiles whose regions cover
// it, neighbours in a fixed order; one workgroup per tile.
template <int T, int H, bool ADD>
__global__ __launch_bounds__(DT) void k_dde_merge(float2* __restrict__ grid, const float2* __restrict__ patch,
                                                  const uint8_t* __restrict__ tile_has, int K, int tpa) {
  using G = DdeGeom<T, H>;
  constexpr int TW = G::TW, R0 = G::R0;
  static_assert(TW - R0 <= 2 * T && R0 <= T, "a region reaches into the neighbouring tiles only");
  const int t = blockIdx.x;
  const int ty = t / tpa, tx = t - (t / tpa) * tpa;
  for (int k = threadIdx.x; k < T * T; k += DT) {
    const int iy = k / T, ix = k - (k / T) * T;
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int ly = iy - dy * T + R0, lx = ix - dx * T + R0;
        if (ly < 0 || ly >= TW || lx < 0 || lx >= TW) continue;
        const int nt = ((ty + dy + tpa) & (tpa - 1)) * tpa + ((tx + dx + tpa) & (tpa - 1));
        if (!tile_has[nt]) continue;
        const float2 h = patch[size_t(nt) * TW * TW + ly * TW + lx];
        acc.x += h.x;
        acc.y += h.y;
      }
    float2* g = &grid[size_t(ty * T + iy) * K + tx * T + ix];
    if (!ADD) {
      *g = acc;
    } else if (acc.x != 0.f || acc.y != 0.f) {
      const float2 o = *g;
      *g = make_float2(o.x + acc.x, o.y + acc.y);
    }
  }
}

int wgs(const Plan& p, int units) {
  const int g = p.persistent_wgs > 0 ? p.persistent_wgs : units;
  return units < g ? (units > 0 ? units : 1) : g;
}

// Calls F.template operator()<T, H>() for the plan's tile and DDE half-width.
template <class F>
int dispatch(const Plan& p, F&& f) {
#define RI_DDE_H(TT)                                                 \
  switch (p.dde.h) {                                                 \
    case 0: return f.template operator()<TT, 0>();                   \
    case 1: return f.template operator()<TT, 1>();                   \
    case 2: return f.template operator()<TT, 2>();                   \
    case 3: return f.template operator()<TT, 3>();                   \
    default: return fail(RI_EINVAL, "unsupported DDE half-width %d", p.dde.h); \
  }
  switch (p.tile) {
    case 16: RI_DDE_H(16)
    case 32: RI_DDE_H(32)
    case 64: RI_DDE_H(64)
    default: return fail(RI_EINVAL, "unsupported tile %d", p.tile);
  }
#undef RI_DDE_H
}

size_t region_cells(const Plan& p) {
  const size_t tw = size_t(p.tile) + p.dde.S - 1;
  return tw * tw;
}

}  // namespace

void dde_destroy(Dde& dd) {
  dev_free(dd.w);
  dev_free(dd.wmax);
  dev_free(dd.tunits);
  dev_free(dd.patch);
  dev_free(dd.tile_has);
  dd = Dde{};
}

int dde_degrid(const Plan& p, const int4* units, int nunits, const Item* items, const uint8_t* mask,
               const float2* grid, float2* out, const float2* y, const float2* v, double* part, hipStream_t s) {
  if (nunits <= 0) return RI_OK;
  const bool resid = y != nullptr;
  return dispatch(p, [&]<int T, int H>() -> int {
    if (resid)
      hipLaunchKernelGGL((k_degrid_dde<T, H, DD_RESIDUAL>), dim3(wgs(p, nunits)), dim3(DT), 0, s, units, nunits,
                         items, mask, p.coord, p.dde.w, p.M, grid, p.K, p.tpa, out, y, v, part);
    else
      hipLaunchKernelGGL((k_degrid_dde<T, H, DD_APPLY>), dim3(wgs(p, nunits)), dim3(DT), 0, s, units, nunits, items,
                         mask, p.coord, p.dde.w, p.M, grid, p.K, p.tpa, out, y, v, part);
    RI_LAUNCH_CHECK();
    return RI_OK;
  });
}

int dde_grid(const Plan& p, const int4* units, int nunits, const Item* items, const uint8_t* mask, const float2* y,
             const float2* e, float2* v, const float* shrink, bool project, bool add_patch, hipStream_t s) {
  if (nunits <= 0) return RI_OK;
  return dispatch(p, [&]<int T, int H>() -> int {
    const dim3 g(wgs(p, nunits)), b(DT);
#define RI_GDDE(PR, AD)                                                                                        \
  hipLaunchKernelGGL((k_grid_dde<T, H, PR, AD>), g, b, 0, s, units, nunits, items, mask, p.coord, p.dde.w,        \
                     p.dde.wmax, p.M, y, e, v, shrink, p.dde.patch, p.tpa)
    if (project && add_patch) RI_GDDE(true, true);
    else if (project) RI_GDDE(true, false);
    else if (add_patch) RI_GDDE(false, true);
    else RI_GDDE(false, false);
#undef RI_GDDE
    RI_LAUNCH_CHECK();
    return RI_OK;
  });
}

int dde_merge(const Plan& p, float2* grid, bool add, hipStream_t s) {
  return dispatch(p, [&]<int T, int H>() -> int {
    if (add)
      hipLaunchKernelGGL((k_dde_merge<T, H, true>), dim3(p.n_tiles), dim3(DT), 0, s, grid, p.dde.patch,
                         p.dde.tile_has, p.K, p.tpa);
    else
      hipLaunchKernelGGL((k_dde_merge<T, H, false>), dim3(p.n_tiles), dim3(DT), 0, s, grid, p.dde.patch,
                         p.dde.tile_has, p.K, p.tpa);
    RI_LAUNCH_CHECK();
    return RI_OK;
  });
}

int dde_zero_patches(const Plan& p, hipStream_t s) {
  return zero_c64(p.dde.patch, size_t(p.n_tiles) * region_cells(p), s);
}

}  // namespace ri

using ri::fail;

extern "C" int ri_plan_dde(ri_plan plan, int jd, const float* d_host, hipStream_t stream) {
  if (!plan) return fail(RI_EINVAL, "plan is NULL");
  ri::Plan& p = plan->p;
  if (jd == 0 || d_host == nullptr) {
    if (jd != 0 || d_host != nullptr) return fail(RI_EINVAL, "removing DDEs takes jd = 0 and d = NULL");
    RI_HIP(hipStreamSynchronize(stream));
    ri::dde_destroy(p.dde);
    return RI_OK;
  }
  if (jd < 1 || jd % 2 == 0 || jd > 2 * ri::MAX_H + 1)
    return fail(RI_EINVAL, "jd = %d must be odd, 1 <= jd <= %d", jd, 2 * ri::MAX_H + 1);
  const int jd2 = jd * jd;
  for (int64_t k = 0; k < 2 * p.M * jd2; ++k)
    if (!std::isfinite(d_host[k])) return fail(RI_EINVAL, "non-finite DDE tap at visibility %lld", (long long)(k / (2 * jd2)));
  RI_HIP(hipStreamSynchronize(stream));
  ri::dde_destroy(p.dde);
  ri::Dde& dd = p.dde;
  const int h = jd / 2;
  dd.h = h;
  dd.S = ri::KB_J + 2 * h;
  int rc = RI_OK;
  float2* d_dev = nullptr;
  try {
    // taps into plan order on the host
    std::vector<float2> dp(size_t(p.M) * jd2);
    const float2* du = reinterpret_cast<const float2*>(d_host);
    for (int64_t k = 0; k < p.M; ++k)
      std::copy(du + size_t(p.order_host[k]) * jd2, du + size_t(p.order_host[k] + 1) * jd2, dp.begin() + k * jd2);
    std::vector<uint8_t> has(p.n_tiles, 0);
    for (const int4& u : p.tile_units_host) has[u.x] = 1;
    const size_t S2 = size_t(dd.S) * dd.S;
    if (rc == RI_OK) rc = ri::dev_alloc(&d_dev, dp.size());
    if (rc == RI_OK) rc = ri::dev_alloc(&dd.w, S2 * p.M);
    if (rc == RI_OK) rc = ri::dev_alloc(&dd.wmax, size_t(p.M));
    if (rc == RI_OK) rc = ri::dev_alloc(&dd.tunits, p.tile_units_host.size());
    if (rc == RI_OK) rc = ri::dev_alloc(&dd.tile_has, size_t(p.n_tiles));
    if (rc == RI_OK) rc = ri::dev_alloc(&dd.patch, size_t(p.n_tiles) * ri::region_cells(p));
    if (rc == RI_OK) {
      dd.n_tunits = int(p.tile_units_host.size());
      if (hipMemcpyAsync(d_dev, dp.data(), dp.size() * sizeof(float2), hipMemcpyHostToDevice, stream) != hipSuccess ||
          hipMemcpyAsync(dd.tunits, p.tile_units_host.data(), dd.n_tunits * sizeof(int4), hipMemcpyHostToDevice,
                         stream) != hipSuccess ||
          hipMemcpyAsync(dd.tile_has, has.data(), has.size(), hipMemcpyHostToDevice, stream) != hipSuccess)
        rc = fail(RI_EHIP, "copy of the DDE tables failed");
    }
    if (rc == RI_OK) rc = ri::dde_zero_patches(p, stream);
    if (rc == RI_OK) {
      const unsigned g = unsigned(std::min<int64_t>((p.M + ri::DT - 1) / ri::DT, 65536));
      switch (h) {
        case 0: hipLaunchKernelGGL(ri::k_dde_weights<0>, dim3(g), dim3(ri::DT), 0, stream, p.M, p.coord, d_dev, p.poly, dd.w, dd.wmax); break;
        case 1: hipLaunchKernelGGL(ri::k_dde_weights<1>, dim3(g), dim3(ri::DT), 0, stream, p.M, p.coord, d_dev, p.poly, dd.w, dd.wmax); break;
        case 2: hipLaunchKernelGGL(ri::k_dde_weights<2>, dim3(g), dim3(ri::DT), 0, stream, p.M, p.coord, d_dev, p.poly, dd.w, dd.wmax); break;
        default: hipLaunchKernelGGL(ri::k_dde_weights<3>, dim3(g), dim3(ri::DT), 0, stream, p.M, p.coord, d_dev, p.poly, dd.w, dd.wmax); break;
      }
      if (hipGetLastError() != hipSuccess) rc = fail(RI_EHIP, "DDE weight kernel launch failed");
    }
    if (rc == RI_OK && hipStreamSynchronize(stream) != hipSuccess) rc = fail(RI_EHIP, "stream sync failed");
  } catch (const std::bad_alloc&) {
    rc = fail(RI_ENOMEM, "host allocation failed");
  }
  ri::dev_free(d_dev);
  if (rc != RI_OK) ri::dde_destroy(dd);
  return rc;
}
