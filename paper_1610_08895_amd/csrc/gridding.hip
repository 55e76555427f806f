// Interpolation G_i (degridding) and its adjoint G_i^dagger (gridding) over sorted
// visibilities, with the per-block work of Algorithm 1 fused in:
//
//   degrid_residual  steps 5 and 8 (first half): e = G_i b_i - y_i, r = v_i + e, and the
//                    FP64 block sums ||r_i||^2 (for the projection, Eq. 10) and ||e||^2
//                    (for Eq. 13).
//   grid_project     steps 8 (second half), 9 and 11: v_i <- r max(0, 1 - eps_i / ||r_i||)
//                    (the Moreau form of v + Gb - P_B(v + Gb)), and the change
//                    G_i^dagger (v_new - v_old) added into the running grid sum
//                    sum_i M_i^dagger v~_i.  Blocks outside A are not visited, so their v_i
//                    and v~_i stay as they are.
//
// Visibilities are sorted by (block, tile, cell).  A work item covers up to `bin`
// visibilities of one block in one T x T grid tile; its workgroup stages the tile plus
// the kernel's reach (3 cells before, 4 after, per axis) in LDS, so every one of the 64
// taps of a visibility is an LDS access.  Gridding accumulates into the LDS tile with
// LDS float atomics and flushes the nonzero cells with global float atomics.  Kernels
// are persistent: a fixed grid of workgroups walks the active item list, which lives in
// device memory so a captured graph replays with whatever mask is current.
#include "plan.hpp"

namespace ri {

namespace {

constexpr int GT = 256;  // threads per workgroup

__device__ __forceinline__ void kb_weights(unsigned packed, const KBPoly& P, float* w, int& cell) {
  cell = int(packed >> FRAC_BITS);
  const float f = float(packed & FRAC_MASK) * (1.0f / float(1u << FRAC_BITS));
  const float x = 2.0f * f - 1.0f;
  const float x2 = x * x;
#pragma unroll
  for (int j = 0; j < KB_J / 2; ++j) {
    float e = P.e[j][KB_HALF_DEG], o = P.o[j][KB_HALF_DEG];
#pragma unroll
    for (int k = KB_HALF_DEG - 1; k >= 0; --k) {
      e = fmaf(e, x2, P.e[j][k]);
      o = fmaf(o, x2, P.o[j][k]);
    }
    w[j] = fmaf(x, o, e);
    w[KB_J - 1 - j] = fmaf(-x, o, e);
  }
}

struct ItemSource {
  const Item* items;
  const int* list;   // active item list, or nullptr for a contiguous range
  const int* count;  // device count of `list`
  int base, count_host;
  __device__ __forceinline__ int n() const { return list ? *count : count_host; }
  __device__ __forceinline__ Item get(int a) const { return items[list ? list[a] : base + a]; }
};

enum { DG_APPLY = 0, DG_RESIDUAL = 1 };

template <int T, int MODE>
__global__ __launch_bounds__(GT) void k_degrid(ItemSource src, const uint2* __restrict__ coord,
                                               const float2* __restrict__ grid, int K, int tpa, KBPoly P,
                                               float2* __restrict__ out, const float2* __restrict__ y,
                                               const float2* __restrict__ v, double* __restrict__ stats) {
  constexpr int TW = T + 8;
  __shared__ float2 tile[TW * TW];
  __shared__ double red[2][GT / 64];
  const int nitems = src.n();
  for (int a = blockIdx.x; a < nitems; a += gridDim.x) {
    const Item it = src.get(a);
    const int ty = it.y / tpa, tx = it.y - (it.y / tpa) * tpa;
    const int gy0 = ty * T - (KB_J / 2 - 1), gx0 = tx * T - (KB_J / 2 - 1);
    for (int idx = threadIdx.x; idx < TW * TW; idx += GT) {
      const int ly = idx / TW, lx = idx - ly * TW;
      const int gy = (gy0 + ly) & (K - 1), gx = (gx0 + lx) & (K - 1);
      tile[idx] = grid[size_t(gy) * K + gx];
    }
    __syncthreads();
    double sr = 0.0, se = 0.0;
    const int end = it.z + it.w;
    for (int m = it.z + threadIdx.x; m < end; m += GT) {
      const uint2 c = coord[m];
      float wx[KB_J], wy[KB_J];
      int cx, cy;
      kb_weights(c.x, P, wx, cx);
      kb_weights(c.y, P, wy, cy);
      const float2* base = &tile[(cy - ty * T) * TW + (cx - tx * T)];
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int ra = 0; ra < KB_J; ++ra) {
        const float2* row = base + ra * TW;
        float2 rs = make_float2(0.f, 0.f);
#pragma unroll
        for (int b = 0; b < KB_J; ++b) {
          const float2 g = row[b];
          rs.x = fmaf(wx[b], g.x, rs.x);
          rs.y = fmaf(wx[b], g.y, rs.y);
        }
        acc.x = fmaf(wy[ra], rs.x, acc.x);
        acc.y = fmaf(wy[ra], rs.y, acc.y);
      }
      if (MODE == DG_APPLY) {
        out[m] = acc;
      } else {
        const float2 yy = y[m], vv = v[m];
        const float2 e = make_float2(acc.x - yy.x, acc.y - yy.y);
        const float2 r = make_float2(vv.x + e.x, vv.y + e.y);
        out[m] = e;
        sr += double(r.x) * r.x + double(r.y) * r.y;
        se += double(e.x) * e.x + double(e.y) * e.y;
      }
    }
    if (MODE == DG_RESIDUAL) {
      sr = wave_sum(sr);
      se = wave_sum(se);
      const int wv = threadIdx.x / 64;
      if ((threadIdx.x & 63) == 0) {
        red[0][wv] = sr;
        red[1][wv] = se;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int k = 0; k < GT / 64; ++k) {
          a0 += red[0][k];
          a1 += red[1][k];
        }
        unsafeAtomicAdd(&stats[2 * it.x], a0);
        unsafeAtomicAdd(&stats[2 * it.x + 1], a1);
      }
    }
    __syncthreads();
  }
}

enum { GR_APPLY = 0, GR_PROJECT = 1 };

template <int T, int MODE>
__global__ __launch_bounds__(GT) void k_grid(ItemSource src, const uint2* __restrict__ coord,
                                             float2* __restrict__ grid, int K, int tpa, KBPoly P,
                                             const float2* __restrict__ y, const float2* __restrict__ e,
                                             float2* __restrict__ v, const double* __restrict__ stats,
                                             const double* __restrict__ eps) {
  constexpr int TW = T + 8;
  __shared__ float acc[2][TW * TW];
  const int nitems = src.n();
  for (int a = blockIdx.x; a < nitems; a += gridDim.x) {
    const Item it = src.get(a);
    const int ty = it.y / tpa, tx = it.y - (it.y / tpa) * tpa;
    for (int idx = threadIdx.x; idx < TW * TW; idx += GT) {
      acc[0][idx] = 0.f;
      acc[1][idx] = 0.f;
    }
    float shrink = 0.f;
    if (MODE == GR_PROJECT) {
      const double nr2 = stats[2 * it.x], ep = eps[it.x];
      shrink = nr2 > ep * ep ? float(1.0 - ep / sqrt(nr2)) : 0.f;
    }
    __syncthreads();
    const int end = it.z + it.w;
    for (int m = it.z + threadIdx.x; m < end; m += GT) {
      float2 val;
      if (MODE == GR_APPLY) {
        val = y[m];
      } else {
        const float2 vo = v[m], ee = e[m];
        const float2 vn = make_float2((vo.x + ee.x) * shrink, (vo.y + ee.y) * shrink);
        v[m] = vn;
        val = make_float2(vn.x - vo.x, vn.y - vo.y);
      }
      const uint2 c = coord[m];
      float wx[KB_J], wy[KB_J];
      int cx, cy;
      kb_weights(c.x, P, wx, cx);
      kb_weights(c.y, P, wy, cy);
      const int b0 = (cy - ty * T) * TW + (cx - tx * T);
#pragma unroll
      for (int ra = 0; ra < KB_J; ++ra) {
        const float tr = wy[ra] * val.x, ti = wy[ra] * val.y;
#pragma unroll
        for (int b = 0; b < KB_J; ++b) {
          atomicAdd(&acc[0][b0 + ra * TW + b], wx[b] * tr);
          atomicAdd(&acc[1][b0 + ra * TW + b], wx[b] * ti);
        }
      }
    }
    __syncthreads();
    const int gy0 = ty * T - (KB_J / 2 - 1), gx0 = tx * T - (KB_J / 2 - 1);
    for (int idx = threadIdx.x; idx < TW * TW; idx += GT) {
      const float re = acc[0][idx], im = acc[1][idx];
      if (re != 0.f || im != 0.f) {
        const int ly = idx / TW, lx = idx - ly * TW;
        const int gy = (gy0 + ly) & (K - 1), gx = (gx0 + lx) & (K - 1);
        float* g = reinterpret_cast<float*>(&grid[size_t(gy) * K + gx]);
        unsafeAtomicAdd(g, re);
        unsafeAtomicAdd(g + 1, im);
      }
    }
    __syncthreads();
  }
}

__global__ void k_build_active(const uint8_t* __restrict__ mask, int d, const int* __restrict__ item_off,
                               int* __restrict__ list, int* __restrict__ count, double* __restrict__ stats) {
  int pos = 0;
  for (int i = 0; i < d; ++i) {
    if (mask == nullptr || mask[i] != 0) {
      const int a = item_off[i], b = item_off[i + 1];
      for (int t = threadIdx.x; t < b - a; t += blockDim.x) list[pos + t] = a + t;
      pos += b - a;
      if (stats != nullptr && threadIdx.x == 0) {
        stats[2 * i] = 0.0;
        stats[2 * i + 1] = 0.0;
      }
    }
  }
  if (threadIdx.x == 0) *count = pos;
}

__global__ __launch_bounds__(GT) void k_block_sumsq(ItemSource src, const float2* __restrict__ y,
                                                    double* __restrict__ out) {
  __shared__ double red[GT / 64];
  const int nitems = src.n();
  for (int a = blockIdx.x; a < nitems; a += gridDim.x) {
    const Item it = src.get(a);
    double acc = 0.0;
    for (int m = it.z + threadIdx.x; m < it.z + it.w; m += GT) {
      const float2 v = y[m];
      acc += double(v.x) * v.x + double(v.y) * v.y;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int k = 0; k < GT / 64; ++k) t += red[k];
      unsafeAtomicAdd(&out[it.x], t);
    }
    __syncthreads();
  }
}

int wgs_for(const Plan& p, int items) {
  int g = p.persistent_wgs > 0 ? p.persistent_wgs : device_cus() * 8;
  return items < g ? (items > 0 ? items : 1) : g;
}

#define RI_TILE_DISPATCH(KERNEL, ...)                                                          \
  switch (p.tile) {                                                                            \
    case 16: hipLaunchKernelGGL((KERNEL<16, __VA_ARGS__>), grid_dim, dim3(GT), 0, s, ARGS); break; \
    case 32: hipLaunchKernelGGL((KERNEL<32, __VA_ARGS__>), grid_dim, dim3(GT), 0, s, ARGS); break; \
    case 64: hipLaunchKernelGGL((KERNEL<64, __VA_ARGS__>), grid_dim, dim3(GT), 0, s, ARGS); break; \
    default: return fail(RI_EINVAL, "unsupported tile %d", p.tile);                            \
  }

}  // namespace

int build_active(const Plan& p, const uint8_t* mask, double* stats_zero, hipStream_t s) {
  hipLaunchKernelGGL(k_build_active, dim3(1), dim3(256), 0, s, mask, p.d, p.item_off, p.active_list,
                     p.active_count, stats_zero);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

int block_sumsq(const Plan& p, const float2* y, double* out, hipStream_t s) {
  ItemSource src{p.items, nullptr, nullptr, 0, p.n_items};
  RI_TRY(zero_f32(reinterpret_cast<float*>(out), 2 * size_t(p.d), s));
  hipLaunchKernelGGL(k_block_sumsq, dim3(wgs_for(p, p.n_items)), dim3(GT), 0, s, src, y, out);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

int degrid_apply(const Plan& p, const float2* grid, float2* y, hipStream_t s) {
  ItemSource src{p.items, p.active_list, p.active_count, 0, 0};
  const dim3 grid_dim(wgs_for(p, p.n_items));
#define ARGS src, p.coord, grid, p.K, p.tpa, p.poly, y, (const float2*)nullptr, (const float2*)nullptr, (double*)nullptr
  RI_TILE_DISPATCH(k_degrid, DG_APPLY)
#undef ARGS
  RI_LAUNCH_CHECK();
  return RI_OK;
}

int degrid_residual(const Plan& p, const float2* grid, const float2* y, const float2* v, float2* e,
                    double* stats, const int* list, const int* count, int base, int count_host,
                    hipStream_t s) {
  ItemSource src{p.items, list, count, base, count_host};
  const dim3 grid_dim(wgs_for(p, list ? p.n_items : count_host));
#define ARGS src, p.coord, grid, p.K, p.tpa, p.poly, e, y, v, stats
  RI_TILE_DISPATCH(k_degrid, DG_RESIDUAL)
#undef ARGS
  RI_LAUNCH_CHECK();
  return RI_OK;
}

int grid_apply(const Plan& p, const float2* y, float2* grid, hipStream_t s) {
  ItemSource src{p.items, p.active_list, p.active_count, 0, 0};
  const dim3 grid_dim(wgs_for(p, p.n_items));
#define ARGS src, p.coord, grid, p.K, p.tpa, p.poly, y, (const float2*)nullptr, (float2*)nullptr, \
             (const double*)nullptr, (const double*)nullptr
  RI_TILE_DISPATCH(k_grid, GR_APPLY)
#undef ARGS
  RI_LAUNCH_CHECK();
  return RI_OK;
}

int grid_all(const Plan& p, const float2* v, float2* grid, hipStream_t s) {
  ItemSource src{p.items, nullptr, nullptr, 0, p.n_items};
  const dim3 grid_dim(wgs_for(p, p.n_items));
#define ARGS src, p.coord, grid, p.K, p.tpa, p.poly, v, (const float2*)nullptr, (float2*)nullptr, \
             (const double*)nullptr, (const double*)nullptr
  RI_TILE_DISPATCH(k_grid, GR_APPLY)
#undef ARGS
  RI_LAUNCH_CHECK();
  return RI_OK;
}

int grid_project(const Plan& p, const float2* e, float2* v, const double* stats, const double* eps,
                 float2* grid, const int* list, const int* count, int base, int count_host,
                 hipStream_t s) {
  ItemSource src{p.items, list, count, base, count_host};
  const dim3 grid_dim(wgs_for(p, list ? p.n_items : count_host));
#define ARGS src, p.coord, grid, p.K, p.tpa, p.poly, (const float2*)nullptr, e, v, stats, eps
  RI_TILE_DISPATCH(k_grid, GR_PROJECT)
#undef ARGS
  RI_LAUNCH_CHECK();
  return RI_OK;
}

}  // namespace ri
