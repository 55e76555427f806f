// Device part of plan creation: the visibilities' coordinates packed as (cell, 20-bit
// fraction) of the oversampled grid, and the stable sort of the visibilities by (block,
// grid tile, cell in the tile) with a radix sort.  The blocks of y stay contiguous (Eq. 8),
// and inside a block the order is the one the work items are cut from.
#include <cmath>
#include <hipcub/hipcub.hpp>

#include "plan.hpp"

namespace ri {
namespace {

// Key bits: cell in the tile (T^2 <= 4096) in [0, 12), tile (tiles per axis <= 256) in
// [12, 28), block (< 4096) in [28, 40).
constexpr int KEY_BITS = 40;

// kappa = u K / (2 pi) wrapped to [0, K), as cell << FRAC_BITS | round(fraction 2^FRAC_BITS)
// (a fraction that rounds to a whole cell carries into the next one).  Each operation is
// rounded on its own (no fused multiply-adds), as written.
__device__ uint32_t pack_coord(float u, double to_cells, int K) {
#pragma clang fp contract(off)
  const double kappa = double(u) * to_cells;
  const double Kd = double(K);
  const double w = kappa - Kd * floor(kappa / Kd);  // [0, K]
  long long cell = (long long)floor(w);
  long long f = llround((w - double(cell)) * double(1u << FRAC_BITS));
  if (f >= (1LL << FRAC_BITS)) {
    f = 0;
    cell += 1;
  }
  cell %= K;
  if (cell < 0) cell += K;
  return (uint32_t(cell) << FRAC_BITS) | uint32_t(f);
}

__global__ __launch_bounds__(256) void k_plan_keys(const float* __restrict__ uv, int64_t M,
                                                   const int64_t* __restrict__ off, int d, int K, int T, int tpa,
                                                   double to_cells, uint2* __restrict__ packed,
                                                   uint64_t* __restrict__ keys, int* __restrict__ idx) {
  for (int64_t m = int64_t(blockIdx.x) * 256 + threadIdx.x; m < M; m += int64_t(gridDim.x) * 256) {
    int lo = 0, hi = d;  // the block b with off[b] <= m < off[b + 1]
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (off[mid] <= m) lo = mid;
      else hi = mid;
    }
    const uint32_t cx = pack_coord(uv[2 * m], to_cells, K), cy = pack_coord(uv[2 * m + 1], to_cells, K);
    packed[m] = make_uint2(cx, cy);
    const uint32_t gx = cx >> FRAC_BITS, gy = cy >> FRAC_BITS;
    const uint64_t tile = uint64_t(gy / T) * tpa + gx / T, local = uint64_t(gy % T) * T + gx % T;
    keys[m] = (uint64_t(lo) << 28) | (tile << 12) | local;
    idx[m] = int(m);
  }
}

__global__ __launch_bounds__(256) void k_gather_coord(const uint2* __restrict__ packed,
                                                      const int64_t* __restrict__ order, int64_t M,
                                                      uint2* __restrict__ coord) {
  for (int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x; k < M; k += int64_t(gridDim.x) * 256)
    coord[k] = packed[order[k]];
}

unsigned grid_of(int64_t M) { return unsigned(std::min<int64_t>((M + 255) / 256, 16384)); }

}  // namespace

int plan_sort(const float* uv, int64_t M, const int64_t* off, int d, int K, int T, int tpa, uint2** packed,
              std::vector<uint64_t>& keys_sorted, std::vector<int>& idx_sorted, hipStream_t s) {
  if (d > (1 << 12) || int64_t(tpa) * tpa > (1 << 16) || T * T > (1 << 12))
    return fail(RI_EINVAL, "plan sort keys: d=%d, %d tiles, tile %d out of range", d, tpa * tpa, T);
  float* d_uv = nullptr;
  int64_t* d_off = nullptr;
  uint64_t *k_in = nullptr, *k_out = nullptr;
  int *v_in = nullptr, *v_out = nullptr;
  void* temp = nullptr;
  size_t temp_bytes = 0;
  *packed = nullptr;
  int rc = RI_OK;
  auto run = [&]() -> int {
    RI_TRY(dev_alloc(&d_uv, size_t(2 * M)));
    RI_TRY(dev_alloc(&d_off, size_t(d + 1)));
    RI_TRY(dev_alloc(packed, size_t(M)));
    RI_TRY(dev_alloc(&k_in, size_t(M)));
    RI_TRY(dev_alloc(&k_out, size_t(M)));
    RI_TRY(dev_alloc(&v_in, size_t(M)));
    RI_TRY(dev_alloc(&v_out, size_t(M)));
    RI_HIP(hipMemcpyAsync(d_uv, uv, size_t(2 * M) * sizeof(float), hipMemcpyHostToDevice, s));
    RI_HIP(hipMemcpyAsync(d_off, off, size_t(d + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_plan_keys, dim3(grid_of(M)), dim3(256), 0, s, d_uv, M, d_off, d, K, T, tpa,
                       double(K) / (2.0 * M_PI), *packed, k_in, v_in);
    RI_LAUNCH_CHECK();
    RI_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, k_in, k_out, v_in, v_out, int(M), 0, KEY_BITS,
                                              s));
    RI_HIP(hipMalloc(&temp, temp_bytes > 0 ? temp_bytes : 1));
    RI_HIP(hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, k_in, k_out, v_in, v_out, int(M), 0, KEY_BITS, s));
    keys_sorted.resize(size_t(M));
    idx_sorted.resize(size_t(M));
    RI_HIP(hipMemcpyAsync(keys_sorted.data(), k_out, size_t(M) * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    RI_HIP(hipMemcpyAsync(idx_sorted.data(), v_out, size_t(M) * sizeof(int), hipMemcpyDeviceToHost, s));
    RI_HIP(hipStreamSynchronize(s));
    return RI_OK;
  };
  rc = run();
  dev_free(d_uv);
  dev_free(d_off);
  dev_free(k_in);
  dev_free(k_out);
  dev_free(v_in);
  dev_free(v_out);
  if (temp) (void)hipFree(temp);
  if (rc != RI_OK) dev_free(*packed);
  return rc;
}

int plan_gather_coord(const uint2* packed, const int64_t* order, int64_t M, uint2* coord, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_coord, dim3(grid_of(M)), dim3(256), 0, s, packed, order, M, coord);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

}  // namespace ri
