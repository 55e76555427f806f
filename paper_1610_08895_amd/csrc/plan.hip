// Measurement-operator plan and the Phi / Phi^dagger entry points (Eq. 3, Eq. 8).
//
// Plan creation:
//   * each u-v coordinate becomes kappa = u K / (2 pi) wrapped to [0, K), stored as a
//     12-bit cell plus a 20-bit fraction (position error <= 2^-21 cell, i.e. < 1e-6 rad of
//     phase at the image edge), in FP64 on the device (plan_sort.hip);
//   * the visibilities are sorted by (block, grid tile, cell) on the device, and inside each
//     block cut on the host into work items of at most `bin` visibilities of one tile;
//   * Kaiser-Bessel weights are fitted per tap by degree-7 polynomials (Chebyshev
//     interpolation of the kernel evaluated with an I0 power series);
//   * twiddles exp(-2 pi i k / K) and the pre-compensation S = 1/phi_hat(l/K) are
//     evaluated in FP64 and rounded to FP32.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "host_math.hpp"
#include "handles.hpp"

namespace ri {
namespace {

__global__ void k_permute(const float2* __restrict__ src, float2* __restrict__ dst,
                          const int64_t* __restrict__ order, int64_t M, int to_plan) {
  for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < M; k += int64_t(gridDim.x) * blockDim.x) {
    if (to_plan) dst[k] = src[order[k]];
    else dst[order[k]] = src[k];
  }
}

__global__ void k_copy_f32(const float* __restrict__ a, float* __restrict__ b, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    b[i] = a[i];
}

void destroy_plan(Plan& p) {
  dev_free(p.coord);
  dev_free(p.order);
  dev_free(p.items);
  dev_free(p.item_box);
  dev_free(p.item_pairs);
  dev_free(p.item_off);
  dev_free(p.block_off);
  dev_free(p.twiddle);
  dev_free(p.scale);
  dev_free(p.grid);
  dev_free(p.rowbuf);
  dev_free(p.titems);
  dev_free(p.units);
  dev_free(p.bunits);
  dev_free(p.dunits);
  dev_free(p.unit_patch);
  dev_free(p.tile_sp_off);
  dev_free(p.tile_sp);
  dev_free(p.spatch);
  dev_free(p.item_part);
  dev_free(p.block_tmp);
  dev_free(p.halo);
  dev_free(p.empty_tiles);
  dev_free(p.norm_tmp);
  dev_free(p.dsum);
  dde_destroy(p.dde);
}

using KV = std::pair<uint64_t, int64_t>;  // (tile << 32 | tile-local cell ly * T + lx, index)

// Reorders a list of visibilities (or of same-cell pairs, by their first member) so that
// every 64 consecutive ones, which one wavefront processes together, spread their
// staged-tile addresses ly * (T + TILE_PAD) + lx evenly over the LDS banks: they are dealt
// round-robin from one queue per bank (32 banks of 8-byte words).
template <class E, class Key>
void lds_bank_order(std::vector<E>& v, int T, Key key) {
  constexpr int NB = 32;
  std::vector<E> q[NB];
  for (const E& e : v) {
    const uint32_t local = uint32_t(key(e));
    const uint32_t ly = local / T, lx = local % T;
    q[(ly * uint32_t(T + TILE_PAD) + lx) % NB].push_back(e);
  }
  size_t head[NB] = {}, out = 0;
  while (out < v.size())
    for (int b = 0; b < NB; ++b)
      if (head[b] < q[b].size()) v[out++] = q[b][head[b]++];
}

// Orders the w visibilities of one work item (sorted by tile-local cell) for the kernels.
// Thread t of a gridding workgroup takes positions t + k GRID_LANES, k = 0 .. MAX_BIN /
// GRID_LANES - 1, and treats slots 2j and 2j + 1 as a pair when t < P_j: two visibilities
// of the same cell whose 64 taps it adds with one atomic each.  Same-cell visibilities are
// paired greedily, and the pairs are placed at positions (t + 2j L, t + (2j + 1) L), t < P_j,
// where L = GRID_LANES and P_j is as many whole wavefronts (64) of pairs as fit; the rest
// (odd members and pairs that do not fit) fill the other positions as singles.  Pairs and singles are each dealt over the LDS
// banks.  Returns P_0 | P_1 << 16.
uint32_t item_order(KV* kv, int64_t w, int T) {
  constexpr int L = GRID_LANES;
  static_assert(MAX_BIN == 4 * L, "two slot pairs per thread");
  std::vector<std::pair<KV, KV>> pairs;
  std::vector<KV> singles;
  for (int64_t k = 0; k < w;) {
    int64_t e = k;
    while (e < w && uint32_t(kv[e].first) == uint32_t(kv[k].first)) ++e;
    for (; k + 1 < e; k += 2) pairs.push_back({kv[k], kv[k + 1]});
    if (k < e) singles.push_back(kv[k++]);
  }
  const int64_t cap0 = std::clamp<int64_t>(w - L, 0, L), cap1 = std::clamp<int64_t>(w - 3 * L, 0, L);
  // whole wavefronts of pairs, so that no wavefront runs both the pair and the single path
  const int64_t p0 = std::min<int64_t>(int64_t(pairs.size()), cap0) / 64 * 64;
  const int64_t p1 = std::min<int64_t>(int64_t(pairs.size()) - p0, cap1) / 64 * 64;
  for (size_t j = size_t(p0 + p1); j < pairs.size(); ++j) {
    singles.push_back(pairs[j].first);
    singles.push_back(pairs[j].second);
  }
  pairs.resize(size_t(p0 + p1));
  lds_bank_order(pairs, T, [](const std::pair<KV, KV>& e) { return e.first.first; });
  lds_bank_order(singles, T, [](const KV& e) { return e.first; });
  std::vector<KV> out(w);
  std::vector<char> used(w, 0);
  for (int64_t j = 0; j < p0 + p1; ++j) {
    const int64_t a = j < p0 ? j : 2 * L + (j - p0);
    out[a] = pairs[j].first;
    out[a + L] = pairs[j].second;
    used[a] = used[a + L] = 1;
  }
  size_t next = 0;
  for (int64_t a = 0; a < w; ++a)
    if (!used[a]) out[a] = singles[next++];
  std::copy(out.begin(), out.end(), kv);
  return uint32_t(p0) | uint32_t(p1) << 16;
}

int create_plan(Plan& p, int n, int64_t M, const float* uv, int d, const int64_t* off, int J, double beta,
                const ri_tuning* tune, hipStream_t s) {
  if (!is_pow2(n) || n < 16 || n > 2048) return fail(RI_EINVAL, "n=%d must be a power of two in [16, 2048]", n);
  if (M < 1 || M > (int64_t(1) << 31) - 1) return fail(RI_EINVAL, "M=%lld out of range", (long long)M);
  if (d < 1 || d > 4096) return fail(RI_EINVAL, "d=%d must be in [1, 4096]", d);
  if (!uv || !off) return fail(RI_EINVAL, "uv and block_off must not be NULL");
  if (J != KB_J) return fail(RI_EINVAL, "only J=%d is supported (got %d)", KB_J, J);
  if (off[0] != 0 || off[d] != M) return fail(RI_EINVAL, "block_off must start at 0 and end at M");
  for (int i = 0; i < d; ++i)
    if (off[i + 1] <= off[i]) return fail(RI_EINVAL, "block %d is empty or offsets decrease", i);
  for (int64_t m = 0; m < 2 * M; ++m)
    if (!std::isfinite(uv[m])) return fail(RI_EINVAL, "non-finite u-v coordinate at %lld", (long long)(m / 2));

  p.n = n;
  p.K = 2 * n;
  p.M = M;
  p.d = d;
  p.J = J;
  p.beta = beta > 0 ? beta : 2.34 * J;
  p.tile = tune && tune->tile ? tune->tile : 32;
  if (p.tile != 16 && p.tile != 32 && p.tile != 64) return fail(RI_EINVAL, "tile must be 16, 32 or 64");
  // gridding phases need two tiles per axis at least (same-colour tiles must not touch)
  while (p.tile > 16 && p.tile > p.K / 2) p.tile /= 2;
  p.bin = tune && tune->bin > 0 ? tune->bin : MAX_BIN;
  if (p.bin > MAX_BIN) return fail(RI_EINVAL, "bin=%d exceeds %d", p.bin, MAX_BIN);
  if (tune && tune->fft_panel != 0) return fail(RI_EINVAL, "fft_panel is reserved and must be 0");
  p.fft_panel = 0;
  p.persistent_wgs = tune ? tune->persistent_wgs : 0;
  p.slice_vis = tune && tune->slice_vis != 0 ? tune->slice_vis : -1;
  p.tpa = p.K / p.tile;
  p.block_off_host.assign(off, off + d + 1);

  // Kaiser-Bessel polynomials
  std::vector<double> mono;
  kb_fit_taps(J, p.beta, 2 * KB_HALF_DEG + 1, mono, &p.poly_err);
  if (!(p.poly_err < 2e-7)) return fail(RI_EINVAL, "kernel polynomial fit error %.3g too large (beta %.3f)", p.poly_err, p.beta);
  for (int j = 0; j < KB_J / 2; ++j)
    for (int k = 0; k <= KB_HALF_DEG; ++k) {
      p.poly.e[j][k] = float(mono[size_t(j) * (2 * KB_HALF_DEG + 2) + 2 * k]);
      p.poly.o[j][k] = float(mono[size_t(j) * (2 * KB_HALF_DEG + 2) + 2 * k + 1]);
    }

  // coordinates and the sort on the device (plan_sort), then the work items of each block
  // on the host (blocks are independent: one host thread each)
  const int K = p.K, T = p.tile, tpa = p.tpa;
  uint2* packed = nullptr;  // M packed coordinates, user order (device)
  std::vector<uint64_t> skeys;
  std::vector<int> sidx;
  RI_TRY(plan_sort(uv, M, off, d, K, T, tpa, &packed, skeys, sidx, s));
  struct Freer {
    uint2*& q;
    ~Freer() { dev_free(q); }
  } free_packed{packed};
  p.order_host.resize(M);
  std::vector<std::vector<Item>> block_items(d);
  std::vector<std::vector<uint32_t>> block_pairs(d), block_boxes(d);
  std::atomic<int> bad{0};
  const unsigned nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  auto work = [&](int i) {
    const int64_t lo = off[i], hi = off[i + 1];
    std::vector<KV> kv(hi - lo);
    for (int64_t k = lo; k < hi; ++k) {
      const uint64_t key = skeys[k];
      if (int64_t(key >> 28) != i) bad = 1;  // the sort keeps the blocks where they are
      kv[k - lo] = {(((key >> 12) & 0xFFFFu) << 32) | (key & 0xFFFu), int64_t(sidx[k])};
    }
    auto& its = block_items[i];
    auto& prs = block_pairs[i];
    auto& bxs = block_boxes[i];
    int64_t k = 0;
    while (k < hi - lo) {
      const uint64_t tile = kv[k].first >> 32;
      int64_t e = k;
      while (e < hi - lo && (kv[e].first >> 32) == tile) ++e;
      for (int64_t a = k; a < e; a += p.bin) {
        const int64_t w = std::min<int64_t>(p.bin, e - a);
        // footprint box: the item's smallest and largest tile-local row and column
        int b[4] = {T, -1, T, -1};
        for (int64_t m = a; m < a + w; ++m) {
          const int local = int(uint32_t(kv[m].first)), ly = local / T, lx = local % T;
          b[0] = std::min(b[0], ly);
          b[1] = std::max(b[1], ly);
          b[2] = std::min(b[2], lx);
          b[3] = std::max(b[3], lx);
        }
        bxs.push_back(uint32_t(b[0]) | uint32_t(b[1]) << 8 | uint32_t(b[2]) << 16 | uint32_t(b[3]) << 24);
        prs.push_back(item_order(kv.data() + a, w, T));
        its.push_back(make_int4(i, int(tile), int(lo + a), int(w)));
      }
      k = e;
    }
    for (int64_t k = 0; k < hi - lo; ++k) p.order_host[lo + k] = kv[k].second;
  };
  {
    std::vector<std::thread> th;
    std::atomic<int> next{0};
    for (unsigned t = 0; t < nthreads; ++t)
      th.emplace_back([&] {
        for (int i = next++; i < d; i = next++) work(i);
      });
    for (auto& t : th) t.join();
  }
  if (bad) return fail(RI_EHIP, "device sort returned visibilities outside their block");
  std::vector<Item> items;
  std::vector<uint32_t> item_pairs, item_box;
  p.item_off_host.assign(d + 1, 0);
  for (int i = 0; i < d; ++i) {
    p.item_off_host[i] = int(items.size());
    items.insert(items.end(), block_items[i].begin(), block_items[i].end());
    item_pairs.insert(item_pairs.end(), block_pairs[i].begin(), block_pairs[i].end());
    item_box.insert(item_box.end(), block_boxes[i].begin(), block_boxes[i].end());
  }
  p.item_off_host[d] = int(items.size());
  p.n_items = int(items.size());

  // items grouped by tile, and tiles grouped into the four gridding colours
  p.n_tiles = tpa * tpa;
  std::vector<int> tile_cnt(p.n_tiles + 1, 0), tile_vis(p.n_tiles, 0);
  for (const Item& it : items) {
    tile_cnt[it.y + 1] += 1;
    tile_vis[it.y] += it.w;
  }
  for (int t = 0; t < p.n_tiles; ++t) tile_cnt[t + 1] += tile_cnt[t];
  std::vector<int> tile_items(items.size()), fill(tile_cnt.begin(), tile_cnt.end() - 1);
  for (int k = 0; k < int(items.size()); ++k) tile_items[fill[items[k].y]++] = k;
  std::vector<int> empty_tiles;
  for (int t = 0; t < p.n_tiles; ++t)
    if (tile_vis[t] == 0) empty_tiles.push_back(t);
  p.n_empty = int(empty_tiles.size());
  std::vector<int4> units, bunits;
  {
    std::vector<int> ts;
    for (int t = 0; t < p.n_tiles; ++t)
      if (tile_vis[t] > 0) ts.push_back(t);
    std::stable_sort(ts.begin(), ts.end(), [&](int a, int b) { return tile_vis[a] > tile_vis[b]; });
    for (int t : ts) units.push_back(make_int4(t, tile_cnt[t], tile_cnt[t + 1], tile_vis[t]));
  }
  p.tile_units_host = units;
  // split dense tiles into slices of whole items
  std::vector<int> unit_patch;
  std::vector<std::vector<int>> tile_patches(p.n_tiles);
  {
    std::vector<int4> sliced;
    for (const int4& un : units) {
      if (p.slice_vis <= 0 || un.w <= p.slice_vis) {
        sliced.push_back(un);
        unit_patch.push_back(-1);
        continue;
      }
      int a = un.y, acc = 0;
      bool first = true;
      auto emit = [&](int e) {
        sliced.push_back(make_int4(un.x, a, e, acc));
        if (first) {
          unit_patch.push_back(-1);
        } else {
          tile_patches[un.x].push_back(p.n_spatch);
          unit_patch.push_back(p.n_spatch++);
        }
        first = false;
      };
      for (int q = un.y; q < un.z; ++q) {
        const int w = items[tile_items[q]].w;
        if (q > a && acc + w > p.slice_vis) {
          emit(q);
          a = q;
          acc = 0;
        }
        acc += w;
      }
      emit(un.z);
    }
    // densest first
    std::vector<int> idx(sliced.size());
    for (size_t k = 0; k < idx.size(); ++k) idx[k] = int(k);
    std::stable_sort(idx.begin(), idx.end(), [&](int l, int r) { return sliced[l].w > sliced[r].w; });
    units.clear();
    std::vector<int> up;
    for (int k : idx) {
      units.push_back(sliced[k]);
      up.push_back(unit_patch[k]);
    }
    unit_patch.swap(up);
  }
  std::vector<int> tile_sp_off(p.n_tiles + 1, 0), tile_sp;
  for (int t = 0; t < p.n_tiles; ++t) {
    tile_sp_off[t + 1] = tile_sp_off[t] + int(tile_patches[t].size());
    tile_sp.insert(tile_sp.end(), tile_patches[t].begin(), tile_patches[t].end());
  }
  p.n_units = int(units.size());
  std::vector<int4> dunits;
  for (const int4& un : units) {
    int a = un.y, acc = 0;
    for (int q = un.y; q < un.z; ++q) {
      const int w = items[tile_items[q]].w;
      if (q > a && acc + w > DUNIT_VIS) {
        dunits.push_back(make_int4(un.x, a, q, acc));
        a = q;
        acc = 0;
      }
      acc += w;
    }
    dunits.push_back(make_int4(un.x, a, un.z, acc));
  }
  std::stable_sort(dunits.begin(), dunits.end(), [](const int4& l, const int4& r) { return l.w > r.w; });
  p.n_dunits = int(dunits.size());
  {
    // XCD-aware order of the degridding units.  The dispatcher deals consecutive
    // workgroups round-robin over the eight XCDs, and a dense tile has several units, each
    // staging the same tile and reach: the tiles are dealt to the XCDs in density order and
    // all units of a tile are placed at positions equal modulo 8, so that their stagings hit
    // the one XCD's L2.  Gaps (XCDs with fewer units) hold empty units.
    constexpr int NX = 8;
    std::vector<std::vector<int4>> per_xcd(NX);
    std::vector<int> tile_xcd(p.n_tiles, -1);
    int next = 0;
    for (int k = 0; k < p.n_dunits; ++k) {
      int& x = tile_xcd[dunits[k].x];
      if (x < 0) x = next++ % NX;
      per_xcd[x].push_back(dunits[k]);
    }
    size_t L = 0;
    for (const auto& v : per_xcd) L = std::max(L, v.size());
    std::vector<int4> ordered(L * NX, make_int4(0, 0, 0, 0));
    for (int x = 0; x < NX; ++x)
      for (size_t j = 0; j < per_xcd[x].size(); ++j) ordered[j * NX + x] = per_xcd[x][j];
    dunits.swap(ordered);
    p.n_dunits = int(dunits.size());
  }
  p.bunit_off_host.assign(size_t(d) + 1, 0);
  for (int i = 0; i < d; ++i) {
    p.bunit_off_host[i] = int(bunits.size());
    for (int k = p.item_off_host[i]; k < p.item_off_host[i + 1];) {
      int e = k, vis = 0;
      while (e < p.item_off_host[i + 1] && items[e].y == items[k].y) vis += items[e++].w;
      bunits.push_back(make_int4(items[k].y, k, e, vis));
      k = e;
    }
  }
  p.bunit_off_host[d] = int(bunits.size());
  // device copies: y = index in block order
  std::vector<Item> items_dev(items), titems(items.size());
  for (size_t k = 0; k < items.size(); ++k) items_dev[k].y = int(k);
  for (size_t q = 0; q < items.size(); ++q) titems[q] = items_dev[tile_items[q]];

  std::vector<float2> tw(K);
  for (int k = 0; k < K; ++k) {
    const double a = -2.0 * M_PI * k / K;
    tw[k] = make_float2(float(std::cos(a)), float(std::sin(a)));
  }
  std::vector<float> sc(n);
  for (int r = 0; r < n; ++r) sc[r] = float(1.0 / kb_hat(double(r - n / 2) / K, J, p.beta));

  RI_TRY(dev_alloc(&p.coord, M));
  RI_TRY(dev_alloc(&p.order, M));
  RI_TRY(dev_alloc(&p.items, items.size()));
  RI_TRY(dev_alloc(&p.item_box, items.size()));
  RI_TRY(dev_alloc(&p.item_pairs, items.size()));
  RI_TRY(dev_alloc(&p.item_off, d + 1));
  RI_TRY(dev_alloc(&p.block_off, d + 1));
  RI_TRY(dev_alloc(&p.twiddle, K));
  RI_TRY(dev_alloc(&p.scale, n));
  RI_TRY(dev_alloc(&p.grid, size_t(K) * K));
  RI_TRY(dev_alloc(&p.rowbuf, size_t(n) * K));
  RI_TRY(dev_alloc(&p.titems, items.size()));
  RI_TRY(dev_alloc(&p.units, units.size()));
  RI_TRY(dev_alloc(&p.bunits, bunits.size()));
  RI_TRY(dev_alloc(&p.dunits, dunits.size()));
  RI_TRY(dev_alloc(&p.unit_patch, unit_patch.size()));
  RI_TRY(dev_alloc(&p.tile_sp_off, tile_sp_off.size()));
  if (p.n_spatch > 0) {
    RI_TRY(dev_alloc(&p.tile_sp, tile_sp.size()));
    RI_TRY(dev_alloc(&p.spatch, size_t(p.n_spatch) * (p.tile + 8) * (p.tile + 8)));
  }
  RI_TRY(dev_alloc(&p.item_part, 2 * size_t(PART_WAVES) * items.size()));
  RI_TRY(dev_alloc(&p.block_tmp, 2 * size_t(d)));
  RI_TRY(dev_alloc(&p.halo, size_t(p.n_tiles) * ring_cells(p.tile)));
  if (p.n_empty > 0) {
    RI_TRY(dev_alloc(&p.empty_tiles, empty_tiles.size()));
    RI_HIP(hipMemcpyAsync(p.empty_tiles, empty_tiles.data(), empty_tiles.size() * sizeof(int), hipMemcpyHostToDevice,
                          s));
  }
  RI_TRY(dev_alloc(&p.norm_tmp, size_t(n) * n));
  RI_TRY(dev_alloc(&p.dsum, SUMSQ_SCRATCH));
  RI_HIP(hipMemcpyAsync(p.order, p.order_host.data(), M * sizeof(int64_t), hipMemcpyHostToDevice, s));
  RI_TRY(plan_gather_coord(packed, p.order, M, p.coord, s));
  RI_HIP(hipMemcpyAsync(p.items, items_dev.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice, s));
  RI_HIP(hipMemcpyAsync(p.titems, titems.data(), items.size() * sizeof(Item), hipMemcpyHostToDevice, s));
  RI_HIP(hipMemcpyAsync(p.item_box, item_box.data(), items.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
  RI_HIP(hipMemcpyAsync(p.item_pairs, item_pairs.data(), items.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
  RI_HIP(hipMemcpyAsync(p.item_off, p.item_off_host.data(), (d + 1) * sizeof(int), hipMemcpyHostToDevice, s));
  RI_HIP(hipMemcpyAsync(p.block_off, p.block_off_host.data(), (d + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  RI_HIP(hipMemcpyAsync(p.twiddle, tw.data(), K * sizeof(float2), hipMemcpyHostToDevice, s));
  RI_HIP(hipMemcpyAsync(p.units, units.data(), units.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  RI_HIP(hipMemcpyAsync(p.bunits, bunits.data(), bunits.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  RI_HIP(hipMemcpyAsync(p.dunits, dunits.data(), dunits.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  RI_HIP(hipMemcpyAsync(p.unit_patch, unit_patch.data(), unit_patch.size() * sizeof(int), hipMemcpyHostToDevice, s));
  RI_HIP(hipMemcpyAsync(p.tile_sp_off, tile_sp_off.data(), tile_sp_off.size() * sizeof(int), hipMemcpyHostToDevice,
                        s));
  if (p.n_spatch > 0)
    RI_HIP(hipMemcpyAsync(p.tile_sp, tile_sp.data(), tile_sp.size() * sizeof(int), hipMemcpyHostToDevice, s));
  RI_HIP(hipMemcpyAsync(p.scale, sc.data(), n * sizeof(float), hipMemcpyHostToDevice, s));
  // tiles without visibilities keep an all-zero halo patch forever
  RI_TRY(zero_c64(p.halo, size_t(p.n_tiles) * ring_cells(p.tile), s));
  RI_HIP(hipStreamSynchronize(s));
  return RI_OK;
}

}  // namespace

int phi_apply(const Plan& p, const float* x, float* y, const uint8_t* mask, hipStream_t s) {
  RI_TRY(fft_forward(p, x, p.grid, s));
  return degrid_apply(p, p.grid, reinterpret_cast<float2*>(y), mask, s);
}

int phi_adj_apply(const Plan& p, const float* y, float* x, const uint8_t* mask, hipStream_t s) {
  RI_TRY(grid_apply(p, reinterpret_cast<const float2*>(y), mask, p.grid, s));
  return fft_adjoint(p, p.grid, x, s);
}

}  // namespace ri

using ri::fail;

extern "C" {

int ri_plan_create(ri_plan* out, int n, int64_t M, const float* uv_host, int d, const int64_t* block_off_host,
                   int J, double beta, const ri_tuning* tune, hipStream_t stream) {
  if (!out) return fail(RI_EINVAL, "out is NULL");
  *out = nullptr;
  ri_plan h = new (std::nothrow) ri_plan_s;
  if (!h) return fail(RI_ENOMEM, "host allocation failed");
  int rc;
  try {
    rc = ri::create_plan(h->p, n, M, uv_host, d, block_off_host, J, beta, tune, stream);
  } catch (const std::bad_alloc&) {
    rc = fail(RI_ENOMEM, "host allocation failed during plan creation");
  }
  if (rc != RI_OK) {
    ri::destroy_plan(h->p);
    delete h;
    return rc;
  }
  *out = h;
  return RI_OK;
}

void ri_plan_destroy(ri_plan plan) {
  if (!plan) return;
  ri::destroy_plan(plan->p);
  delete plan;
}

int ri_plan_info(ri_plan plan, int* n, int64_t* M, int* d, int* K, int* tile, int* n_items) {
  if (!plan) return fail(RI_EINVAL, "plan is NULL");
  if (n) *n = plan->p.n;
  if (M) *M = plan->p.M;
  if (d) *d = plan->p.d;
  if (K) *K = plan->p.K;
  if (tile) *tile = plan->p.tile;
  if (n_items) *n_items = plan->p.n_items;
  return RI_OK;
}

int ri_plan_order(ri_plan plan, int64_t* order_host) {
  if (!plan || !order_host) return fail(RI_EINVAL, "NULL argument");
  std::memcpy(order_host, plan->p.order_host.data(), plan->p.M * sizeof(int64_t));
  return RI_OK;
}

int ri_plan_permute(ri_plan plan, const float* src, float* dst, int to_plan, hipStream_t stream) {
  if (!plan || !src || !dst) return fail(RI_EINVAL, "NULL argument");
  if (src == dst) return fail(RI_EINVAL, "src and dst must differ");
  hipLaunchKernelGGL(ri::k_permute, dim3(2048), dim3(256), 0, stream, reinterpret_cast<const float2*>(src),
                     reinterpret_cast<float2*>(dst), plan->p.order, plan->p.M, to_plan);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

int ri_phi(ri_plan plan, const float* x, float* y, const uint8_t* mask, hipStream_t stream) {
  if (!plan || !x || !y) return fail(RI_EINVAL, "NULL argument");
  return ri::phi_apply(plan->p, x, y, mask, stream);
}

int ri_phi_adj(ri_plan plan, const float* y, float* x, const uint8_t* mask, hipStream_t stream) {
  if (!plan || !x || !y) return fail(RI_EINVAL, "NULL argument");
  return ri::phi_adj_apply(plan->p, y, x, mask, stream);
}

int ri_block_sumsq(ri_plan plan, const float* y, double* out, hipStream_t stream) {
  if (!plan || !y || !out) return fail(RI_EINVAL, "NULL argument");
  return ri::block_sumsq(plan->p, reinterpret_cast<const float2*>(y), out, stream);
}

int ri_phi_norm(ri_plan plan, float* x0, int max_it, double rtol, double* norm_host, int* iters_host,
                hipStream_t stream) {
  if (!plan || !x0 || !norm_host || max_it < 1) return fail(RI_EINVAL, "bad argument");
  ri::Plan& p = plan->p;
  const size_t N = size_t(p.n) * p.n;
  float* y = nullptr;
  RI_TRY(ri::dev_alloc(&y, 2 * size_t(p.M)));
  float* cur = x0;
  float* nxt = p.norm_tmp;
  double lam = 0.0, lam_prev = 0.0, sq = 0.0;
  int it = 0, rc = RI_OK;
  rc = ri::sumsq_f32(cur, N, p.dsum, stream);
  if (rc == RI_OK) rc = ri::scale_by_rsqrt(cur, N, p.dsum, stream);
  for (it = 1; rc == RI_OK && it <= max_it; ++it) {
    rc = ri::phi_apply(p, cur, y, nullptr, stream);
    if (rc == RI_OK) rc = ri::phi_adj_apply(p, y, nxt, nullptr, stream);
    if (rc == RI_OK) rc = ri::sumsq_f32(nxt, N, p.dsum, stream);
    if (rc == RI_OK && hipMemcpyAsync(&sq, p.dsum, sizeof(double), hipMemcpyDeviceToHost, stream) != hipSuccess)
      rc = fail(RI_EHIP, "copy of the norm failed");
    if (rc == RI_OK && hipStreamSynchronize(stream) != hipSuccess) rc = fail(RI_EHIP, "stream sync failed");
    if (rc != RI_OK) break;
    lam = std::sqrt(sq);
    rc = ri::scale_by_rsqrt(nxt, N, p.dsum, stream);
    std::swap(cur, nxt);
    if (lam == 0.0 || std::fabs(lam - lam_prev) <= rtol * lam) break;
    lam_prev = lam;
  }
  if (rc == RI_OK && cur != x0) {
    hipLaunchKernelGGL(ri::k_copy_f32, dim3(1024), dim3(256), 0, stream, cur, x0, N);
    if (hipGetLastError() != hipSuccess) rc = fail(RI_EHIP, "copy launch failed");
  }
  if (rc == RI_OK && hipStreamSynchronize(stream) != hipSuccess) rc = fail(RI_EHIP, "stream sync failed");
  ri::dev_free(y);
  if (rc != RI_OK) return rc;
  *norm_host = std::sqrt(lam);
  if (iters_host) *iters_host = std::min(it, max_it);
  return RI_OK;
}

}  // extern "C"
