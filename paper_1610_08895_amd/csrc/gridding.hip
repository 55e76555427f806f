// Interpolation G_i (degridding) and its adjoint G_i^dagger (gridding) over sorted
// visibilities, with the per-block work of Algorithm 1 fused in:
//
//   degrid_residual  steps 5 and 8 (first half): r = v_i + G_i b_i - y_i stored, and the
//                    FP64 block sums ||r_i||^2 (for the projection, Eq. 10) and
//                    ||G_i b_i - y_i||^2 (for Eq. 13).
//   grid_project     steps 8 (second half), 9 and 11: v_i <- r max(0, 1 - eps_i / ||r_i||)
//                    (the Moreau form of v + Gb - P_B(v + Gb)), and the change
//                    G_i^dagger (v_new - v_old) added into the running grid sum
//                    sum_i M_i^dagger v~_i.  Blocks outside A are not visited, so their v_i
//                    and v~_i stay as they are.
//   grid_project_all with every block active: v_i <- r max(0, 1 - eps_i / ||r_i||) and the
//                    sum rebuilt from scratch, G^dagger v_new stored (it reads r and writes
//                    v, 24 bytes per visibility, and stores the grid instead of updating it).
//
// Visibilities are sorted by (block, tile, cell); a work item holds up to `bin`
// visibilities of one block in one T x T grid tile.
//
// Degridding walks the items with a persistent grid of workgroups, skipping the items
// of inactive blocks (the mask is read on the device, so a captured graph follows
// whatever mask is current); each stages
// its tile plus the kernel's reach (3 cells before, 4 after, per axis) in LDS so all 64
// taps of a visibility are LDS reads.  Block norms are accumulated per item in FP64 and
// reduced per block by a second kernel in a fixed order (no atomics, deterministic).
//
// Gridding is owner-computes per tile: one workgroup accumulates every active item of a
// tile (all blocks) into an LDS copy of the tile and its reach (exact integer LDS atomics
// per item, see k_grid_tiles), adds the tile interior to the grid with a plain
// read-modify-write (no other workgroup writes it) and stores the reach outside the
// interior in a per-tile halo patch; a second kernel adds the neighbours' patches into
// each tile's border cells.  No global atomics are needed, and one launch covers all tiles
// (densest first).  Inside an item thread t takes positions t, t + 256, t + 512 and
// t + 768; the plan puts two visibilities of the same cell into slots (0, 1) or (2, 3) of
// whole wavefronts where it can, and both kernels then treat them as a pair: the
// degridding reads each staged value once for both, the gridding adds both contributions
// with one atomic per tap.  The plan also deals the pairs and the single visibilities of a
// wavefront evenly over the LDS banks of the staged tile.  Items whose values are all zero
// (a block whose dual did not change) are skipped.
#include "plan.hpp"

namespace ri {

namespace {

constexpr int GT = 256;    // threads per workgroup
static_assert(GT / 64 == PART_WAVES, "one norm partial per wavefront of a workgroup");
constexpr int GGT = GRID_LANES;  // threads per workgroup of the tile gridding

// Items base .. base + count - 1.
struct ItemSource {
  const Item* items;
  int base, count;
};


enum { DG_APPLY = 0, DG_RESIDUAL = 1, DG_NORMS = 2 };  // NORMS: the residual's norms only

// LDS row pitch of a staged tile: one more than the region width, so that rows of the
// tile start in different LDS banks.
template <int T>
struct Pitch {
  static constexpr int TW = T + 8;  // region: the tile plus the kernel's reach
  static constexpr int TP = T + TILE_PAD;
};

// Position of region cell (ly, lx), outside the tile interior [R0, R0 + T)^2, in the tile's
// halo ring, which is stored compactly: the full-width rows above the interior, then those
// below it, then for each interior row its R0 cells on the left and its TW - T - R0 cells on
// the right.  Readers of the left and right edges then take whole cache lines.
template <int T>
__device__ __forceinline__ int ring_index(int ly, int lx) {
  constexpr int TW = Pitch<T>::TW, R0 = KB_J / 2 - 1;
  if (ly < R0) return ly * TW + lx;
  if (ly >= R0 + T) return (ly - T) * TW + lx;
  return (TW - T) * TW + (ly - R0) * (TW - T) + (lx < R0 ? lx : lx - T);
}
static_assert((Pitch<32>::TW - 32) * Pitch<32>::TW + 32 * (Pitch<32>::TW - 32) == ring_cells(32), "ring layout");

// Degridding over units {tile, first, end} of the unit-ordered items (items of one tile,
// several blocks): the tile and its reach are staged once per unit, then the waves go
// through the unit's items without synchronising.  Each thread loads all of its (at most
// MAX_BIN / GT) visibilities of an item before computing any, and the residual norms of
// an item are left as one FP64 partial pair per wavefront (part[(item * NWAVES + w) * 2],
// item = its index in block order).
template <int T, int MODE>
__global__ __launch_bounds__(GT) void k_degrid(const int4* __restrict__ units, int nunits,
                                               const Item* __restrict__ items,
                                               const uint32_t* __restrict__ item_pairs,
                                               const uint8_t* __restrict__ mask,
                                               const uint2* __restrict__ coord, const float2* __restrict__ grid, int K,
                                               int tpa, KBPoly P, float2* __restrict__ out,
                                               const float2* __restrict__ y, const float2* __restrict__ v,
                                               double* __restrict__ part, int ustride,
                                               float2* __restrict__ zero_grid, const int* __restrict__ zero_tiles) {
  constexpr int TW = Pitch<T>::TW, TP = Pitch<T>::TP;
  constexpr int NV = MAX_BIN / GT;
  constexpr int NWV = GT / 64;
  static_assert(GT == GRID_LANES && NV == 4, "the item order's slot pairs (item_order)");
  // the data branch's kernels issue ahead of the sparsity branch's waves sharing their SIMDs
  __builtin_amdgcn_s_setprio(3);
  __shared__ float2 tile[TW * TP];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (int(blockIdx.x) >= ustride) {
    // a further workgroup: zeroes the interior of one tile without visibilities in
    // zero_grid (a grid that the step's gridding will rebuild, untouched until then)
    const int t = zero_tiles[blockIdx.x - ustride];
    const int ty = t / tpa, tx = t - (t / tpa) * tpa;
    for (int c = threadIdx.x; c < T * T; c += GT)
      zero_grid[size_t(ty * T + c / T) * K + tx * T + c % T] = make_float2(0.f, 0.f);
    return;
  }
  for (int u = blockIdx.x; u < nunits; u += ustride) {
    const int4 un = units[u];
    bool any = mask == nullptr && un.y < un.z;  // an empty unit fills a gap of the XCD order
    for (int q = un.y; q < un.z && !any; ++q) any = mask[items[q].x] != 0;
    if (!any) continue;
    const int ty = un.x / tpa, tx = un.x - (un.x / tpa) * tpa;
    const int gy0 = ty * T - (KB_J / 2 - 1), gx0 = tx * T - (KB_J / 2 - 1);
    for (int idx = threadIdx.x; idx < TW * TW; idx += GT) {
      const int ly = idx / TW, lx = idx - ly * TW;
      const int gy = (gy0 + ly) & (K - 1), gx = (gx0 + lx) & (K - 1);
      tile[ly * TP + lx] = grid[size_t(gy) * K + gx];
    }
    __syncthreads();
    for (int q = un.y; q < un.z; ++q) {
      const Item it = items[q];
      if (mask != nullptr && mask[it.x] == 0) continue;
      uint2 c[NV];
      float2 yy[NV], vv[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const int s = threadIdx.x + k * GT;
        if (s < it.w) {
          c[k] = coord[it.z + s];
          if (MODE != DG_APPLY) {
            yy[k] = y[it.z + s];
            vv[k] = v[it.z + s];
          }
        }
      }
      double sr = 0.0, se = 0.0;
      auto emit = [&](int k, float2 acc) {
        const int s = threadIdx.x + k * GT;
        if (MODE == DG_APPLY) {
          out[it.z + s] = acc;
        } else {
          const float2 e = make_float2(acc.x - yy[k].x, acc.y - yy[k].y);
          const float2 r = make_float2(vv[k].x + e.x, vv[k].y + e.y);
          if (MODE == DG_RESIDUAL) out[it.z + s] = r;
          sr += double(r.x) * r.x + double(r.y) * r.y;
          se += double(e.x) * e.x + double(e.y) * e.y;
        }
      };
      auto single = [&](int k) {
        float wx[KB_J], wy[KB_J];
        int cx, cy;
        kb_weights(c[k].x, P, wx, cx);
        kb_weights(c[k].y, P, wy, cy);
        const float2* base = &tile[(cy - ty * T) * TP + (cx - tx * T)];
        float2 acc = make_float2(0.f, 0.f);
#pragma unroll
        for (int ra = 0; ra < KB_J; ++ra) {
          const float2* row = base + ra * TP;
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
        emit(k, acc);
      };
      // two visibilities of one cell: each staged value is read once for both
      auto pair = [&](int k, int k2) {
        float wx[KB_J], wy[KB_J], wx2[KB_J], wy2[KB_J];
        int cx, cy, cx2, cy2;
        kb_weights(c[k].x, P, wx, cx);
        kb_weights(c[k].y, P, wy, cy);
        kb_weights(c[k2].x, P, wx2, cx2);
        kb_weights(c[k2].y, P, wy2, cy2);
        const float2* base = &tile[(cy - ty * T) * TP + (cx - tx * T)];
        float2 acc = make_float2(0.f, 0.f), acc2 = make_float2(0.f, 0.f);
#pragma unroll
        for (int ra = 0; ra < KB_J; ++ra) {
          const float2* row = base + ra * TP;
          float2 rs = make_float2(0.f, 0.f), rs2 = make_float2(0.f, 0.f);
#pragma unroll
          for (int b = 0; b < KB_J; ++b) {
            const float2 g = row[b];
            rs.x = fmaf(wx[b], g.x, rs.x);
            rs.y = fmaf(wx[b], g.y, rs.y);
            rs2.x = fmaf(wx2[b], g.x, rs2.x);
            rs2.y = fmaf(wx2[b], g.y, rs2.y);
          }
          acc.x = fmaf(wy[ra], rs.x, acc.x);
          acc.y = fmaf(wy[ra], rs.y, acc.y);
          acc2.x = fmaf(wy2[ra], rs2.x, acc2.x);
          acc2.y = fmaf(wy2[ra], rs2.y, acc2.y);
        }
        emit(k, acc);
        emit(k2, acc2);
      };
      const uint32_t npair = item_pairs[it.y];
#pragma unroll
      for (int j = 0; j < NV / 2; ++j) {
        const int k = 2 * j, s = threadIdx.x + k * GT;
        if (threadIdx.x < int((npair >> (16 * j)) & 0xffffu)) {
          pair(k, k + 1);
        } else {
          if (s < it.w) single(k);
          if (s + GT < it.w) single(k + 1);
        }
      }
      if (MODE != DG_APPLY) {
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

// stats[2i], stats[2i+1] = sums of the per-item, per-wavefront partials of block i, for
// active blocks; a copy goes to out (if not null), with NaN for inactive blocks.
__global__ __launch_bounds__(GT) void k_block_stats(const uint8_t* __restrict__ mask, const int* __restrict__ item_off,
                                                    const double* __restrict__ part, double* __restrict__ stats,
                                                    double* __restrict__ out, const double* __restrict__ eps,
                                                    float* __restrict__ shrink) {
  __shared__ double red[2][GT / 64];
  const int i = blockIdx.x;
  // the data branch's kernels issue ahead of the sparsity branch's waves sharing their SIMDs
  __builtin_amdgcn_s_setprio(3);
  if (mask != nullptr && mask[i] == 0) {
    if (out != nullptr && threadIdx.x == 0) {  // quiet NaN, stored as its bit pattern
      unsigned long long* o = reinterpret_cast<unsigned long long*>(out);
      o[2 * i] = 0x7ff8000000000000ull;
      o[2 * i + 1] = 0x7ff8000000000000ull;
    }
    return;
  }
  // the same sequence of additions as a plain strided loop, with eight loads in flight
  double a0 = 0.0, a1 = 0.0;
  const int kb = item_off[i] * PART_WAVES, ke = item_off[i + 1] * PART_WAVES;
  const double2* p2 = reinterpret_cast<const double2*>(part);
  for (int k0 = kb + threadIdx.x; k0 < ke; k0 += 8 * GT) {
    double2 t[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) t[j] = k0 + j * GT < ke ? p2[k0 + j * GT] : make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      a0 += t[j].x;
      a1 += t[j].y;
    }
  }
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x / 64] = a0;
    red[1][threadIdx.x / 64] = a1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int k = 0; k < GT / 64; ++k) {
      s0 += red[0][k];
      s1 += red[1][k];
    }
    stats[2 * i] = s0;
    stats[2 * i + 1] = s1;
    if (shrink != nullptr) {  // step 8 through its Moreau form: r max(0, 1 - eps / ||r||)
      const double ep = eps[i];
      shrink[i] = s0 > ep * ep ? float(1.0 - ep / sqrt(s0)) : 0.f;
    }
    if (out != nullptr) {
      out[2 * i] = s0;
      out[2 * i + 1] = s1;
    }
  }
}

// APPLY: grid y.  PROJECT: step 8 from r and v_old, grid v_new - v_old.  FRESH: every block
// active, step 8 from r alone, grid v_new.
enum { GR_APPLY = 0, GR_PROJECT = 1, GR_FRESH = 2 };

// Rounding of a float t with |t| < 2^22 to an integer by adding 1.5 * 2^23 (see below).
constexpr float ROUND_BIAS = 12582912.0f;
constexpr unsigned long long ROUND_BIAS_BITS = 0x4B4000004B400000ull;

// A gridding unit: one tile and the range [b, e) of idx[] listing the items that fall in
// it (x = tile, y = b, z = e, w = their visibility count).
//
// Per item the contributions are accumulated exactly in LDS with 64-bit integer atomics
// (LDS integer atomics are an order of magnitude faster than LDS float atomics on this
// hardware), Re in the low and Im in the high 32 bits of one word: every value is scaled
// by a power of two 2^E such that the item's sum of |Re| + |Im|, which bounds any cell's
// sum (the kernel weights are at most 1), stays below 2^30, and the sum of the two
// contributions of a thread's slot pair (one rounded word for a same-cell pair) below 2^22
// in magnitude.  A contribution t = w x is rounded to an integer n by one FMA
// that adds B = 1.5 * 2^23: for |t| < 2^22 the result lies in [2^23, 2^24), where floats are
// the integers, so it is B + n with n = t rounded to nearest (ties to even), and its bit
// pattern is 0x4B400000 + n.  A same-cell pair adds its second contribution with a second
// FMA onto B + n_2, which is again an integer in that range, so it yields B + n_2 + n_1.  The word is then (bits of Im) 2^32 + (bits of Re) minus the
// constant 0x4B4000004B400000, which equals n_re + n_im 2^32 in two's complement (a
// negative n_re borrows from the high half); decoding subtracts the sign-extended low field.
// Rounding is at most 2^-E-1 per contribution.
//
// Two integer tiles alternate between items: while item q is accumulated into one, the
// cells of item q-1's footprint box are folded out of the other (and cleared) into FP32
// accumulators held in registers, each thread owning fixed cells of the region.  Each
// thread also keeps the values and coordinates of its (at most MAX_BIN / GGT) visibilities
// of the current item in registers and loads those of the next active item meanwhile, so
// one barrier per item separates the phases.  At the end the tile interior (owned by this
// workgroup alone) is added to the grid and the reach outside it is stored in the tile's
// halo patch for k_grid_halo (a further slice of a split tile stores its whole region in
// its slice patch instead).
// Register budget: four wavefronts per SIMD (<= 128 VGPRs) for tiles up to 32, which
// measured faster than the three the unconstrained allocation allows; the 64 tile is held
// to one workgroup per CU by its LDS anyway.
template <int T>
constexpr int grid_waves_per_simd() {
  return T <= 32 ? 4 : 1;
}

template <int T, int MODE>
__global__ __launch_bounds__(GGT, grid_waves_per_simd<T>()) void k_grid_tiles(const int4* __restrict__ units, int nunits,
                                                   const Item* __restrict__ items,
                                                   const uint32_t* __restrict__ item_box,
                                                   const uint32_t* __restrict__ item_pairs,
                                                   const uint8_t* __restrict__ mask, const uint2* __restrict__ coord,
                                                   float2* __restrict__ grid, float2* __restrict__ halo, int K,
                                                   int tpa, KBPoly P, const float2* __restrict__ y,
                                                   const float2* __restrict__ e, float2* __restrict__ v,
                                                   const float* __restrict__ shrink,
                                                   const int* __restrict__ unit_patch, float2* __restrict__ spatch,
                                                   int fresh, int ring_add, int ustride,
                                                   const int* __restrict__ zero_tiles) {
  constexpr int TW = Pitch<T>::TW, TP = Pitch<T>::TP;
  constexpr int R0 = KB_J / 2 - 1;  // reach before the tile
  constexpr int NV = MAX_BIN / GGT;
  constexpr int NWV = GGT / 64;
  // region cells per thread: thread t owns the words t + j GGT of the pitched layout (the
  // pad column included), so that its cells lie a whole number of 512-byte strides apart
  // and two of them move with one LDS instruction
  constexpr int NC = (TW * TP + GGT - 1) / GGT;
  static_assert(NV == 4, "two slot pairs per thread (item_order)");
  // the data branch's kernels issue ahead of the sparsity branch's waves sharing their SIMDs
  __builtin_amdgcn_s_setprio(3);
  __shared__ unsigned long long acci[2][TW * TP];
  __shared__ float red_b[2][NWV], red_m[2][NWV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

  // with a mask, the current unit's active items as bits (item act_base + k: bit k), every
  // lane testing one item at once; a unit of more than 64 items tests them one by one
  const bool masked = MODE != GR_FRESH && mask != nullptr;
  unsigned long long act = 0ull;
  int act_base = 0;
  bool bits = false;
  auto is_active = [&](int q) {
    return bits ? ((act >> (q - act_base)) & 1ull) != 0ull : mask[items[q].x] != 0;
  };
  auto next_active = [&](int q, int end) {
    if (!masked) return q;
    if (bits) {
      const int o = q - act_base;
      const unsigned long long m = o < 64 ? act >> o : 0ull;
      return m != 0ull ? q + __builtin_ctzll(m) : end;
    }
    while (q < end && mask[items[q].x] == 0) ++q;
    return q;
  };
  // operands of the current item, and the raw loads of the next one
  float2 val[NV], ra[NV], rb[NV];
  uint2 crd[NV], rc[NV];
  auto load_raw = [&](const Item& it) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int s = threadIdx.x + k * GGT;
      if (s < it.w) {
        const int m = it.z + s;
        rc[k] = coord[m];
        if (MODE == GR_APPLY) {
          ra[k] = y[m];
        } else if (MODE == GR_FRESH) {
          rb[k] = e[m];
        } else {
          ra[k] = v[m];
          rb[k] = e[m];
        }
      }
    }
  };
  // values (with the dual update of step 8) and the bounds into red_b[buf], red_m[buf]
  auto finish = [&](const Item& it, int buf) {
    const float sh = MODE != GR_APPLY ? shrink[it.x] : 0.f;
    float babs = 0.f, bmax = 0.f;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int s = threadIdx.x + k * GGT;
      if (s < it.w) {
        const int m = it.z + s;
        if (MODE == GR_APPLY) {
          val[k] = ra[k];
        } else if (MODE == GR_FRESH) {
          const float2 vn = make_float2(rb[k].x * sh, rb[k].y * sh);
          v[m] = vn;
          val[k] = vn;
        } else {
          const float2 vn = make_float2(rb[k].x * sh, rb[k].y * sh);
          v[m] = vn;
          val[k] = make_float2(vn.x - ra[k].x, vn.y - ra[k].y);
        }
        crd[k] = rc[k];
        babs += fabsf(val[k].x) + fabsf(val[k].y);
      } else {
        val[k] = make_float2(0.f, 0.f);
      }
    }
    // the largest sum of one component over a slot pair (a same-cell pair adds both
    // contributions into one rounded word; for two singles this bounds each as well)
#pragma unroll
    for (int k = 0; k < NV; k += 2)
      bmax = fmaxf(bmax, fmaxf(fabsf(val[k].x) + fabsf(val[k + 1].x), fabsf(val[k].y) + fabsf(val[k + 1].y)));
    babs = wave_sum(babs);
    bmax = wave_max(bmax);
    if (lane == 0) {
      red_b[buf][wv] = babs;
      red_m[buf][wv] = bmax;
    }
  };
  // this thread's region cells
  float2 acc[NC];
  // Only the slices of cells that meet the box's rows are visited (a test that is the same
  // for the whole workgroup); cells outside the box were never touched and read as zero.
  static_assert(TP > TW, "pitched rows");
  auto fold = [&](int buf, uint32_t box, float inv) {
    const int r0 = box & 255u, r1 = int((box >> 8) & 255u) + KB_J;
    // slices are taken two at a time (one row test, and two cells per LDS instruction)
#pragma unroll
    for (int j = 0; j < NC; j += 2) {
      const int jn = j + 1 < NC ? 2 : 1;
      if ((j * GGT + jn * GGT - 1) / TP < r0 || (j * GGT) / TP >= r1) continue;
#pragma unroll
      for (int h = 0; h < jn; ++h) {
        const int c = threadIdx.x + (j + h) * GGT;
        if ((j + h + 1) * GGT <= TW * TP || c < TW * TP) {
          unsigned long long* cell = &acci[buf][c];
          const unsigned long long w64 = *cell;
          *cell = 0ull;
          // Re is the low field as a signed integer; Im is the high field plus the borrow
          // that a negative Re took from it
          const int ir = static_cast<int>(static_cast<unsigned>(w64));
          const int ii = static_cast<int>(static_cast<unsigned>(w64 >> 32) + (static_cast<unsigned>(ir) >> 31));
          acc[j + h].x = fmaf(float(ir), inv, acc[j + h].x);
          acc[j + h].y = fmaf(float(ii), inv, acc[j + h].y);
        }
      }
    }
  };

  if (int(blockIdx.x) >= ustride) {
    // a further workgroup of a fresh launch: zeroes the interior of one tile without
    // visibilities, which no unit writes (dispatched after the units, in their tail)
    const int t = zero_tiles[blockIdx.x - ustride];
    const int ty = t / tpa, tx = t - (t / tpa) * tpa;
    for (int c = threadIdx.x; c < T * T; c += GGT)
      grid[size_t(ty * T + c / T) * K + tx * T + c % T] = make_float2(0.f, 0.f);
    return;
  }
  for (int k = threadIdx.x; k < 2 * TW * TP; k += GGT) (&acci[0][0])[k] = 0ull;
  for (int u = blockIdx.x; u < nunits; u += ustride) {
    const int4 un = units[u];
    const int ty = un.x / tpa, tx = un.x - (un.x / tpa) * tpa;
#pragma unroll
    for (int j = 0; j < NC; ++j) acc[j] = make_float2(0.f, 0.f);
    // the first item's loads are issued before its block's mask is read (units are never
    // empty, and a masked item's loads are simply not used)
    int q = un.y, buf = 0;
    Item it = items[q];
    load_raw(it);
    if (masked) {
      bits = un.z - un.y <= 64;
      act_base = un.y;
      if (bits) act = __ballot(lane < un.z - un.y && mask[items[un.y + lane].x] != 0);
    }
    if (masked && !is_active(q)) {
      q = next_active(q + 1, un.z);
      if (q < un.z) {
        it = items[q];
        load_raw(it);
      }
    }
    if (q < un.z) finish(it, 0);
    __syncthreads();
    bool pend = false;  // a fold of the previous item is due
    uint32_t pbox = 0;
    float pinv = 0.f;
    while (q < un.z) {
      float bound = 0.f, bmax = 0.f;
#pragma unroll
      for (int w = 0; w < NWV; ++w) {
        bound += red_b[buf][w];
        bmax = fmaxf(bmax, red_m[buf][w]);
      }
      const uint32_t box = item_box[it.y];
      const int qn = next_active(q + 1, un.z);
      Item itn = make_int4(0, 0, 0, 0);
      if (qn < un.z) {
        itn = items[qn];
        load_raw(itn);
      }
      // 2^E with bound * 2^E < 2^30 and bmax * 2^E < 2^22 / 1.001, so that a pair's two
      // rounded contributions sum to less than 2^22 (the factors guard the bounds' own
      // rounding, the kernel fit's excess over 1 and the rounding of w x)
      int ex = 0, exm = 0;
      if (bound > 0.f) {
        frexpf(bound * 1.0001f, &ex);
        frexpf(bmax * 1.001f, &exm);
      }
      const int e2 = min(30 - ex, 22 - exm);
      const float scale = ldexpf(1.f, e2), inv = ldexpf(1.f, -e2);
      if (bound > 0.f) {
        const uint32_t npair = item_pairs[it.y];
        // one visibility: per tap an FMA per component and one atomic
        auto single = [&](int k) {
          const float vr = val[k].x * scale, vi = val[k].y * scale;
          float wx[KB_J], wy[KB_J];
          int cx, cy;
          kb_weights(crd[k].x, P, wx, cx);
          kb_weights(crd[k].y, P, wy, cy);
          unsigned long long* base = &acci[buf][(cy - ty * T) * TP + (cx - tx * T)];
#pragma unroll
          for (int r = 0; r < KB_J; ++r) {
            const float tr = wy[r] * vr, ti = wy[r] * vi;
#pragma unroll
            for (int b = 0; b < KB_J; ++b) {
              const unsigned lo = __float_as_uint(fmaf(wx[b], tr, ROUND_BIAS));
              const unsigned hi = __float_as_uint(fmaf(wx[b], ti, ROUND_BIAS));
              atomicAdd(base + r * TP + b, ((static_cast<unsigned long long>(hi) << 32) | lo) - ROUND_BIAS_BITS);
            }
          }
        };
        // two visibilities of one cell (the plan guarantees it): each contribution is
        // rounded by its own FMA (the inner one leaves an integer-valued float, so the outer
        // one adds the second rounded value exactly) and the pair takes one atomic per tap
        auto pair = [&](int k, int k2) {
          const float vr = val[k].x * scale, vi = val[k].y * scale;
          const float vr2 = val[k2].x * scale, vi2 = val[k2].y * scale;
          float wx[KB_J], wy[KB_J], wx2[KB_J], wy2[KB_J];
          int cx, cy, cx2, cy2;
          kb_weights(crd[k].x, P, wx, cx);
          kb_weights(crd[k].y, P, wy, cy);
          kb_weights(crd[k2].x, P, wx2, cx2);
          kb_weights(crd[k2].y, P, wy2, cy2);
          unsigned long long* base = &acci[buf][(cy - ty * T) * TP + (cx - tx * T)];
#pragma unroll
          for (int r = 0; r < KB_J; ++r) {
            const float tr = wy[r] * vr, ti = wy[r] * vi, tr2 = wy2[r] * vr2, ti2 = wy2[r] * vi2;
#pragma unroll
            for (int b = 0; b < KB_J; ++b) {
              const unsigned lo = __float_as_uint(fmaf(wx[b], tr, fmaf(wx2[b], tr2, ROUND_BIAS)));
              const unsigned hi = __float_as_uint(fmaf(wx[b], ti, fmaf(wx2[b], ti2, ROUND_BIAS)));
              atomicAdd(base + r * TP + b, ((static_cast<unsigned long long>(hi) << 32) | lo) - ROUND_BIAS_BITS);
            }
          }
        };
#pragma unroll
        for (int j = 0; j < NV / 2; ++j) {
          const int k = 2 * j, s = threadIdx.x + k * GGT;
          if (threadIdx.x < int((npair >> (16 * j)) & 0xffffu)) {
            pair(k, k + 1);
          } else {
            if (s < it.w) single(k);
            if (s + GGT < it.w) single(k + 1);
          }
        }
      }
      if (pend) fold(buf ^ 1, pbox, pinv);
      pend = bound > 0.f;
      pbox = box;
      pinv = inv;
      if (qn < un.z) finish(itn, buf ^ 1);
      __syncthreads();
      q = qn;
      it = itn;
      buf ^= 1;
    }
    const int sp = unit_patch != nullptr ? unit_patch[u] : -1;
    if (pend) fold(buf ^ 1, pbox, pinv);
    float2* patch = sp >= 0 ? spatch + size_t(sp) * TW * TW : halo + size_t(un.x) * ring_cells(T);
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      // the cell's coordinates and addresses are recomputed for every unit (an empty asm
      // hides that they do not change): keeping them across the unit loop costs registers
      int c = threadIdx.x + j * GGT;
      asm volatile("" : "+v"(c));
      if (c >= TW * TP) continue;
      const int ly = c / TP, lx = c - (c / TP) * TP;
      if (lx >= TW) continue;  // the pad column
      const float2 a = acc[j];
      const bool inside = ly >= R0 && ly < R0 + T && lx >= R0 && lx < R0 + T;
      if (inside && sp < 0) {
        float2* g = &grid[size_t(ty * T + ly - R0) * K + tx * T + lx - R0];
        if (fresh) {
          *g = a;  // the workgroup owns the interior: no read of the old value
        } else if (a.x != 0.f || a.y != 0.f) {
          const float2 old = *g;
          *g = make_float2(old.x + a.x, old.y + a.y);
        }
      } else if (sp < 0) {
        float2* h = &patch[ring_index<T>(ly, lx)];  // the ring
        if (!ring_add) {
          *h = a;
        } else if (a.x != 0.f || a.y != 0.f) {
          const float2 old = *h;
          *h = make_float2(old.x + a.x, old.y + a.y);
        }
      } else {
        patch[ly * TW + lx] = a;  // a further slice's whole region
      }
    }
  }
}

// Adds the halo patches of the eight neighbours of each tile into its interior cells
// within reach of its edges (3 cells from the far edge, 4 from the near edge).  Each patch
// cell outside its tile lies in exactly one other tile's interior, so it has exactly one
// reader.  The patches are only read: the batched gridding rewrites the whole ring of
// every tile with visibilities in each launch, and the per-block form zeroes all rings
// before its first block and accumulates into them.  Where the tile or a neighbour has
// slice patches (sp_off not null), their cells that fall in this tile's interior are added
// too, in a fixed order; every slice rewrites its whole patch in each gridding launch.
template <int T>
__global__ __launch_bounds__(GT) void k_grid_halo(const float2* __restrict__ halo, float2* __restrict__ grid, int K,
                                                  int tpa, const int* __restrict__ sp_off,
                                                  const int* __restrict__ sp_list,
                                                  const float2* __restrict__ spatch) {
  constexpr int TW = T + 8;
  constexpr int R0 = KB_J / 2 - 1;
  constexpr int NEAR = KB_J / 2, FAR = R0;  // edge rows / columns reached from outside
  // the data branch's kernels issue ahead of the sparsity branch's waves sharing their SIMDs
  __builtin_amdgcn_s_setprio(3);
  constexpr int NE = T * T - (T - NEAR - FAR) * (T - NEAR - FAR);  // edge cells
  const int t = blockIdx.x;
  const int ty = t / tpa, tx = t - (t / tpa) * tpa;
  bool slices = false;
  if (sp_off != nullptr)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int nt = ((ty + dy + tpa) & (tpa - 1)) * tpa + ((tx + dx + tpa) & (tpa - 1));
        slices = slices || sp_off[nt + 1] > sp_off[nt];
      }
  const int ncell = slices ? T * T : NE;
  for (int k = threadIdx.x; k < ncell; k += GT) {
    int iy, ix;
    if (slices) {
      iy = k / T;
      ix = k - iy * T;
    } else if (k < (NEAR + FAR) * T) {  // full edge rows
      const int r = k / T;
      iy = r < NEAR ? r : T - NEAR - FAR + r;
      ix = k - r * T;
    } else {  // the edge columns of the rows between
      const int k2 = k - (NEAR + FAR) * T;
      const int c = k2 % (NEAR + FAR);
      iy = NEAR + k2 / (NEAR + FAR);
      ix = c < NEAR ? c : T - NEAR - FAR + c;
    }
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        // local coordinates of this cell in the neighbour's region
        const int ly = iy - dy * T + R0, lx = ix - dx * T + R0;
        if (ly < 0 || ly >= TW || lx < 0 || lx >= TW) continue;
        const int nt = ((ty + dy + tpa) & (tpa - 1)) * tpa + ((tx + dx + tpa) & (tpa - 1));
        if (dy != 0 || dx != 0) {
          const float2 h = halo[size_t(nt) * ring_cells(T) + ring_index<T>(ly, lx)];
          acc.x += h.x;
          acc.y += h.y;
        }
        if (slices)
          for (int j = sp_off[nt]; j < sp_off[nt + 1]; ++j) {
            const float2 h = spatch[size_t(sp_list[j]) * TW * TW + ly * TW + lx];
            acc.x += h.x;
            acc.y += h.y;
          }
      }
    if (acc.x != 0.f || acc.y != 0.f) {
      float2* g = &grid[size_t(ty * T + iy) * K + tx * T + ix];
      const float2 old = *g;
      *g = make_float2(old.x + acc.x, old.y + acc.y);
    }
  }
}

__global__ __launch_bounds__(GT) void k_block_sumsq(ItemSource src, const float2* __restrict__ y,
                                                    double* __restrict__ part) {
  const int wv = threadIdx.x >> 6;
  for (int a = blockIdx.x; a < src.count; a += gridDim.x) {
    const int iidx = src.base + a;
    const Item it = src.items[iidx];
    double acc = 0.0;
    for (int m = it.z + threadIdx.x; m < it.z + it.w; m += GT) {
      const float2 v = y[m];
      acc += double(v.x) * v.x + double(v.y) * v.y;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) {
      part[(size_t(iidx) * PART_WAVES + wv) * 2] = acc;
      part[(size_t(iidx) * PART_WAVES + wv) * 2 + 1] = 0.0;
    }
  }
}

__global__ void k_take_even(const double* __restrict__ in, double* __restrict__ out, int d) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d; i += gridDim.x * blockDim.x) out[i] = in[2 * i];
}

// Workgroups of a launch over `units` units: one per unit unless the plan fixes a count
// (then each takes every gridDim.x-th unit).  With one workgroup per unit, densest first,
// the hardware dispatcher hands each freed slot the next unit, which balances the uneven
// units better than any fixed assignment measured.
int wgs_for(const Plan& p, int units) {
  const int g = p.persistent_wgs > 0 ? p.persistent_wgs : units;
  return units < g ? (units > 0 ? units : 1) : g;
}

// sliced: after a launch over the plan's tile slices (slice patches are merged too);
// otherwise after the per-block launches, which never write slice patches.
template <int T>
void launch_halo(const Plan& p, float2* grid, bool sliced, hipStream_t s) {
  const bool sp = sliced && p.n_spatch > 0;
  hipLaunchKernelGGL((k_grid_halo<T>), dim3(p.n_tiles), dim3(GT), 0, s, p.halo, grid, p.K, p.tpa,
                     sp ? p.tile_sp_off : nullptr, sp ? p.tile_sp : nullptr, sp ? p.spatch : nullptr);
}

// units/items: the plan's tile slices over titems (sliced = true) or one block's units
// over items (whole tiles).
// fresh: the launch overwrites the grid (tile interiors stored, tiles without visibilities
// zeroed by further workgroups of the launch unless `zeroed` says that is done) instead of
// adding into it.  Over the plan's tile slices (sliced)
// each tile's ring is overwritten; over one block's units it is added to, and the caller
// zeroes the rings before the first block and runs the halo pass after the last.
template <int T, int MODE>
int launch_grid(const Plan& p, bool sliced, const int4* units, int nunits, const Item* items, const uint8_t* mask,
                float2* grid, const float2* y, const float2* e, float2* v, const float* shrink, hipStream_t s,
                bool with_halo = true, bool fresh = false, bool zeroed = false) {
  const int g = wgs_for(p, nunits), extra = fresh && !zeroed ? p.n_empty : 0;
  if (nunits > 0 || extra > 0) {
    hipLaunchKernelGGL((k_grid_tiles<T, MODE>), dim3(g + extra), dim3(GGT), 0, s, units, nunits, items, p.item_box,
                       p.item_pairs, mask, p.coord, grid, p.halo, p.K, p.tpa, p.poly, y, e, v, shrink,
                       sliced ? p.unit_patch : nullptr, p.spatch, fresh ? 1 : 0, sliced ? 0 : 1, g, p.empty_tiles);
    RI_LAUNCH_CHECK();
  }
  if (with_halo) {
    launch_halo<T>(p, grid, sliced, s);
    RI_LAUNCH_CHECK();
  }
  return RI_OK;
}

template <int MODE>
int grid_units(const Plan& p, bool sliced, const int4* units, int nunits, const Item* items, const uint8_t* mask,
               float2* grid, const float2* y, const float2* e, float2* v, const float* shrink, hipStream_t s,
               bool with_halo = true, bool fresh = false, bool zeroed = false) {
#define RI_GRID_T(TT) \
  launch_grid<TT, MODE>(p, sliced, units, nunits, items, mask, grid, y, e, v, shrink, s, with_halo, fresh, zeroed)
  switch (p.tile) {
    case 16: return RI_GRID_T(16);
    case 32: return RI_GRID_T(32);
    case 64: return RI_GRID_T(64);
    default: return fail(RI_EINVAL, "unsupported tile %d", p.tile);
  }
#undef RI_GRID_T
}

#define RI_TILE_DISPATCH(KERNEL, ...)                                                          \
  switch (p.tile) {                                                                            \
    case 16: hipLaunchKernelGGL((KERNEL<16, __VA_ARGS__>), grid_dim, dim3(GT), 0, s, ARGS); break; \
    case 32: hipLaunchKernelGGL((KERNEL<32, __VA_ARGS__>), grid_dim, dim3(GT), 0, s, ARGS); break; \
    case 64: hipLaunchKernelGGL((KERNEL<64, __VA_ARGS__>), grid_dim, dim3(GT), 0, s, ARGS); break; \
    default: return fail(RI_EINVAL, "unsupported tile %d", p.tile);                            \
  }

}  // namespace

int block_sumsq(const Plan& p, const float2* y, double* out, hipStream_t s) {
  ItemSource src{p.items, 0, p.n_items};
  hipLaunchKernelGGL(k_block_sumsq, dim3(wgs_for(p, p.n_items)), dim3(GT), 0, s, src, y, p.item_part);
  RI_LAUNCH_CHECK();
  RI_TRY(block_stats(p, nullptr, p.block_tmp, nullptr, s));
  hipLaunchKernelGGL(k_take_even, dim3((p.d + 255) / 256), dim3(256), 0, s, p.block_tmp, out, p.d);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

int block_stats(const Plan& p, const uint8_t* mask, double* stats, double* out, hipStream_t s, const double* eps,
                float* shrink, const double* part) {
  if ((eps == nullptr) != (shrink == nullptr)) return fail(RI_EINVAL, "block_stats: eps and shrink go together");
  hipLaunchKernelGGL(k_block_stats, dim3(p.d), dim3(GT), 0, s, mask, p.item_off, part ? part : p.item_part, stats,
                     out, eps, shrink);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

namespace {

// Degridding over the plan's units (in XCD order, see create_plan).
// zero: a grid whose tiles without visibilities further workgroups of the same launch
// zero (or null).
template <int T, int MODE>
int degrid_batched_t(const Plan& p, const float2* grid, float2* out, const float2* y, const float2* v,
                     double* part, const uint8_t* mask, float2* zero, hipStream_t s) {
  const int g = wgs_for(p, p.n_dunits), extra = zero != nullptr ? p.n_empty : 0;
  if (p.n_dunits > 0 || extra > 0) {
    hipLaunchKernelGGL((k_degrid<T, MODE>), dim3(g + extra), dim3(GT), 0, s, p.dunits, p.n_dunits, p.titems,
                       p.item_pairs, mask, p.coord, grid, p.K, p.tpa, p.poly, out, y, v, part, g, zero,
                       p.empty_tiles);
    RI_LAUNCH_CHECK();
  }
  return RI_OK;
}

template <int MODE>
int degrid_batched(const Plan& p, const float2* grid, float2* out, const float2* y, const float2* v, double* part,
                   const uint8_t* mask, hipStream_t s, float2* zero = nullptr) {
  switch (p.tile) {
    case 16: return degrid_batched_t<16, MODE>(p, grid, out, y, v, part, mask, zero, s);
    case 32: return degrid_batched_t<32, MODE>(p, grid, out, y, v, part, mask, zero, s);
    case 64: return degrid_batched_t<64, MODE>(p, grid, out, y, v, part, mask, zero, s);
    default: return fail(RI_EINVAL, "unsupported tile %d", p.tile);
  }
}

}  // namespace

int degrid_apply(const Plan& p, const float2* grid, float2* y, const uint8_t* mask, hipStream_t s) {
  if (p.dde.on()) return dde_degrid(p, p.dunits, p.n_dunits, p.titems, mask, grid, y, nullptr, nullptr, nullptr, s);
  return degrid_batched<DG_APPLY>(p, grid, y, nullptr, nullptr, nullptr, mask, s);
}

int degrid_residual(const Plan& p, const float2* grid, const float2* y, const float2* v, float2* e,
                    const uint8_t* mask, hipStream_t s, float2* zero_empty) {
  if (p.dde.on()) {
    if (zero_empty != nullptr) return fail(RI_EINVAL, "degrid_residual: no tile zeroing with DDEs");
    return dde_degrid(p, p.dunits, p.n_dunits, p.titems, mask, grid, e, y, v, p.item_part, s);
  }
  return degrid_batched<DG_RESIDUAL>(p, grid, e, y, v, p.item_part, mask, s, zero_empty);
}

int degrid_norms(const Plan& p, const float2* grid, const float2* y, const float2* v, double* part, hipStream_t s) {
  if (p.dde.on()) return dde_degrid(p, p.dunits, p.n_dunits, p.titems, nullptr, grid, nullptr, y, v, part, s);
  return degrid_batched<DG_NORMS>(p, grid, nullptr, y, v, part, nullptr, s);
}

int degrid_residual_block(const Plan& p, int block, const float2* grid, const float2* y, const float2* v,
                          float2* e, hipStream_t s) {
  const int a = p.bunit_off_host[block], b = p.bunit_off_host[block + 1];
  if (p.dde.on()) return dde_degrid(p, p.bunits + a, b - a, p.items, nullptr, grid, e, y, v, p.item_part, s);
  const dim3 grid_dim(wgs_for(p, b - a));
#define ARGS p.bunits + a, b - a, p.items, p.item_pairs, (const uint8_t*)nullptr, p.coord, grid, p.K, p.tpa, \
             p.poly, e, y, v, p.item_part, int(grid_dim.x), (float2*)nullptr, (const int*)nullptr
  RI_TILE_DISPATCH(k_degrid, DG_RESIDUAL)
#undef ARGS
  RI_LAUNCH_CHECK();
  return RI_OK;
}

int grid_apply(const Plan& p, const float2* y, const uint8_t* mask, float2* grid, hipStream_t s) {
  if (p.dde.on()) {
    RI_TRY(dde_grid(p, p.dde.tunits, p.dde.n_tunits, p.titems, mask, y, nullptr, nullptr, nullptr, false, false, s));
    return dde_merge(p, grid, false, s);
  }
  return grid_units<GR_APPLY>(p, true, p.units, p.n_units, p.titems, mask, grid, y, nullptr, nullptr, nullptr,
                              s, true, true);
}

int grid_all(const Plan& p, const float2* v, float2* grid, hipStream_t s) {
  if (p.dde.on()) return grid_apply(p, v, nullptr, grid, s);
  return grid_units<GR_APPLY>(p, true, p.units, p.n_units, p.titems, nullptr, grid, v, nullptr, nullptr,
                              nullptr, s, true, true);
}

int grid_project(const Plan& p, const float2* e, float2* v, const float* shrink, const uint8_t* mask, float2* grid,
                 hipStream_t s) {
  if (p.dde.on())  // the tiles' patches; grid_halo adds them into the grid
    return dde_grid(p, p.dde.tunits, p.dde.n_tunits, p.titems, mask, nullptr, e, v, shrink, true, false, s);
  return grid_units<GR_PROJECT>(p, true, p.units, p.n_units, p.titems, mask, grid, nullptr, e, v, shrink, s,
                                false);
}

int grid_project_all(const Plan& p, const float2* r, float2* v, const float* shrink, float2* grid, hipStream_t s,
                     bool zeroed) {
  if (p.dde.on()) return fail(RI_EINVAL, "grid_project_all: the DDE kernels update the running sum instead");
  return grid_units<GR_FRESH>(p, true, p.units, p.n_units, p.titems, nullptr, grid, nullptr, r, v, shrink, s, false,
                              true, zeroed);
}

int grid_halo(const Plan& p, float2* grid, hipStream_t s) {
  if (p.dde.on()) return dde_merge(p, grid, true, s);
  switch (p.tile) {
    case 16: launch_halo<16>(p, grid, true, s); break;
    case 32: launch_halo<32>(p, grid, true, s); break;
    case 64: launch_halo<64>(p, grid, true, s); break;
    default: return fail(RI_EINVAL, "unsupported tile %d", p.tile);
  }
  RI_LAUNCH_CHECK();
  return RI_OK;
}

int grid_project_block(const Plan& p, int block, const float2* e, float2* v, const float* shrink, float2* grid,
                       hipStream_t s) {
  const int a = p.bunit_off_host[block], b = p.bunit_off_host[block + 1];
  if (p.dde.on()) return dde_grid(p, p.bunits + a, b - a, p.items, nullptr, nullptr, e, v, shrink, true, true, s);
  return grid_units<GR_PROJECT>(p, false, p.bunits + a, b - a, p.items, nullptr, grid, nullptr, e, v, shrink, s,
                                false);
}

int grid_blocks_begin(const Plan& p, hipStream_t s) {
  if (p.dde.on()) return dde_zero_patches(p, s);
  return zero_c64(p.halo, size_t(p.n_tiles) * ring_cells(p.tile), s);
}

int grid_blocks_end(const Plan& p, float2* grid, hipStream_t s) {
  if (p.dde.on()) return dde_merge(p, grid, true, s);
  switch (p.tile) {
    case 16: launch_halo<16>(p, grid, false, s); break;
    case 32: launch_halo<32>(p, grid, false, s); break;
    case 64: launch_halo<64>(p, grid, false, s); break;
    default: return fail(RI_EINVAL, "unsupported tile %d", p.tile);
  }
  RI_LAUNCH_CHECK();
  return RI_OK;
}

}  // namespace ri
