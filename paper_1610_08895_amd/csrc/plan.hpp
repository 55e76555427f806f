// Internal state of a measurement-operator plan (Phi = G M F Z, Eq. 3 / Eq. 8).
#pragma once

#include <vector>

#include "common.hpp"

namespace ri {

// Kaiser-Bessel weights of the J = 8 taps as polynomials in x = 2 f - 1 (f the fractional
// grid coordinate): w_j = E_j(x^2) + x O_j(x^2) and w_{7-j} = E_j(x^2) - x O_j(x^2), j < 4.
constexpr int KB_J = 8;
// E_j, O_j of degree 3 in x^2 (total degree 7): fit error below 1e-7 (for beta from 1.8 J
// to 2.7 J), about the FP32 resolution of the weights themselves; degree 9 measured no
// different in Phi and Phi^dagger and costs 16 more FMAs per visibility
constexpr int KB_HALF_DEG = 3;
struct KBPoly {
  float e[KB_J / 2][KB_HALF_DEG + 1];
  float o[KB_J / 2][KB_HALF_DEG + 1];
};

// Fixed-point grid coordinate: cell index in the high 12 bits, fraction in the low 20.
constexpr int FRAC_BITS = 20;
constexpr unsigned FRAC_MASK = (1u << FRAC_BITS) - 1u;

// The J = 8 weights phi(f + 3 - j) of a packed coordinate (f its fraction) and its cell
// floor(kappa); tap j sits at cell floor(kappa) - 3 + j.
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

// A work item: up to `bin` visibilities of one block that fall in one grid tile.
// x = block, y = tile (ty * tiles_per_axis + tx), z = first plan position, w = count.
// The device copies carry in y the item's index in block order instead (which indexes the
// per-item arrays); the tile comes from the unit that lists the item.
using Item = int4;
constexpr int MAX_BIN = 1024;    // largest `bin` (4 visibilities per thread of a gridding workgroup)
constexpr int GRID_LANES = 256;  // threads per workgroup of the tile gridding
// LDS row pitch of a staged tile region in 8-byte cells: the region's width T + 8 plus
// TILE_PAD - 8 more, so that consecutive rows start in different LDS banks (the plan deals
// a wavefront's visibilities over the banks of this layout)
constexpr int TILE_PAD = 9;
constexpr int DUNIT_VIS = 2048;  // visibilities per degridding unit (several items of one tile)
constexpr int PART_WAVES = 4;    // FP64 norm partials per work item (one per wavefront)
// Cells of a tile's halo ring: its (tile + 8)^2 region (the tile and the kernel's reach)
// less the tile itself.
constexpr int ring_cells(int tile) { return (tile + 8) * (tile + 8) - tile * tile; }

// Direction-dependent effects folded into G (Eq. 1's D, Sec. II): each visibility's row of
// G is its DDE kernel (jd x jd taps, jd = 2h + 1) convolved with the Kaiser-Bessel kernel,
// S = J + 2h taps per axis, stored per visibility.
struct Dde {
  int h = -1;                     // -1: no DDEs (plain G)
  int S = 0;                      // taps per axis
  float2* w = nullptr;            // S * S * M weights, tap-major: w[t * M + m] (plan order)
  float* wmax = nullptr;          // M: max over taps of |Re w| + |Im w| (fixed-point bound)
  int4* tunits = nullptr;         // whole-tile units {tile, first, end, vis} over titems
  int n_tunits = 0;
  float2* patch = nullptr;        // n_tiles * (T + S - 1)^2: each tile's gridded region
  uint8_t* tile_has = nullptr;    // n_tiles: tile has visibilities (its patch is written)
  bool on() const { return h >= 0; }
};

struct Plan {
  int n = 0, K = 0, J = KB_J, d = 0;
  int64_t M = 0;
  double beta = 0.0;
  int tile = 32, bin = 1024, tpa = 0;  // tiles per axis
  int n_items = 0;
  int fft_panel = 0;
  int persistent_wgs = 0;
  int slice_vis = -1;  // <= 0: tiles are never split
  KBPoly poly{};
  double poly_err = 0.0;

  std::vector<int> item_off_host;  // d + 1
  int n_tiles = 0;                  // tpa * tpa
  // gridding units {tile, first, end} over an item index list: all blocks together (densest
  // tile first), and block by block
  int n_units = 0;
  int n_dunits = 0;                 // degridding units: items of one tile, <= DUNIT_VIS visibilities
  std::vector<int> bunit_off_host;  // d + 1
  std::vector<int64_t> order_host;  // plan position -> user index
  std::vector<int64_t> block_off_host;

  // device
  uint2* coord = nullptr;     // M packed (x, y) coordinates, plan order
  int64_t* order = nullptr;   // M, plan position -> user index
  Item* items = nullptr;      // n_items, block order (y = own index)
  Item* titems = nullptr;     // n_items grouped by tile (all blocks), y = index in block order
  // n_items footprint boxes: the smallest and largest row and column of the item's first
  // taps relative to its tile origin, one byte each (row min, row max, column min, column
  // max from the low byte up)
  uint32_t* item_box = nullptr;
  // n_items: P_0 | P_1 << 16, the threads of a gridding workgroup that hold a same-cell pair
  // in slots (0, 1) and (2, 3) of the item (see item_order)
  uint32_t* item_pairs = nullptr;
  int* item_off = nullptr;    // d + 1
  int64_t* block_off = nullptr;  // d + 1 block offsets (visibilities, plan order = user order per block)
  float2* twiddle = nullptr;  // K forward twiddles exp(-2 pi i k / K)
  float* scale = nullptr;     // n: S along one axis, 1 / phi_hat(l / K)
  float2* grid = nullptr;     // K * K work grid
  float2* rowbuf = nullptr;   // n * K half-transformed rows
  int4* units = nullptr;        // tile slices with items, densest first; ranges into titems
  // A tile with more than slice_vis visibilities is split into slices (units of whole
  // items); the first accumulates into the grid and the tile's halo patch, each further
  // one into a whole-region slice patch, which the halo pass adds in a fixed order.
  int n_spatch = 0;
  int* unit_patch = nullptr;    // n_units: slice patch of the unit, -1 for a tile's first slice
  int* tile_sp_off = nullptr;   // n_tiles + 1: slice patches of each tile
  int* tile_sp = nullptr;       // n_spatch
  float2* spatch = nullptr;     // n_spatch * (tile + 8)^2
  int4* bunits = nullptr;       // per block; ranges into items
  int4* dunits = nullptr;       // degridding units, densest first; ranges into titems
  double* item_part = nullptr;  // 2 * PART_WAVES * n_items partial sums of the block norms
  double* block_tmp = nullptr;  // 2 * d
  float2* halo = nullptr;       // n_tiles * ring_cells(tile) halo rings of the gridding
  int n_empty = 0;
  int* empty_tiles = nullptr;   // n_empty tiles without visibilities
  std::vector<int4> tile_units_host;  // whole-tile units over titems, densest first
  Dde dde;
  int* active_count = nullptr;
  float* norm_tmp = nullptr;  // n * n scratch for power iterations
  double* dsum = nullptr;     // FP64 reduction scratch
};

// ---- launchers implemented in fft.hip ----
// grid = F Z S x (x: n*n real).
int fft_forward(const Plan& p, const float* x, float2* grid, hipStream_t s);
// x = Re S Z^dagger F^dagger grid (x: n*n real).
int fft_adjoint(const Plan& p, const float2* grid, float* x, hipStream_t s);
// The two passes of each, through the plan's n x K row buffer.
int fft_forward_rows(const Plan& p, const float* x, hipStream_t s);
int fft_forward_cols(const Plan& p, float2* grid, hipStream_t s);
int fft_adjoint_cols(const Plan& p, const float2* grid, hipStream_t s);
int fft_adjoint_rows(const Plan& p, float* x, hipStream_t s);
// Steps 17-18 fused into the adjoint row pass: with g = Re S Z^dagger F^dagger of the
// plan's row buffer, x <- max(0, x - tau (sigma st + varsigma g)) and xt = 2 x_new - x_old,
// elementwise over the n x n image (g itself is not stored).
struct PrimalUpdate {
  const float* st;
  float* x;
  float* xt;
  float tau, sigma, varsigma;
};
int fft_adjoint_rows_update(const Plan& p, const PrimalUpdate& u, hipStream_t s);

// ---- launchers implemented in gridding.hip ----
// stats[2i], stats[2i+1] = per-block sums of the degridding partials, active blocks only;
// copied to out (may be null) with NaN rows for inactive blocks.  With eps and shrink
// given, also shrink[i] = max(0, 1 - eps_i / ||r_i||) (0 inside the ball) for active blocks.
// part: the per-item partials to reduce (null: the plan's).
int block_stats(const Plan& p, const uint8_t* mask, double* stats, double* out, hipStream_t s,
                const double* eps = nullptr, float* shrink = nullptr, const double* part = nullptr);
// out[i] = ||y_i||^2 (FP64) for every block.
int block_sumsq(const Plan& p, const float2* y, double* out, hipStream_t s);
// y = G b for the items of active blocks (operator form).
int degrid_apply(const Plan& p, const float2* grid, float2* y, const uint8_t* mask, hipStream_t s);
// grid = G^dagger y for the active blocks (operator form; the whole grid is written, tiles
// without visibilities set to zero).
int grid_apply(const Plan& p, const float2* y, const uint8_t* mask, float2* grid, hipStream_t s);
// PD residual pass: r = v + G b - y stored in r_out; stats[2i] = ||r_i||^2, stats[2i+1] =
// ||G_i b_i - y_i||^2 for the blocks whose items are processed (per-item partial sums, then
// a per-block reduction).  All items (those of inactive blocks skipped), or one block's.
// zero_empty (not with DDEs): a grid whose tiles without visibilities the same launch sets
// to zero (for grid_project_all(..., zeroed = true), which then skips that).
int degrid_residual(const Plan& p, const float2* grid, const float2* y, const float2* v, float2* e,
                    const uint8_t* mask, hipStream_t s, float2* zero_empty = nullptr);
// The norms of degrid_residual over all items, without storing e, into the given partials
// (2 * PART_WAVES * n_items doubles).
int degrid_norms(const Plan& p, const float2* grid, const float2* y, const float2* v, double* part, hipStream_t s);
int degrid_residual_block(const Plan& p, int block, const float2* grid, const float2* y, const float2* v,
                          float2* e, hipStream_t s);
// PD projection pass: v_new = r shrink_i (r from degrid_residual, shrink from block_stats);
// grid += G^dagger (v_new - v); v = v_new, for the active blocks (tile interiors; grid_halo
// must follow) or for one block.  grid_project_all, with every block active: v = v_new and
// grid = G^dagger v_new (tile interiors stored; grid_halo must follow); not with DDEs.
int grid_project(const Plan& p, const float2* e, float2* v, const float* shrink, const uint8_t* mask, float2* grid,
                 hipStream_t s);
// Adds the tile halos left by grid_project (which stores them) into the grid.
int grid_project_all(const Plan& p, const float2* r, float2* v, const float* shrink, float2* grid, hipStream_t s,
                     bool zeroed = false);
int grid_halo(const Plan& p, float2* grid, hipStream_t s);
// y = Phi x over the blocks with mask[i] != 0 (mask may be null: all); x = Re Phi^dagger y.
// y is complex interleaved (M), x real (n*n); both use the plan's work grid.
int phi_apply(const Plan& p, const float* x, float* y, const uint8_t* mask, hipStream_t s);
int phi_adj_apply(const Plan& p, const float* y, float* x, const uint8_t* mask, hipStream_t s);
// Per-block form of grid_project: grid_blocks_begin zeroes the halo rings, each
// grid_project_block adds one block's tile interiors into the grid and its rings into the
// zeroed rings, and grid_blocks_end adds the rings into the grid (one halo pass).
int grid_blocks_begin(const Plan& p, hipStream_t s);
int grid_project_block(const Plan& p, int block, const float2* e, float2* v, const float* shrink, float2* grid,
                       hipStream_t s);
int grid_blocks_end(const Plan& p, float2* grid, hipStream_t s);
// grid = G^dagger v over all items (rebuilds the running sum from scratch).
int grid_all(const Plan& p, const float2* v, float2* grid, hipStream_t s);

// ---- plan creation on the device (plan_sort.hip) ----
// Packs the M coordinates (uv host, user order) into *packed (device, allocated here, the
// caller frees it) and sorts the visibilities by (block, tile, cell in the tile), stably;
// keys_sorted / idx_sorted receive the sorted keys (block << 28 | tile << 12 | cell) and
// the user index of each sorted position.  Synchronises s.
int plan_sort(const float* uv, int64_t M, const int64_t* off, int d, int K, int T, int tpa, uint2** packed,
              std::vector<uint64_t>& keys_sorted, std::vector<int>& idx_sorted, hipStream_t s);
// coord[k] = packed[order[k]] (device arrays of M).
int plan_gather_coord(const uint2* packed, const int64_t* order, int64_t M, uint2* coord, hipStream_t s);

// ---- DDE-aware G (dde.hip); used by the functions above when p.dde.on() ----
int dde_degrid(const Plan& p, const int4* units, int nunits, const Item* items, const uint8_t* mask,
               const float2* grid, float2* out, const float2* y, const float2* v, double* part, hipStream_t s);
// gridding over whole-tile units into the tiles' patches (ADD: added to them, per-block use)
int dde_grid(const Plan& p, const int4* units, int nunits, const Item* items, const uint8_t* mask,
             const float2* y, const float2* e, float2* v, const float* shrink, bool project, bool add_patch,
             hipStream_t s);
// grid (=, or += with add) the sum of the patches covering each cell
int dde_merge(const Plan& p, float2* grid, bool add, hipStream_t s);
int dde_zero_patches(const Plan& p, hipStream_t s);
void dde_destroy(Dde& dd);

// ---- reductions (reduce.hip) ----
int zero_f32(float* p, size_t n, hipStream_t s);
int zero_c64(float2* p, size_t n, hipStream_t s);
// out[0] = sum x^2 (FP64); out holds SUMSQ_SCRATCH doubles.
constexpr int SUMSQ_SCRATCH = 1025;
int sumsq_f32(const float* x, size_t n, double* out, hipStream_t s);
// x *= 1 / sqrt(*sq) (device scalar, FP64)
int scale_by_rsqrt(float* x, size_t n, const double* sq, hipStream_t s);

}  // namespace ri
