// Algorithm 1, randomised forward-backward primal-dual, one iteration per call.
//
// Data-fidelity branch (steps 4-11): b~ = F Z x~; for active blocks r = v_i + G_i b_i - y_i
// with FP64 block norms; v_i <- r max(0, 1 - eps_i / ||r||); the change of G_i^dagger v_i is
// added to the running sum sum_i M_i^dagger v~_i, which therefore holds the latest v~_i of
// active blocks and the kept v~_i of inactive ones (step 11) (with every block active the
// sum is rebuilt from the new v instead); then g = Re Z^dagger F^dagger (that sum).
// Sparsity branch (steps 13-14): s <- clip(s + Psi^dagger x~, -alpha, alpha), then
// s~ = Psi s.
// The two branches depend only on x~ of the previous iteration (the paper runs them
// concurrently); the batched step forks the sparsity branch onto a side stream after the
// forward FFT and joins before the last kernel, the adjoint row pass, which applies the
// elementwise steps 17-18 to g as it produces it (g is never stored).
//
// The running sum is kept in FP32 and updated by differences when blocks are masked;
// ri_pd_refresh (and setting V) rebuilds it from the stored v, bounding accumulated rounding.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "handles.hpp"
#include "sara.hpp"
#include "vjp.hpp"

struct ri_pd_s {
  ri::Plan* plan = nullptr;
  ri::Sara* sara = nullptr;
  ri_pd_params prm{};
  float alpha = 0.f;
  float2* y = nullptr;
  float2* v = nullptr;
  float2* e = nullptr;     // r = v + G b - y of the last step's active blocks
  float* x = nullptr;
  float* xt = nullptr;
  float* s = nullptr;
  float* st = nullptr;     // s~ = Psi s
  // weights of a weighted l1 prior (b*n*n, the layout of s; null: the plain prior), which
  // make the bound of step 13's clip alpha w_k per coefficient (reweighted SARA)
  float* wts = nullptr;
  float2* sum = nullptr;   // sum_i M_i^dagger v~_i on the K x K grid
  double* eps = nullptr;   // d
  double* stats = nullptr; // d x 2
  float* shrink = nullptr;  // d: max(0, 1 - eps_i / ||r_i||) of the current step
  uint8_t* mask_dev = nullptr;
  int64_t iter = 0;
  // scratch of the reverse sweep, allocated on its first call
  float* vj_z = nullptr;      // n*n: zbar
  float* vj_st = nullptr;     // n*n: Psi s_new
  float* vj_g = nullptr;      // n*n: Re Phi^dagger v_new, then Re Phi_A^dagger rbar
  float* vj_w = nullptr;      // b*n*n: Psi^dagger zbar
  float2* vj_phiz = nullptr;  // M: Phi zbar
  double* vj_part = nullptr;  // dot-product and per-block partials
  double* vj_coef = nullptr;  // 2 d
  // residual at x of ri_pd_residual (M complex), allocated on its first call
  float2* res_e = nullptr;
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // optional per-stage timing: an event pair around each stage, on the stage's stream
  bool timing = false;
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  int open[RI_STAGE_COUNT] = {};
};

namespace ri {
namespace {

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

int take_event(ri_pd_s* P, hipEvent_t* e) {
  if (!P->pool.empty()) {
    *e = P->pool.back();
    P->pool.pop_back();
    return RI_OK;
  }
  RI_HIP(hipEventCreate(e));
  return RI_OK;
}

int stage_begin(ri_pd_s* P, int st, hipStream_t s) {
  if (!P->timing || capturing(s)) return RI_OK;
  ri_pd_s::Rec r{st, nullptr, nullptr};
  RI_TRY(take_event(P, &r.a));
  RI_TRY(take_event(P, &r.b));
  RI_HIP(hipEventRecord(r.a, s));
  P->open[st] = int(P->recs.size());
  P->recs.push_back(r);
  return RI_OK;
}

int stage_end(ri_pd_s* P, int st, hipStream_t s) {
  if (!P->timing || capturing(s)) return RI_OK;
  RI_HIP(hipEventRecord(P->recs[P->open[st]].b, s));
  return RI_OK;
}

#define RI_STAGE(P, ST, S, CALL)       \
  do {                                \
    RI_TRY(ri::stage_begin(P, ST, S)); \
    RI_TRY(CALL);                     \
    RI_TRY(ri::stage_end(P, ST, S));   \
  } while (0)

void destroy_pd(ri_pd_s* P) {
  dev_free(P->y);
  dev_free(P->v);
  dev_free(P->e);
  dev_free(P->x);
  dev_free(P->xt);
  dev_free(P->s);
  dev_free(P->st);
  dev_free(P->wts);
  dev_free(P->sum);
  dev_free(P->eps);
  dev_free(P->stats);
  dev_free(P->shrink);
  dev_free(P->mask_dev);
  dev_free(P->vj_z);
  dev_free(P->vj_st);
  dev_free(P->vj_g);
  dev_free(P->vj_w);
  dev_free(P->vj_phiz);
  dev_free(P->vj_part);
  dev_free(P->vj_coef);
  dev_free(P->res_e);
  if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
  if (P->ev_join) (void)hipEventDestroy(P->ev_join);
  if (P->side) (void)hipStreamDestroy(P->side);
  for (auto& r : P->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : P->pool) (void)hipEventDestroy(e);
}

int refresh_sum(ri_pd_s* P, hipStream_t s) {
  const Plan& p = *P->plan;
  return grid_all(p, P->v, P->sum, s);
}

int sparsity_branch(ri_pd_s* P, hipStream_t s) {
  // step 13 (Moreau form of the soft-threshold), then step 14
  RI_STAGE(P, RI_STAGE_PSI_ADJ, s, psi_adj_apply(*P->sara, P->xt, P->s, true, P->alpha, s, P->wts));
  RI_STAGE(P, RI_STAGE_PSI_SYNTH, s, psi_apply(*P->sara, P->s, P->st, s));
  return RI_OK;
}

// w_k = delta / (delta + |c_k|) in place, c = Psi^dagger x
__global__ __launch_bounds__(256) void k_reweight(size_t count, float delta, float* __restrict__ w) {
  for (size_t k = size_t(blockIdx.x) * 256 + threadIdx.x; k < count; k += size_t(gridDim.x) * 256)
    w[k] = delta / (delta + fabsf(w[k]));
}

__global__ __launch_bounds__(256) void k_fill(size_t count, float v, float* __restrict__ w) {
  for (size_t k = size_t(blockIdx.x) * 256 + threadIdx.x; k < count; k += size_t(gridDim.x) * 256) w[k] = v;
}

unsigned grid_for(size_t count) { return unsigned(std::min<size_t>((count + 255) / 256, 8192)); }

int ensure_weights(ri_pd_s* P, hipStream_t s) {
  if (P->wts) return RI_OK;
  const size_t nb = size_t(P->sara->b) * P->plan->n * P->plan->n;
  RI_TRY(dev_alloc(&P->wts, nb));
  hipLaunchKernelGGL(k_fill, dim3(grid_for(nb)), dim3(256), 0, s, nb, 1.f, P->wts);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

}  // namespace
}  // namespace ri

using ri::fail;

extern "C" {

int ri_pd_create(ri_pd* out, ri_plan plan, ri_sara sara, const float* y, const double* eps_host,
                 const ri_pd_params* params, hipStream_t stream) {
  if (!out || !plan || !sara || !y || !eps_host || !params) return fail(RI_EINVAL, "NULL argument");
  *out = nullptr;
  ri::Plan& p = plan->p;
  ri::Sara& S = sara->s;
  if (S.n != p.n) return fail(RI_EINVAL, "image sizes differ (plan %d, dictionary %d)", p.n, S.n);
  const ri_pd_params& q = *params;
  if (!(q.tau > 0 && q.sigma > 0 && q.varsigma > 0 && q.kappa > 0 && q.psi_norm > 0 && q.phi_norm > 0))
    return fail(RI_EINVAL, "tau, sigma, varsigma, kappa and the norms must be positive");
  const double cond = q.tau * (q.sigma * q.psi_norm * q.psi_norm + q.varsigma * q.phi_norm * q.phi_norm);
  if (!(cond < 1.0)) return fail(RI_EINVAL, "tau (sigma ||Psi||^2 + varsigma ||Phi||^2) = %.6g must be < 1", cond);
  for (int i = 0; i < p.d; ++i)
    if (!(eps_host[i] > 0)) return fail(RI_EINVAL, "eps[%d] must be positive", i);

  ri_pd_s* P = new (std::nothrow) ri_pd_s;
  if (!P) return fail(RI_ENOMEM, "host allocation failed");
  P->plan = &p;
  P->sara = &S;
  P->prm = q;
  P->alpha = float(q.kappa * q.psi_norm);
  const size_t N = size_t(p.n) * p.n, M = size_t(p.M), KK = size_t(p.K) * p.K;
  int rc = RI_OK;
  auto step = [&](int r) {
    if (rc == RI_OK) rc = r;
  };
  step(ri::dev_alloc(&P->y, M));
  step(ri::dev_alloc(&P->v, M));
  step(ri::dev_alloc(&P->e, M));
  step(ri::dev_alloc(&P->x, N));
  step(ri::dev_alloc(&P->xt, N));
  step(ri::dev_alloc(&P->s, size_t(S.b) * N));
  step(ri::dev_alloc(&P->st, N));
  step(ri::dev_alloc(&P->sum, KK));
  step(ri::dev_alloc(&P->eps, size_t(p.d)));
  step(ri::dev_alloc(&P->stats, 2 * size_t(p.d)));
  step(ri::dev_alloc(&P->shrink, size_t(p.d)));
  step(ri::dev_alloc(&P->mask_dev, size_t(p.d)));
  if (rc == RI_OK && hipStreamCreateWithFlags(&P->side, hipStreamNonBlocking) != hipSuccess)
    rc = fail(RI_EHIP, "side stream creation failed");
  if (rc == RI_OK && (hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming) != hipSuccess ||
                      hipEventCreateWithFlags(&P->ev_join, hipEventDisableTiming) != hipSuccess))
    rc = fail(RI_EHIP, "event creation failed");
  if (rc == RI_OK && hipMemcpyAsync(P->y, y, M * sizeof(float2), hipMemcpyDeviceToDevice, stream) != hipSuccess)
    rc = fail(RI_EHIP, "copy of y failed");
  if (rc == RI_OK &&
      hipMemcpyAsync(P->eps, eps_host, p.d * sizeof(double), hipMemcpyHostToDevice, stream) != hipSuccess)
    rc = fail(RI_EHIP, "copy of eps failed");
  step(rc == RI_OK ? ri::zero_c64(P->v, M, stream) : rc);
  step(rc == RI_OK ? ri::zero_c64(P->e, M, stream) : rc);
  step(rc == RI_OK ? ri::zero_f32(P->x, N, stream) : rc);
  step(rc == RI_OK ? ri::zero_f32(P->xt, N, stream) : rc);
  step(rc == RI_OK ? ri::zero_f32(P->s, size_t(S.b) * N, stream) : rc);
  step(rc == RI_OK ? ri::zero_f32(P->st, N, stream) : rc);
  step(rc == RI_OK ? ri::zero_c64(P->sum, KK, stream) : rc);
  if (rc == RI_OK && hipStreamSynchronize(stream) != hipSuccess) rc = fail(RI_EHIP, "stream sync failed");
  if (rc != RI_OK) {
    ri::destroy_pd(P);
    delete P;
    return rc;
  }
  *out = P;
  return RI_OK;
}

void ri_pd_destroy(ri_pd pd) {
  if (!pd) return;
  ri::destroy_pd(pd);
  delete pd;
}

int ri_pd_step(ri_pd P, const uint8_t* mask, double* stats, hipStream_t stream) {
  if (!P) return fail(RI_EINVAL, "pd is NULL");
  const ri::Plan& p = *P->plan;
  // data-fidelity branch
  RI_STAGE(P, RI_STAGE_FFT_ROWS, stream, ri::fft_forward_rows(p, P->xt, stream));
  RI_STAGE(P, RI_STAGE_FFT_COLS, stream, ri::fft_forward_cols(p, p.grid, stream));
  // fork: the sparsity branch needs only x~ of the previous iteration.  It starts after the
  // forward FFT so that it shares the GPU with the gather / scatter kernels rather than with
  // the column FFT pass, which needs most of a CU's LDS per workgroup (measured faster).
  // Timed runs keep it on the calling stream so that each stage is measured alone.  The
  // data branch is enqueued (and, under capture, recorded) before the sparsity branch: a
  // replayed graph then keeps it on the queue of the forward FFT, so neither the fork nor
  // the join (the sparsity branch ends first) puts a wait between two queues on its path.
  const bool fork = !(P->timing && !ri::capturing(stream));
  if (fork) RI_HIP(hipEventRecord(P->ev_fork, stream));
  // every block active (no mask): the sum is rebuilt from the new duals, reading r only
  // (the degridding launch also zeroes its tiles without visibilities); otherwise the active
  // blocks' changes are added to it
  const bool fresh = mask == nullptr && !p.dde.on();
  RI_STAGE(P, RI_STAGE_DEGRID, stream,
           ri::degrid_residual(p, p.grid, P->y, P->v, P->e, mask, stream, fresh ? P->sum : nullptr));
  RI_STAGE(P, RI_STAGE_BLOCK_NORMS, stream, ri::block_stats(p, mask, P->stats, stats, stream, P->eps, P->shrink));
  if (fresh)
    RI_STAGE(P, RI_STAGE_GRID, stream, ri::grid_project_all(p, P->e, P->v, P->shrink, P->sum, stream, true));
  else
    RI_STAGE(P, RI_STAGE_GRID, stream, ri::grid_project(p, P->e, P->v, P->shrink, mask, P->sum, stream));
  RI_STAGE(P, RI_STAGE_GRID_HALO, stream, ri::grid_halo(p, P->sum, stream));
  RI_STAGE(P, RI_STAGE_IFFT_COLS, stream, ri::fft_adjoint_cols(p, P->sum, stream));
  if (fork) {
    RI_HIP(hipStreamWaitEvent(P->side, P->ev_fork, 0));
    RI_TRY(ri::sparsity_branch(P, P->side));
    RI_HIP(hipEventRecord(P->ev_join, P->side));
    // join, then the adjoint row pass with steps 17-18 fused into its output
    RI_HIP(hipStreamWaitEvent(stream, P->ev_join, 0));
  } else {
    RI_TRY(ri::sparsity_branch(P, stream));
  }
  const ri::PrimalUpdate upd{P->st, P->x, P->xt, float(P->prm.tau), float(P->prm.sigma), float(P->prm.varsigma)};
  RI_STAGE(P, RI_STAGE_IFFT_ROWS, stream, ri::fft_adjoint_rows_update(p, upd, stream));
  P->iter += 1;
  return RI_OK;
}

// The plain form differs from ri_pd_step only in the data term: one degridding and one
// gridding launch per active block (over that block's own tiles) instead of one launch
// over all active blocks; the halo rings of all blocks' launches are merged by one pass
// after the last block.  Everything else (the sparsity branch forked after the forward
// FFT, steps 17-18 fused into the adjoint row pass) is the same, so timing the two forms
// against each other measures what batching the blocks gains.
int ri_pd_step_plain(ri_pd P, const uint8_t* mask_host, double* stats, hipStream_t stream) {
  if (!P) return fail(RI_EINVAL, "pd is NULL");
  const ri::Plan& p = *P->plan;
  std::vector<uint8_t> ones;
  if (!mask_host) {
    ones.assign(p.d, 1);
    mask_host = ones.data();
  }
  RI_HIP(hipMemcpyAsync(P->mask_dev, mask_host, p.d, hipMemcpyHostToDevice, stream));
  RI_STAGE(P, RI_STAGE_FFT_ROWS, stream, ri::fft_forward_rows(p, P->xt, stream));
  RI_STAGE(P, RI_STAGE_FFT_COLS, stream, ri::fft_forward_cols(p, p.grid, stream));
  const bool fork = !(P->timing && !ri::capturing(stream));
  if (fork) {
    RI_HIP(hipEventRecord(P->ev_fork, stream));
    RI_HIP(hipStreamWaitEvent(P->side, P->ev_fork, 0));
    RI_TRY(ri::sparsity_branch(P, P->side));
    RI_HIP(hipEventRecord(P->ev_join, P->side));
  } else {
    RI_TRY(ri::sparsity_branch(P, stream));
  }
  RI_TRY(ri::stage_begin(P, RI_STAGE_DEGRID, stream));
  for (int i = 0; i < p.d; ++i) {
    if (!mask_host[i]) continue;
    RI_TRY(ri::degrid_residual_block(p, i, p.grid, P->y, P->v, P->e, stream));
  }
  RI_TRY(ri::stage_end(P, RI_STAGE_DEGRID, stream));
  RI_STAGE(P, RI_STAGE_BLOCK_NORMS, stream,
           ri::block_stats(p, P->mask_dev, P->stats, stats, stream, P->eps, P->shrink));
  RI_TRY(ri::stage_begin(P, RI_STAGE_GRID, stream));
  RI_TRY(ri::grid_blocks_begin(p, stream));
  for (int i = 0; i < p.d; ++i) {
    if (!mask_host[i]) continue;
    RI_TRY(ri::grid_project_block(p, i, P->e, P->v, P->shrink, P->sum, stream));
  }
  RI_TRY(ri::stage_end(P, RI_STAGE_GRID, stream));
  RI_STAGE(P, RI_STAGE_GRID_HALO, stream, ri::grid_blocks_end(p, P->sum, stream));
  RI_STAGE(P, RI_STAGE_IFFT_COLS, stream, ri::fft_adjoint_cols(p, P->sum, stream));
  if (fork) RI_HIP(hipStreamWaitEvent(stream, P->ev_join, 0));
  const ri::PrimalUpdate upd{P->st, P->x, P->xt, float(P->prm.tau), float(P->prm.sigma), float(P->prm.varsigma)};
  RI_STAGE(P, RI_STAGE_IFFT_ROWS, stream, ri::fft_adjoint_rows_update(p, upd, stream));
  P->iter += 1;
  return RI_OK;
}

int ri_pd_timing(ri_pd P, int enable) {
  if (!P) return fail(RI_EINVAL, "pd is NULL");
  for (auto& r : P->recs) {
    P->pool.push_back(r.a);
    P->pool.push_back(r.b);
  }
  P->recs.clear();
  P->timing = enable != 0;
  return RI_OK;
}

int ri_pd_stage_times(ri_pd P, double* total_ms, int* launches, int n) {
  if (!P || !total_ms || !launches || n < 1) return fail(RI_EINVAL, "bad argument");
  for (int i = 0; i < n; ++i) {
    total_ms[i] = 0.0;
    launches[i] = 0;
  }
  for (auto& r : P->recs) {
    RI_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    RI_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    if (r.stage < n) {
      total_ms[r.stage] += ms;
      launches[r.stage] += 1;
    }
    P->pool.push_back(r.a);
    P->pool.push_back(r.b);
  }
  P->recs.clear();
  return RI_OK;
}

int ri_pd_refresh(ri_pd P, hipStream_t stream) {
  if (!P) return fail(RI_EINVAL, "pd is NULL");
  return ri::refresh_sum(P, stream);
}

int ri_pd_residual(ri_pd P, double* out, hipStream_t stream) {
  if (!P || !out) return fail(RI_EINVAL, "pd and out must not be NULL");
  const ri::Plan& p = *P->plan;
  if (!P->res_e) RI_TRY(ri::dev_alloc(&P->res_e, size_t(p.M)));
  // Eq. 13 needs Phi_i x - y_i at the primal iterate x, for every block: the forward FFT of
  // x into the plan's grid (each step recomputes that grid from x~ first), the residual
  // pass over all items with the norms in fixed order, into scratch so that the step's
  // state (v, the running sum, RI_PD_E) is untouched
  RI_TRY(ri::fft_forward(p, P->x, p.grid, stream));
  RI_TRY(ri::degrid_residual(p, p.grid, P->y, P->v, P->res_e, nullptr, stream));
  return ri::block_stats(p, nullptr, P->stats, out, stream);
}

}  // extern "C"

// ---- Eq. 13 at x without allocating, for callers that cannot allocate ----
//
// The per-item partial norms of the residual pass and the per-block statistics live in
// this file-scope device array instead of memory the library allocates.  Every GPU the
// library runs on holds its own copy until the process ends; its address is taken once per
// device (with that device current) and only that address is passed to kernels.  Calls on
// one GPU share the array: calls that overlap on different streams of one GPU race.
// Nothing in it needs to start at zero (every partial the reduction reads is written first).
namespace ri {
namespace {
constexpr size_t RESID_SCRATCH_DOUBLES = size_t(1) << 19;  // 4 MiB
constexpr int MAX_DEVICES = 64;
}  // namespace
}  // namespace ri

static __device__ __align__(256) double scratch[ri::RESID_SCRATCH_DOUBLES];

namespace ri {
namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

int scratch_for_device(double** out) {
  int dev = 0;
  RI_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(RI_EINVAL, "device %d beyond the %d supported", dev, MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(RI_EHIP, "hipGetSymbolAddress of the residual scratch failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return RI_OK;
}
}  // namespace
}  // namespace ri

extern "C" {

int ri_pd_residual_noalloc(ri_pd P, double* out, hipStream_t stream) {
  if (!P || !out) return fail(RI_EINVAL, "pd and out must not be NULL");
  const ri::Plan& p = *P->plan;
  const size_t nparts = 2 * size_t(ri::PART_WAVES) * p.n_items, need = nparts + 2 * size_t(p.d);
  if (need > ri::RESID_SCRATCH_DOUBLES)
    return fail(RI_EINVAL, "the plan needs %zu doubles of scratch (%d work items, %d blocks); the static scratch "
                "holds %zu", need, p.n_items, p.d, ri::RESID_SCRATCH_DOUBLES);
  double* sc = nullptr;
  RI_TRY(ri::scratch_for_device(&sc));
  double* part = sc;
  double* stats = sc + nparts;
  RI_TRY(ri::fft_forward(p, P->x, p.grid, stream));
  RI_TRY(ri::degrid_norms(p, p.grid, P->y, P->v, part, stream));
  return ri::block_stats(p, nullptr, stats, out, stream, nullptr, nullptr, part);
}

int ri_pd_get(ri_pd P, int which, void* buf, size_t bytes, hipStream_t stream) {
  if (!P || !buf) return fail(RI_EINVAL, "NULL argument");
  const size_t N = size_t(P->plan->n) * P->plan->n;
  const void* src = nullptr;
  size_t need = 0;
  switch (which) {
    case RI_PD_X: src = P->x; need = N * 4; break;
    case RI_PD_XTILDE: src = P->xt; need = N * 4; break;
    case RI_PD_S: src = P->s; need = size_t(P->sara->b) * N * 4; break;
    case RI_PD_V: src = P->v; need = size_t(P->plan->M) * 8; break;
    case RI_PD_E: src = P->e; need = size_t(P->plan->M) * 8; break;
    case RI_PD_W:
      if (!P->wts) return fail(RI_ESTATE, "the solver has no weights (plain l1 prior)");
      src = P->wts;
      need = size_t(P->sara->b) * N * 4;
      break;
    case RI_PD_ITER:
      if (bytes != sizeof(int64_t)) return fail(RI_EINVAL, "ITER needs %zu bytes", sizeof(int64_t));
      *static_cast<int64_t*>(buf) = P->iter;
      return RI_OK;
    default: return fail(RI_EINVAL, "unknown state %d", which);
  }
  if (bytes != need) return fail(RI_EINVAL, "state %d needs %zu bytes, got %zu", which, need, bytes);
  RI_HIP(hipMemcpyAsync(buf, src, bytes, hipMemcpyDeviceToDevice, stream));
  return RI_OK;
}

int ri_pd_set(ri_pd P, int which, const void* buf, size_t bytes, hipStream_t stream) {
  if (!P) return fail(RI_EINVAL, "NULL argument");
  if (which == RI_PD_W && !buf) {  // back to the plain l1 prior
    if (bytes != 0) return fail(RI_EINVAL, "clearing the weights takes buf = NULL and bytes = 0");
    ri::dev_free(P->wts);
    return RI_OK;
  }
  if (!buf) return fail(RI_EINVAL, "NULL argument");
  const size_t N = size_t(P->plan->n) * P->plan->n;
  void* dst = nullptr;
  size_t need = 0;
  switch (which) {
    case RI_PD_X: dst = P->x; need = N * 4; break;
    case RI_PD_XTILDE: dst = P->xt; need = N * 4; break;
    case RI_PD_S: dst = P->s; need = size_t(P->sara->b) * N * 4; break;
    case RI_PD_V: dst = P->v; need = size_t(P->plan->M) * 8; break;
    case RI_PD_W:
      need = size_t(P->sara->b) * N * 4;
      if (bytes != need) return fail(RI_EINVAL, "state %d needs %zu bytes, got %zu", which, need, bytes);
      RI_TRY(ri::ensure_weights(P, stream));
      dst = P->wts;
      break;
    case RI_PD_ITER:
      if (bytes != sizeof(int64_t)) return fail(RI_EINVAL, "ITER needs %zu bytes", sizeof(int64_t));
      P->iter = *static_cast<const int64_t*>(buf);
      return RI_OK;
    default: return fail(RI_EINVAL, "unknown state %d", which);
  }
  if (bytes != need) return fail(RI_EINVAL, "state %d needs %zu bytes, got %zu", which, need, bytes);
  RI_HIP(hipMemcpyAsync(dst, buf, bytes, hipMemcpyDeviceToDevice, stream));
  if (which == RI_PD_V) return ri::refresh_sum(P, stream);
  return RI_OK;
}

int ri_pd_reweight(ri_pd P, double delta, hipStream_t stream) {
  if (!P) return fail(RI_EINVAL, "pd is NULL");
  if (!(delta > 0) || !std::isfinite(delta)) return fail(RI_EINVAL, "delta = %g must be positive and finite", delta);
  RI_TRY(ri::ensure_weights(P, stream));
  const size_t nb = size_t(P->sara->b) * P->plan->n * P->plan->n;
  // Psi^dagger x into the weights' storage, then w = delta / (delta + |.|) in place
  RI_TRY(ri::psi_adj_apply(*P->sara, P->x, P->wts, false, 0.f, stream));
  hipLaunchKernelGGL(ri::k_reweight, dim3(ri::grid_for(nb)), dim3(256), 0, stream, nb, float(delta), P->wts);
  RI_LAUNCH_CHECK();
  return RI_OK;
}

int ri_pd_weighted(ri_pd P, int* out) {
  if (!P || !out) return fail(RI_EINVAL, "NULL argument");
  *out = P->wts != nullptr;
  return RI_OK;
}

int ri_pd_step_vjp(ri_pd P, const uint8_t* mask, const float* x_new, const float* s_new, const float* v_new,
                   const float* r, const double* stats, float* xbar, float* xtbar, float* sbar, float* vbar,
                   double* pgrad, hipStream_t stream) {
  if (!P || !mask || !x_new || !s_new || !v_new || !r || !stats || !xbar || !xtbar || !sbar || !vbar || !pgrad)
    return fail(RI_EINVAL, "NULL argument");
  const ri::Plan& p = *P->plan;
  const ri::Sara& S = *P->sara;
  const int N = p.n * p.n;
  const size_t NB = size_t(S.b) * N;
  constexpr int DOT_PARTS = 512;
  if (!P->vj_z) {
    const size_t nparts = std::max<size_t>(2 * DOT_PARTS, size_t(p.d) * ri::ball_chunks(p));
    RI_TRY(ri::dev_alloc(&P->vj_z, size_t(N)));
    RI_TRY(ri::dev_alloc(&P->vj_st, size_t(N)));
    RI_TRY(ri::dev_alloc(&P->vj_g, size_t(N)));
    RI_TRY(ri::dev_alloc(&P->vj_w, NB));
    RI_TRY(ri::dev_alloc(&P->vj_phiz, size_t(p.M)));
    RI_TRY(ri::dev_alloc(&P->vj_part, nparts));
    RI_TRY(ri::dev_alloc(&P->vj_coef, 2 * size_t(p.d)));
  }
  const double tau = P->prm.tau, sigma = P->prm.sigma, vs = P->prm.varsigma;
  const float2* rr = reinterpret_cast<const float2*>(r);
  float2* vb = reinterpret_cast<float2*>(vbar);
  // steps 17-18
  RI_TRY(ri::vjp_primal(N, x_new, xbar, xtbar, P->vj_z, stream));
  RI_TRY(ri::psi_apply(S, s_new, P->vj_st, stream));
  RI_TRY(ri::phi_adj_apply(p, v_new, P->vj_g, nullptr, stream));
  RI_TRY(ri::vjp_param_grads(N, P->vj_z, P->vj_st, P->vj_g, tau, sigma, vs, P->vj_part, DOT_PARTS, pgrad, stream));
  // step 13 (through s~ = Psi s'), then x~bar = Psi abar
  RI_TRY(ri::psi_adj_apply(S, P->vj_z, P->vj_w, false, 0.f, stream));
  RI_TRY(ri::vjp_clip(NB, s_new, P->alpha, P->wts, P->vj_w, float(-tau * sigma), sbar, stream));
  RI_TRY(ri::psi_apply(S, sbar, xtbar, stream));
  // steps 5-11 (through g = Re Phi^dagger v'), then x~bar += Re Phi_A^dagger rbar
  RI_TRY(ri::phi_apply(p, P->vj_z, reinterpret_cast<float*>(P->vj_phiz), nullptr, stream));
  RI_TRY(ri::vjp_ball(p, mask, vb, P->vj_phiz, float(-tau * vs), rr, stats, P->eps, P->vj_part, P->vj_coef, stream));
  RI_TRY(ri::phi_adj_apply(p, vbar, P->vj_g, mask, stream));
  return ri::axpy(N, 1.f, P->vj_g, xtbar, stream);
}

}  // extern "C"
