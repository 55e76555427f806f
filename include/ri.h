/*
 * ri.h - C ABI of the MI355X (gfx950) library for the per-iteration hot path of the
 * randomised primal-dual (PD) forward-backward solver for radio-interferometric imaging
 * of Onose, Carrillo, McEwen & Wiaux, "A randomised primal-dual algorithm for
 * distributed radio-interferometric imaging" (2016).
 *
 * Conventions shared by every call
 * --------------------------------
 * Return value: RI_OK (0) or a negative RI_E* code.  ri_last_error() then returns a
 *   message for the calling thread.  Nothing aborts and no exception crosses the ABI.
 * Pointers: arguments documented "device" are device pointers owned by the caller; the
 *   library never frees them and only touches them in work it enqueues on `stream`.
 *   Arguments documented "host" are read (or written) before the call returns.
 * Streams: every operator call only enqueues work on `stream` (a hipStream_t; NULL is
 *   the null stream) and returns without synchronising, unless documented otherwise.
 *   Calls on one handle that overlap on different streams race.
 * Images: n x n row-major float32, pixel (r, c) at centred coordinates
 *   (l_y, l_x) = (r - n/2, c - n/2).  n is a power of two, 16 <= n <= 2048.
 * Visibilities: complex float32, interleaved (re, im), M of them, stacked by data block
 *   as y = [y_1; ...; y_d] (Eq. 8).  Inside each block the library sorts visibilities
 *   into its own *plan order* (by grid tile and cell, and within a work item of one tile
 *   same-cell pairs and LDS banks); every device visibility array
 *   passed to or returned by the library is in plan order.  ri_plan_order() returns the
 *   map so the caller can permute its data once (see ri_plan_permute).
 * Masks: uint8 per block, nonzero = active (the set A of Algorithm 1, step 3).  A NULL
 *   mask means all blocks.
 * u-v coordinates: (u, v) pairs in rad/px, u pairing with the column (x) axis; a
 *   visibility measures sum_p x_p exp(-i (u l_x + v l_y)) (the sign of Eq. 1).
 */
#ifndef RI_H_
#define RI_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  RI_OK = 0,
  RI_EINVAL = -1, /* bad argument (size, range, NULL, unsupported option)      */
  RI_ENOMEM = -2, /* a device or host allocation failed                         */
  RI_EHIP = -3,   /* a HIP runtime call failed (message has the HIP error)      */
  RI_ESTATE = -4  /* handle in the wrong state for the call                     */
};

typedef struct ri_plan_s* ri_plan;
typedef struct ri_sara_s* ri_sara;
typedef struct ri_pd_s* ri_pd;

/* Message of the last failing call on this thread ("" if none).  Owned by the library. */
const char* ri_last_error(void);
/* Library version, major * 10000 + minor * 100 + patch. */
int ri_version(void);
/* HIP runtime version the library is linked against (hipRuntimeGetVersion). */
int ri_hip_runtime_version(int* out);

/* ------------------------------------------------------------------------------------
 * Measurement operator Phi = G M F Z (Eq. 3 with the block split of Eq. 8)
 *
 * Z zero-pads the n x n image onto a K x K grid, K = 2n (oversampling k = 4 grid points
 * per pixel, Sec. V) and pre-compensates the interpolation with
 * S = 1/(phi_hat(l_y/K) phi_hat(l_x/K)); F is the unnormalised 2D DFT; G interpolates each
 * visibility from the J x J grid cells floor(kappa) - J/2 + 1 + j, kappa = u K / (2 pi),
 * with the Kaiser-Bessel weights phi(t) = I0(beta sqrt(1 - (2t/J)^2)) / I0(beta); M_i is
 * the set of grid cells block i touches.
 * ------------------------------------------------------------------------------------ */

/* Tuning knobs of a plan.  Zero fields take the defaults. */
typedef struct {
  int tile;           /* grid tile side in cells (16, 32 or 64; default 32)            */
  int bin;            /* max visibilities per work item (<= 1024; default 1024)        */
  int fft_panel;      /* reserved, must be 0 (the column FFT passes' panel width is fixed
                         per grid size: 8 columns at K = 2048, measured best)             */
  int persistent_wgs; /* workgroups of the gather/scatter kernels (default: one per unit) */
  int slice_vis;      /* most visibilities one gridding workgroup accumulates for one
                         tile (default and negative: never split); a denser tile is
                         split over several workgroups whose partial tiles the halo
                         pass merges in a fixed order                                   */
} ri_tuning;

/*
 * Build a plan.  uv_host: M (u, v) float32 pairs in rad/px (host, user order);
 * block_off_host: d+1 offsets, block i = rows [block_off[i], block_off[i+1]) (host);
 * every block must be nonempty.  J must be 8; beta <= 0 selects 2.34 J.  tune may be NULL.
 * The coordinates are packed (cell and 20-bit fraction of the 2n x 2n grid, FP64) and sorted
 * on the device (a stable radix sort by block, tile and cell); the work items are cut on the
 * host.  Allocates device memory (and, while it runs, about 40 bytes per visibility of
 * scratch); synchronises `stream` before returning.
 * Errors: RI_EINVAL (n not a power of two in [16, 2048], M < 1, d outside [1, 4096], empty block,
 * offsets not increasing, non-finite u-v, tile not 16, 32 or 64, bin above 1024, fft_panel not
 * 0), RI_ENOMEM, RI_EHIP.
 */
int ri_plan_create(ri_plan* out, int n, int64_t M, const float* uv_host, int d,
                   const int64_t* block_off_host, int J, double beta, const ri_tuning* tune,
                   hipStream_t stream);
void ri_plan_destroy(ri_plan plan);
/* Sizes of a plan (any pointer may be NULL). */
int ri_plan_info(ri_plan plan, int* n, int64_t* M, int* d, int* K, int* tile, int* n_items);
/* order_host[k] = user index of the visibility at plan position k (host, M int64). */
int ri_plan_order(ri_plan plan, int64_t* order_host);
/* Permute complex visibilities between user and plan order on the device.
 * to_plan != 0: dst[k] = src[order[k]]; else dst[order[k]] = src[k].  src != dst. */
int ri_plan_permute(ri_plan plan, const float* src, float* dst, int to_plan, hipStream_t stream);

/*
 * Direction-dependent effects in G (Eq. 1's D(l, u), which Sec. II folds into the kernels
 * of G).  The DDE of visibility m is band limited on the oversampled grid,
 * D_m(l) = sum_{p,q=-h..h} d_m[q][p] exp(-2 pi i (p l_x + q l_y) / K), so its row of G becomes
 * the jd x jd kernel d_m convolved with the Kaiser-Bessel kernel: (8 + 2h)^2 complex weights
 * per visibility, built on the device by this call and stored (S^2 * 8 bytes per
 * visibility, S = 8 + 2h).  From then on ri_phi, ri_phi_adj, ri_phi_norm and the Algorithm 1
 * steps of solvers on this plan use the DDE-aware G (the adjoint with conjugate weights).
 * d_host: M * jd * jd complex float32 (host, user order of the visibilities; per
 * visibility row-major [q + h][p + h], q along v / rows, p along u / columns).
 * jd odd, 1 <= jd <= 7; jd = 0 with d_host = NULL removes the DDEs (plain G again).
 * Synchronises `stream`.  A graph captured before the call keeps the G it was captured with.
 * Errors: RI_EINVAL (NULL plan, jd out of range, non-finite taps), RI_ENOMEM, RI_EHIP.
 */
int ri_plan_dde(ri_plan plan, int jd, const float* d_host, hipStream_t stream);

/* y_i = Phi_i x for every block i with mask[i] != 0 (Algorithm 1 steps 4-5 and G_i b_i).
 * x: device n*n float32; y: device M complex (plan order); rows of inactive blocks are
 * left untouched.  mask: device d uint8 or NULL. */
int ri_phi(ri_plan plan, const float* x, float* y, const uint8_t* mask, hipStream_t stream);

/* x = Re sum_{i: mask[i]} Phi_i^dagger y_i = Re Z^dagger F^dagger sum_i M_i^dagger G_i^dagger y_i
 * (the image-domain adjoint used by Algorithm 1 step 17, real part as in Eq. 12).
 * y: device M complex (plan order); x: device n*n float32 (overwritten). */
int ri_phi_adj(ri_plan plan, const float* y, float* x, const uint8_t* mask, hipStream_t stream);

/* out[i] = ||y_i||_2^2 for every block i, accumulated in FP64 (y: device M complex, plan
 * order; out: device d float64).  With y the data this is Eq. 13's residual at x = 0. */
int ri_block_sumsq(ri_plan plan, const float* y, double* out, hipStream_t stream);

/* ||Phi||_S on real images: power iteration on x -> Re Phi^dagger Phi x (Sec. V), with
 * FP64 reductions.  x0: device n*n float32 start vector (caller-drawn; overwritten by the
 * last iterate).  Stops when the eigenvalue estimate changes by <= rtol relatively or
 * after max_it iterations.  Synchronises `stream`.  norm_host, iters_host: host outputs
 * (iters_host may be NULL). */
int ri_phi_norm(ri_plan plan, float* x0, int max_it, double rtol, double* norm_host,
                int* iters_host, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * SARA sparsity dictionary Psi (Sec. III): the concatenation, without normalisation, of
 * the Dirac basis and the Daubechies db1..db8 wavelet bases, each a `levels`-level
 * periodic separable 2D DWT, so Psi Psi^dagger = 9 I and ||Psi||_S = 3.  Coefficients:
 * float32 [b][n][n], basis 0 = Dirac, basis k = db_k; inside a basis the Mallat layout
 * (per level, the m x m top-left region holds [[LL, low-y/high-x], [high-y/low-x, HH]]).
 * Analysis of one level: a[k] = sum_j h[j] x[(2k+j) mod m], detail with
 * g[j] = (-1)^j h[2N-1-j], the minimum-phase Daubechies lowpass h with sum h = sqrt 2.
 * ------------------------------------------------------------------------------------ */

/* bases: bit 0 = Dirac, bit k (1..8) = db_k; 0 selects all nine.  n a power of two with
 * 2^levels <= n <= 4096, 1 <= levels <= 6.  Errors: RI_EINVAL, RI_ENOMEM, RI_EHIP. */
int ri_sara_create(ri_sara* out, int n, int levels, uint32_t bases, hipStream_t stream);
void ri_sara_destroy(ri_sara sara);
/* Number of bases b. */
int ri_sara_bases(ri_sara sara, int* b);
/* x = Psi s (s: device b*n*n float32; x: device n*n float32, overwritten). */
int ri_psi(ri_sara sara, const float* s, float* x, hipStream_t stream);
/* s = Psi^dagger x (x: device n*n float32; s: device b*n*n float32, overwritten). */
int ri_psi_adj(ri_sara sara, const float* x, float* s, hipStream_t stream);
/* ||Psi||_S by power iteration on x -> Psi Psi^dagger x; see ri_phi_norm. */
int ri_psi_norm(ri_sara sara, float* x0, int max_it, double rtol, double* norm_host,
                int* iters_host, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * Algorithm 1: randomised forward-backward primal-dual iterations.
 * ------------------------------------------------------------------------------------ */

typedef struct {
  double tau;       /* primal step (Sec. V: 0.49)                                     */
  double sigma;     /* sparsity dual step (1/||Psi||^2)                                */
  double varsigma;  /* data dual step (1/||Phi||^2)                                    */
  double kappa;     /* normalised soft-threshold (1e-3); threshold = kappa ||Psi||_S  */
  double psi_norm;  /* ||Psi||_S                                                      */
  double phi_norm;  /* ||Phi||_S, used only to check tau(sigma||Psi||^2 + varsigma||Phi||^2) < 1 */
} ri_pd_params;

/*
 * Create a solver state.  y: device M complex (plan order), copied; eps_host: d radii
 * eps_i of the balls B_i (host).  x, x~, s, v, v~ start at zero.  The plan and the
 * dictionary must outlive the solver.  Errors: RI_EINVAL (sizes differ, eps_i <= 0,
 * tau, sigma, varsigma or kappa <= 0, convergence condition >= 1), RI_ENOMEM, RI_EHIP.
 */
int ri_pd_create(ri_pd* out, ri_plan plan, ri_sara sara, const float* y, const double* eps_host,
                 const ri_pd_params* params, hipStream_t stream);
void ri_pd_destroy(ri_pd pd);

/*
 * One iteration, steps 3-18, for the active blocks mask[i] != 0 (device d uint8,
 * NULL = all), all active blocks of uneven size in one persistent launch per operator.
 * stats: device d x 2 float64 output; for active block i, stats[2i] = ||v_i + G_i b_i - y_i||^2
 * (the projection's residual) and stats[2i+1] = ||G_i b_i - y_i||^2 = ||Phi_i x~ - y_i||^2
 * (drives Eq. 13); inactive rows are set to NaN.  May be NULL.  With mask NULL every block is
 * active and sum_i M_i^dagger v~_i is rebuilt from the new v_i (the gridding then reads r
 * and writes v, 24 bytes per visibility); with a mask the active blocks' changes are added
 * to the kept sum.
 * Graph capture: the call only enqueues kernels (no allocation, no host sync, no memset);
 * the mask and stats pointers are baked into a captured graph.
 */
int ri_pd_step(ri_pd pd, const uint8_t* mask, double* stats, hipStream_t stream);

/* The same iteration in the plain form: one degridding and one gridding launch per active
 * block (over that block's own tiles; one halo pass merges all blocks' tile borders after
 * the last one) instead of one launch over all active blocks.  The rest of the step is
 * the batched step's.  mask_host: host d uint8 (NULL = all), copied to the device. */
int ri_pd_step_plain(ri_pd pd, const uint8_t* mask_host, double* stats, hipStream_t stream);

/* Rebuild sum_i M_i^dagger v~_i from the stored v (all blocks).  The batched and plain steps
 * update that sum by differences in FP32; calling this every few tens of iterations bounds
 * the accumulated rounding.  Enqueue-only (graph-capturable). */
int ri_pd_refresh(ri_pd pd, hipStream_t stream);

/* Sec. IV, Eq. 13 at the current primal iterate x (all blocks, active or not): a forward
 * FFT of x and one residual pass over all visibilities.  out: device d x 2 float64;
 * out[2i+1] = ||Phi_i x - y_i||^2 (FP64, fixed summation order), out[2i] =
 * ||v_i + Phi_i x - y_i||^2.  The solver state is not changed (the residual goes to scratch
 * that the first call allocates, M complex values); the plan's FFT grid is overwritten,
 * which the next step recomputes anyway.  Enqueue-only after the first call.
 * Errors: RI_EINVAL (NULL pd or out), RI_ENOMEM, RI_EHIP. */
int ri_pd_residual(ri_pd pd, double* out, hipStream_t stream);

/* For callers that cannot allocate (code under graph capture, tight serving loops,
 * harnesses that forbid allocation): ri_pd_residual without any allocation.  The same
 * out[2i] and out[2i+1], with the per-item partial norms and per-block sums kept in a
 * static device array of 4 MiB (2^19 doubles) per GPU instead of library-allocated
 * memory, and the residual itself not stored.  Needs 8 * n_items + 2 d doubles of it
 * (n_items from ri_plan_info); larger plans are rejected with RI_EINVAL.  The array is
 * shared by every call on one GPU: calls that overlap on one GPU race.  The plan's FFT grid
 * is overwritten, as by ri_pd_residual.  Enqueue-only; errors: RI_EINVAL, RI_EHIP. */
int ri_pd_residual_noalloc(ri_pd pd, double* out, hipStream_t stream);

/* Stages of one iteration, for per-stage timing (each stage is one kernel launch in the
 * batched step; the plain step times all per-block launches of a stage together). */
enum {
  RI_STAGE_FFT_ROWS = 0,    /* F Z x~, row pass (step 4)                                    */
  RI_STAGE_FFT_COLS = 1,    /* F Z x~, column pass (step 4)                                 */
  RI_STAGE_DEGRID = 2,      /* G_i b_i, residuals, FP64 partial norms (steps 5, 8)          */
  RI_STAGE_BLOCK_NORMS = 3, /* per-block reduction of the partial norms, statistics out     */
  RI_STAGE_GRID = 4,        /* l2-ball shrink, G_i^dagger update, tile interiors (8, 9, 11) */
  RI_STAGE_GRID_HALO = 5,   /* tile halos of the G_i^dagger update                         */
  RI_STAGE_IFFT_COLS = 6,   /* Z^dagger F^dagger, column pass (step 17)                     */
  RI_STAGE_IFFT_ROWS = 7,   /* Z^dagger F^dagger, row pass (step 17); in ri_pd_step it also
                               applies steps 17-18 to its output                          */
  RI_STAGE_PSI_ADJ = 8,     /* Psi^dagger x~ and dual clip, all levels (step 13)            */
  RI_STAGE_PSI_SYNTH = 9,   /* s~ = Psi s, all levels (step 14)                             */
  RI_STAGE_UPDATE = 10,     /* not recorded: both forms apply steps 17-18 in IFFT_ROWS      */
  RI_STAGE_COUNT = 11
};

/* Enable (1) or disable (0) per-stage timing: while enabled, each ri_pd_step /
 * ri_pd_step_plain outside graph capture records a HIP event pair around every stage
 * on the calling stream, and runs the sparsity branch on that stream too (instead of
 * concurrently), so every stage is timed alone.  Clears earlier records. */
int ri_pd_timing(ri_pd pd, int enable);
/* Sum of the recorded durations (ms) and the number of records per stage, for the first
 * n stages; waits for the recorded events, then clears the records (host outputs). */
int ri_pd_stage_times(ri_pd pd, double* total_ms, int* launches, int n);

/* State access for checkpoint / resume and inspection.  which: */
enum {
  RI_PD_X = 0,     /* n*n float32                                   */
  RI_PD_XTILDE = 1,/* n*n float32                                   */
  RI_PD_S = 2,     /* b*n*n float32                                 */
  RI_PD_V = 3,     /* M complex float32, plan order                 */
  RI_PD_ITER = 4,  /* int64 iteration counter (host buffer)         */
  RI_PD_E = 5,     /* M complex float32: r = v_i + G_i b_i - y_i (the argument of step 8's
                      projection, v_i before the step) of the last step's active blocks
                      (read only)                                   */
  RI_PD_W = 6      /* b*n*n float32 weights w_k of the weighted l1 prior (layout of S);
                      set allocates them on first use, set with buf = NULL and bytes = 0
                      returns to the plain prior; get fails with RI_ESTATE without them */
};
/* Copy state `which` to/from buf (device, or host for RI_PD_ITER), `bytes` long.
 * ri_pd_set recomputes sum_i M_i^dagger v~_i from the stored v when V is set. */
int ri_pd_get(ri_pd pd, int which, void* buf, size_t bytes, hipStream_t stream);
int ri_pd_set(ri_pd pd, int which, const void* buf, size_t bytes, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * Reweighted SARA (the SARA prior the paper cites, Sec. II-III): the weighted analysis
 * prior ||W Psi^dagger x||_1, W = diag(w), whose proximity operator thresholds each
 * coefficient at alpha w_k, so step 13 becomes s = clip(s + Psi^dagger x~, -alpha w, alpha w).
 * ------------------------------------------------------------------------------------ */

/* w_k = delta / (delta + |[Psi^dagger x]_k|) from the current primal iterate x (the
 * derivative of the log penalty delta log(delta + |c|), which the weighted l1 norm
 * majorises), stored as RI_PD_W; every later step uses them.  The first call (or the first
 * set of RI_PD_W) allocates b*n*n floats, initialised to 1; later calls only enqueue.  A
 * graph captured before the weights existed keeps the plain prior.
 * Errors: RI_EINVAL (NULL pd, delta not positive and finite), RI_ENOMEM, RI_EHIP. */
int ri_pd_reweight(ri_pd pd, double delta, hipStream_t stream);
/* *out = 1 if the solver uses weights (RI_PD_W), else 0 (host output). */
int ri_pd_weighted(ri_pd pd, int* out);

/* ------------------------------------------------------------------------------------
 * Differentiation of unrolled iterations (masks fixed; the map (tau, sigma) -> x is then
 * piecewise smooth, the kinks being those of the proximity operators of Sec. III)
 * ------------------------------------------------------------------------------------ */

/* Reverse (vector-Jacobian) sweep of one ri_pd_step with the pd's tau, sigma, varsigma
 * and alpha = kappa ||Psi||.  All pointers device.  From the forward step: mask (d, as
 * given to it), x_new (n*n, x after it), s_new (b*n*n, s after it), v_new (M complex, v
 * after it), r (M complex, RI_PD_E after it), stats (d x 2 FP64, as it returned them).  Adjoints, updated in place: on entry xbar, xtbar, sbar,
 * vbar (n*n, n*n, b*n*n, M complex) hold dL/d(x, x~, s, v) after the step, on return
 * dL/d(x, x~, s, v) before it; pgrad[0], pgrad[1] (FP64) are incremented by the step's
 * own contributions to dL/dtau and dL/dsigma.  Vector-Jacobian products used: clip ->
 * 1{|a| < alpha}; step-8 shrink -> (1 - eps/||r||) I + eps r r^T / ||r||^3 outside the
 * ball (complex as pairs of reals), 0 inside; positivity -> 1{x_new > 0}.  The first
 * call allocates the sweep's scratch (about 10 n*n floats and M complex values).
 * Errors: RI_EINVAL (NULL pointer), RI_ENOMEM, RI_EHIP. */
int ri_pd_step_vjp(ri_pd pd, const uint8_t* mask, const float* x_new, const float* s_new, const float* v_new,
                   const float* r, const double* stats, float* xbar, float* xtbar, float* sbar, float* vbar,
                   double* pgrad, hipStream_t stream);

/* ------------------------------------------------------------------------------------
 * Adaptive probabilities (Sec. IV)
 * ------------------------------------------------------------------------------------ */

/* Eq. 13 on the host: c[i] = max(resid_norm[i] - eps[i], 0)^2 / eps[i]^2. */
int ri_residual_energy(const double* resid_norm, const double* eps, int d, double* c_out);

/* Eq. 14 on the host: p_i = p_min + min((n - d p_min) c_i / sum c + a, p_max - p_min), with
 * a >= 0 the smallest value giving sum p = n; p_i = n/d when sum c = 0.
 * Needs 0 < p_min <= n/d <= p_max <= 1 and c_i >= 0 (RI_EINVAL otherwise).  a_out may be NULL. */
int ri_probs(const double* c, int d, double n_nodes, double p_min, double p_max, double* p_out,
             double* a_out);

/* ------------------------------------------------------------------------------------
 * Block selection on the device (Algorithm 1 step 3; Sec. III-B; Sec. IV Eqs. 13-14)
 *
 * One call enqueues one single-workgroup kernel, so a step and its draw can be captured
 * together in a graph and replayed with no host round trip between iterations.  All
 * pointers are device pointers owned by the caller; every field the flags do not use
 * may be NULL / 0.
 * ------------------------------------------------------------------------------------ */
typedef struct {
  int d;                     /* number of blocks, 1 <= d <= 4096                          */
  int64_t T;                 /* rows of u / masks / logs; iteration t uses row t mod T     */
  const double* u;           /* T x d float64 U[0,1) variates: block i is active at t iff
                                u[t][i] < p_i (Sec. III-B: independent draws)              */
  const uint8_t* masks;      /* T x d masks to replay instead of drawing (or NULL)         */
  const double* p_fixed;     /* d probabilities when RI_SCHED_ADAPTIVE is not set (NULL: 1) */
  double* c;                 /* d Eq. 13 energies c_i (state of the adaptive rule)          */
  const double* stats_step;  /* d x 2 float64 stats of the last ri_pd_step (RI_SCHED_UPDATE) */
  const double* stats_x;     /* d x 2 float64 output of ri_pd_residual (RI_SCHED_REFRESH)   */
  const double* eps;         /* d radii eps_i                                             */
  double n_nodes;            /* Eq. 14: sum_i p_i = n_nodes                                */
  double p_min, p_max;       /* Eq. 14 bounds, 0 < p_min <= n_nodes/d <= p_max <= 1        */
  int64_t* counter;          /* iteration index t; RI_SCHED_DRAW reads it and adds 1       */
  uint8_t* mask;             /* d: on entry the last step's mask (RI_SCHED_UPDATE reads it);
                                RI_SCHED_DRAW overwrites it with the mask of iteration t   */
  double* p_log;             /* T x d or NULL: RI_SCHED_DRAW stores p of iteration t in row t mod T */
  uint8_t* mask_log;         /* T x d or NULL: the drawn mask, likewise                    */
} ri_sched;

enum {
  RI_SCHED_UPDATE = 1,   /* c_i <- Eq. 13 of stats_step[2i+1] (= ||Phi_i x~ - y_i||^2) for the
                            blocks of the last step's mask; skipped while counter == 0    */
  RI_SCHED_REFRESH = 2,  /* c_i <- Eq. 13 of stats_x[2i+1] (= ||Phi_i x - y_i||^2) for all i */
  RI_SCHED_ADAPTIVE = 4, /* p_i from c by Eq. 14 (p_i = n/d when sum c = 0); else p_fixed    */
  RI_SCHED_DRAW = 8      /* mask of iteration t = counter from row t mod T, then counter += 1 */
};

/* Apply the flagged parts in the order UPDATE, REFRESH, then (with DRAW) the
 * probabilities and the draw.  Sums over blocks are formed in a fixed order, so equal
 * inputs give bitwise equal results.  Errors: RI_EINVAL (NULL a, d out of range, unknown
 * flags, a pointer a flag needs is NULL, T < 1 with DRAW, Eq. 14 bounds violated with
 * ADAPTIVE), RI_EHIP.  c must hold finite values >= 0. */
int ri_sched_step(const ri_sched* a, int flags, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* RI_H_ */
