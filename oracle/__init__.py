"""FP64 CPU oracle for the per-iteration hot path of the randomised primal-dual solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, deliberately unoptimised
reference of what the method computes, written from Onose, Carrillo, McEwen & Wiaux,
"A randomised primal-dual algorithm for distributed radio-interferometric imaging"
(2016).  Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
may import it.  It shares no code, table or constant generator with the GPU library;
the only thing both sides share is the seeded input generator (``synth``).

Contents, each citing the passage it follows:
  kaiser_bessel  interpolation kernel and its Fourier transform (Eq. 3's G and Z)
  measurement    Phi = G M F Z per data block, its adjoint, and a direct NUDFT (Eqs. 2, 3, 8)
  dde            DDE-aware G (Eq. 1's D folded into G's kernels, Sec. II) and its direct NUDFT
  wavelets       Daubechies filters and the SARA dictionary Psi (Sec. III)
  prox           Eqs. 10, 11, 12 and the Moreau forms of Algorithm 1 steps 8 and 13
  probs          Eqs. 13 and 14
  power          power method for operator norms (Sec. V)
  pd             Algorithm 1
  reweight       the weighted l1 prior of reweighted SARA and its reweighting loop
  metrics        Eq. 15 and objective / feasibility diagnostics
  parallel       optional thread pool for the par-for over blocks and the per-basis loop

Every function is pinned by tests marked ``not gpu`` against something other than
itself (closed forms, brute force, textbook routines, invariants); see the pin list
at the top of each module.
"""
