"""Reweighted SARA: the weighted l1 prior and its outer reweighting loop (oracle, FP64).

The paper regularises with the SARA prior of Carrillo et al. (2012), which it cites
without restating.  The reading used here: the weighted analysis prior ||W Psi^dagger x||_1,
W = diag(w) with w_k in (0, 1], replaces ||Psi^dagger x||_1 in the problem Algorithm 1
solves; its proximity operator is soft-thresholding with one threshold per coefficient, so
step 13 becomes

    s = (s + Psi^dagger x~) - S_{alpha w}(s + Psi^dagger x~) = clip(s + Psi^dagger x~, -alpha w, alpha w).

The weights come from the current primal iterate,

    w_k = delta / (delta + |[Psi^dagger x]_k|),

the derivative of the log penalty delta log(delta + |c|) at |c| (the weighted l1 norm with
these weights majorises that penalty to first order), and delta shrinks by a factor beta
at every reweighting.  ``run_reweighted`` runs Algorithm 1 with the given masks, starting
with w = 1 (the plain prior), and replaces w every K iterations, keeping the state (x, s,
v) as the warm start of the next weighted problem.

Pins: weighted soft-thresholding equals a brute-force minimisation of
1/2 (z - u)^2 + alpha w |z| per coefficient; w = 1 gives the unweighted step bitwise;
the weights equal central differences of the log penalty; w = 1 at c = 0, 1/2 at |c| = delta.
"""
import numpy as np

from .pd import init_state, iteration, split_blocks


def weights(sara, x, delta):
    """w_k = delta / (delta + |[Psi^dagger x]_k|), shape (b, n, n)."""
    if not delta > 0:
        raise ValueError("delta must be positive")
    return delta / (delta + np.abs(sara.adj(x)))


def run_reweighted(meas, sara, y, eps, prm, masks, every, delta0, beta, x_true=None):
    """Algorithm 1 with reweighting every `every` iterations (delta0, delta0 beta, ...).
    Returns (state, history, deltas used)."""
    from .metrics import snr

    yb = split_blocks(meas, y)
    st = init_state(meas, sara)
    hist, deltas = [], []
    delta = float(delta0)
    for t, mask in enumerate(np.asarray(masks, dtype=bool)):
        if t > 0 and t % every == 0:
            st.w = weights(sara, st.x, delta)
            deltas.append(delta)
            delta *= beta
        iteration(meas, sara, yb, eps, prm, st, mask)
        rec = {"t": st.t}
        if x_true is not None:
            rec["snr"] = snr(x_true, st.x)
        hist.append(rec)
    return st, hist, deltas
