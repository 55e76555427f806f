"""Reverse-mode derivatives of Algorithm 1 (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

With the active sets fixed, the T-iteration map (tau, sigma) -> x^(T) of Algorithm 1 is
piecewise smooth: every step is linear except the three proximity operators of Sec. III,
used through their Moreau forms.  Their vector-Jacobian products (complex values taken as
pairs of reals, inner product Re <a, b>):

* step 8, r -> r max(0, 1 - eps/||r||) with r = v + G b - y: for ||r|| > eps the
  Jacobian is (1 - eps/||r||) I + eps r r^T / ||r||^3 (symmetric), and 0 inside the ball;
* step 13, a -> clip(a, -alpha, alpha) (a = s + Psi^dagger x~): 1 where |a| < alpha;
* step 17, z -> max(Re z, 0) (Eq. 12): 1 where z > 0.

``unrolled_gradient`` runs the iteration forward keeping what the backward sweep needs and
then propagates adjoints of (x, x~, s, v) back through every step to d x^(T) / d(tau,
sigma) contracted with dL/dx^(T) for L = SNR (Eq. 15).  varsigma = 1/||Phi||^2 and alpha
are held fixed; the start x = x~ = s = v = 0 does not depend on the parameters.

Pins: each VJP against central differences of its forward map; the gradient of
1/2 ||Phi x - y||^2 (whose closed form is Re Phi^dagger (Phi x - y)) against central
differences of the objective; the unrolled gradient against central differences of the
unrolled SNR.
"""
import numpy as np

from .metrics import snr
from .pd import Params, init_state, iteration, split_blocks

LN10 = np.log(10.0)


def vjp_ball_shrink(r, eps, g):
    """VJP of r -> r max(0, 1 - eps / ||r||) (Algorithm 1 step 8) at r, cotangent g."""
    nr = np.linalg.norm(r)
    if nr <= eps:
        return np.zeros_like(g)
    rg = np.real(np.vdot(r, g))  # r^T g with complex numbers as pairs of reals
    return (1.0 - eps / nr) * g + eps * r * rg / nr ** 3


def vjp_clip(a, alpha, g):
    """VJP of a -> clip(a, -alpha, alpha) (step 13's Moreau form)."""
    return np.where(np.abs(a) < alpha, g, 0.0)


def vjp_pos(z, g):
    """VJP of z -> max(z, 0) (Eq. 12 on real images)."""
    return np.where(z > 0, g, 0.0)


def snr_grad(x_true, x):
    """d SNR / d x for Eq. 15: (20 / ln 10) (x_true - x) / ||x_true - x||^2."""
    e = np.asarray(x_true, float) - np.asarray(x, float)
    return (20.0 / LN10) * e / np.dot(e.ravel(), e.ravel())


def data_fit_grad(meas, x, y):
    """Gradient of 1/2 ||Phi x - y||^2 over real images: Re Phi^dagger (Phi x - y)."""
    return meas.phi_adj_real(meas.phi(x) - y)


def unrolled_snr(meas, sara, y, eps, prm: Params, masks, x_true):
    """SNR of x^(T) after len(masks) iterations from the zero start."""
    yb = split_blocks(meas, y)
    st = init_state(meas, sara)
    for m in np.asarray(masks, bool):
        iteration(meas, sara, yb, eps, prm, st, m)
    return snr(x_true, st.x)


def unrolled_gradient(meas, sara, y, eps, prm: Params, masks, x_true):
    """Returns (SNR(x^(T)), dSNR/dtau, dSNR/dsigma) by the reverse sweep."""
    masks = np.asarray(masks, bool)
    yb = split_blocks(meas, y)
    st = init_state(meas, sara)
    tape = []
    for m in masks:
        rec = {"mask": m, "x_old": st.x.copy(), "xt_old": st.xt.copy(), "s_old": st.s.copy(),
               "v_old": [a.copy() for a in st.v]}
        # the step-8 residuals r_i = v_i + G_i b_i - y_i of the active blocks
        b_full = meas.F(meas.Z(st.xt))
        rec["r"] = {i: st.v[i] + meas.Gi(i, meas.Mi(i, b_full)) - yb[i] for i in np.flatnonzero(m)}
        iteration(meas, sara, yb, eps, prm, st, m)
        rec["x_new"] = st.x.copy()
        rec["s_new"] = st.s.copy()
        rec["v_new"] = [a.copy() for a in st.v]
        tape.append(rec)
    s_T = snr(x_true, st.x)

    tau, sigma, vs, alpha = prm.tau, prm.sigma, prm.varsigma, prm.alpha
    offs = [meas.block_range(i) for i in range(meas.d)]
    xbar = snr_grad(x_true, st.x)
    xtbar = np.zeros_like(st.x)
    sbar = np.zeros_like(st.s)
    vbar = np.zeros(meas.M, dtype=np.complex128)
    dtau = dsigma = 0.0
    for rec in reversed(tape):
        # steps 17-18: x' = max(z, 0), z = x - tau (sigma Psi s' + varsigma g), x~' = 2 x' - x
        stilde = sara.fwd(rec["s_new"])
        g = meas.phi_adj_real(np.concatenate(rec["v_new"]))
        zbar = vjp_pos(rec["x_new"], xbar + 2.0 * xtbar)
        x_adj = zbar - xtbar
        dtau -= float(np.sum(zbar * (sigma * stilde + vs * g)))
        dsigma -= float(tau * np.sum(zbar * stilde))
        s_tot = sbar - tau * sigma * sara.adj(zbar)            # s~ = Psi s'
        v_tot = vbar - tau * vs * meas.phi(zbar)               # g = Re Phi^dagger v'
        # step 13: s' = clip(a, +-alpha), a = s + Psi^dagger x~ (the Moreau form a - S_alpha(a)
        # rounds clipped entries to alpha(1 +- ulp), so the mask is taken on a itself)
        abar = vjp_clip(rec["s_old"] + sara.adj(rec["xt_old"]), alpha, s_tot)
        s_adj = abar
        xt_adj = sara.fwd(abar)
        # steps 5-11: active blocks v_i' = shrink(v_i + G_i M_i F Z x~ - y_i), others kept
        v_adj = v_tot.copy()
        rbar = np.zeros(meas.M, dtype=np.complex128)
        for i, r in rec["r"].items():
            lo, hi = offs[i]
            rb = vjp_ball_shrink(r, eps[i], v_tot[lo:hi])
            rbar[lo:hi] = rb
            v_adj[lo:hi] = rb
        if rec["r"]:
            xt_adj = xt_adj + meas.phi_adj_real(rbar, blocks=list(rec["r"].keys()))
        xbar, xtbar, sbar, vbar = x_adj, xt_adj, s_adj, v_adj
    return s_T, dtau, dsigma


def central_difference(f, p, h=1e-6):
    """(f(p + h) - f(p - h)) / (2 h)."""
    return (f(p + h) - f(p - h)) / (2.0 * h)
