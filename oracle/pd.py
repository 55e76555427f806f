"""Algorithm 1, randomised forward-backward primal-dual (oracle, FP64).

One iteration follows the algorithm's steps in order and notation:

  step 3        the active set A is given (a boolean mask over the d blocks)
  step 4        b~ = F Z x~
  step 5        b_i = M_i b~                                  (i in A)
  steps 7-9     v_i = v_i + G_i b_i - P_{B_i}(v_i + G_i b_i);  v~_i = G_i^dagger v_i
  step 11       blocks outside A keep v_i and v~_i
  step 13       s = s + Psi^dagger x~ - S_{kappa ||Psi||}(s + Psi^dagger x~)
  step 14       s~ = Psi s
  step 17       x = P_C(x - tau (sigma s~ + varsigma Z^dagger F^dagger sum_i M_i^dagger v~_i))
  step 18       x~ = 2 x_new - x_old

with x, x~, s, v_i, v~_i all zero at the start (the paper lists them as given without
values).  v~_i is kept on block i's kN_i cells, as in Eq. 8.

Per active block the iteration also reports ||v_i + G_i b_i - y_i|| (the norm the
projection uses) and ||G_i b_i - y_i|| = ||Phi_i x~ - y_i||.  The second one drives
Eq. 13 in ``run_adaptive``: c_i is refreshed from it when block i is active and kept
otherwise, and at the start is computed from x = 0 (the paper leaves open when c_i is
evaluated; Eq. 13 itself asks for Phi_i x at the current iterate).  With refresh_every = K,
every K iterations c_i is also recomputed for all blocks exactly as Eq. 13 states, from
||Phi_i x - y_i|| at the current primal iterate x (``residual_norms``).

Pins: invariants every iteration (x >= 0, |s| <= alpha, v_i = 0 whenever the block's
residual is inside its ball), the x = 0 special case, mask-all-ones equal to the
deterministic run, inactive blocks untouched, and convergence to the solution of the
constrained problem found by an independent general-purpose solver on a tiny case.
"""
import dataclasses

import numpy as np

from .parallel import pmap
from .probs import adaptive_probabilities, residual_energy
from .prox import data_dual_update, proj_pos, sparsity_dual_update


@dataclasses.dataclass
class Params:
    tau: float
    sigma: float
    varsigma: float
    kappa: float
    psi_norm: float

    @property
    def alpha(self):
        """Soft-threshold size kappa ||Psi||_S that replaces gamma / sigma (Sec. III)."""
        return self.kappa * self.psi_norm

    def condition(self, phi_norm):
        """tau (sigma ||Psi||^2 + varsigma ||Phi||^2), which must stay below 1 (Sec. III-B)."""
        return self.tau * (self.sigma * self.psi_norm ** 2 + self.varsigma * phi_norm ** 2)


def default_params(psi_norm, phi_norm, tau=0.49, kappa=1e-3):
    """Sec. V: sigma = 1/||Psi||^2, varsigma = 1/||Phi||^2, tau = 0.49, kappa = 1e-3."""
    return Params(tau=tau, sigma=1.0 / psi_norm ** 2, varsigma=1.0 / phi_norm ** 2,
                  kappa=kappa, psi_norm=psi_norm)


@dataclasses.dataclass
class State:
    x: np.ndarray
    xt: np.ndarray
    s: np.ndarray
    v: list
    vt: list
    t: int = 0
    w: np.ndarray | None = None  # per-coefficient weights of a weighted l1 prior (None: all 1)

    def copy(self):
        return State(self.x.copy(), self.xt.copy(), self.s.copy(),
                     [a.copy() for a in self.v], [a.copy() for a in self.vt], self.t,
                     None if self.w is None else self.w.copy())


def init_state(meas, sara):
    n = meas.ny
    return State(
        x=np.zeros((meas.ny, meas.nx)),
        xt=np.zeros((meas.ny, meas.nx)),
        s=np.zeros((sara.b, n, n)),
        v=[np.zeros(hi - lo, dtype=np.complex128) for lo, hi in map(meas.block_range, range(meas.d))],
        vt=[np.zeros(meas.cells(i).size, dtype=np.complex128) for i in range(meas.d)],
    )


def split_blocks(meas, y):
    return [np.asarray(y[lo:hi]) for lo, hi in map(meas.block_range, range(meas.d))]


def iteration(meas, sara, y_blocks, eps, prm: Params, st: State, active):
    """One pass of steps 3-18.  Returns stats[d, 2] (NaN rows for inactive blocks)."""
    d = meas.d
    active = np.asarray(active, dtype=bool)
    stats = np.full((d, 2), np.nan)

    b_full = meas.F(meas.Z(st.xt))                                  # step 4

    def data_block(i):                                              # steps 5-10, block i
        b_i = meas.Mi(i, b_full)                                    # step 5
        Gb = meas.Gi(i, b_i)
        r0 = np.linalg.norm(st.v[i] + Gb - y_blocks[i])
        r1 = np.linalg.norm(Gb - y_blocks[i])
        v_i = data_dual_update(st.v[i], Gb, y_blocks[i], eps[i])    # step 8
        return r0, r1, v_i, meas.GiH(i, v_i)                        # step 9

    act = np.flatnonzero(active)
    for i, (r0, r1, v_i, vt_i) in zip(act, pmap(data_block, act)):  # the par-for over A
        stats[i] = r0, r1
        st.v[i], st.vt[i] = v_i, vt_i
    # step 11: v_i, v~_i of inactive blocks are left as they are

    thr = prm.alpha if st.w is None else prm.alpha * st.w
    st.s = sparsity_dual_update(st.s, sara.adj(st.xt), thr)         # step 13
    s_tilde = sara.fwd(st.s)                                        # step 14

    acc = np.zeros(meas.Ky * meas.Kx, dtype=np.complex128)          # sum_i M_i^dagger v~_i
    for i in range(d):
        acc[meas.cells(i)] += st.vt[i]
    g = meas.ZH(meas.FH(acc.reshape(meas.Ky, meas.Kx)))
    x_new = proj_pos(st.x - prm.tau * (prm.sigma * s_tilde + prm.varsigma * g))  # step 17
    st.xt = 2.0 * x_new - st.x                                      # step 18
    st.x = x_new
    st.t += 1
    return stats


def run(meas, sara, y, eps, prm: Params, masks, x_true=None, state=None, callback=None):
    """Iterate with the given per-iteration active masks (shape T x d)."""
    from .metrics import snr

    yb = split_blocks(meas, y)
    st = init_state(meas, sara) if state is None else state
    hist = []
    for t, mask in enumerate(np.asarray(masks, dtype=bool)):
        stats = iteration(meas, sara, yb, eps, prm, st, mask)
        rec = {"t": st.t, "active": int(mask.sum())}
        if x_true is not None:
            rec["snr"] = snr(x_true, st.x)
        hist.append(rec)
        if callback is not None:
            callback(st, stats, rec)
    return st, hist


def residual_norms(meas, x, y_blocks):
    """||Phi_i x - y_i|| for every block i (the residual of Eq. 13 at x)."""
    b_full = meas.F(meas.Z(x))
    return np.array([np.linalg.norm(meas.Gi(i, meas.Mi(i, b_full)) - y_blocks[i]) for i in range(meas.d)])


def run_adaptive(meas, sara, y, eps, prm: Params, uniforms, n_nodes, p_min, p_max, x_true=None,
                 refresh_every=0):
    """Algorithm 1 with Eq. 14 probabilities; block i is active at iteration t iff
    uniforms[t, i] < p_i^(t).  With refresh_every = K > 0, before iteration t (t > 0,
    t a multiple of K) every c_i is recomputed from Eq. 13 at the current x.  Returns
    (state, history, masks, probabilities)."""
    from .metrics import snr

    yb = split_blocks(meas, y)
    st = init_state(meas, sara)
    # c_i at x = 0: ||y_i|| against eps_i
    c = residual_energy([np.linalg.norm(b) for b in yb], eps)
    masks, probs, hist = [], [], []
    for t, u in enumerate(np.asarray(uniforms)):
        if refresh_every and t > 0 and t % refresh_every == 0:
            c = residual_energy(residual_norms(meas, st.x, yb), eps)
        p, _ = adaptive_probabilities(c, n_nodes, p_min, p_max)
        mask = u < p
        stats = iteration(meas, sara, yb, eps, prm, st, mask)
        act = np.flatnonzero(mask)
        c[act] = residual_energy(stats[act, 1], eps[act])
        masks.append(mask)
        probs.append(p)
        rec = {"t": st.t, "active": int(mask.sum())}
        if x_true is not None:
            rec["snr"] = snr(x_true, st.x)
        hist.append(rec)
    return st, hist, np.array(masks), np.array(probs)
