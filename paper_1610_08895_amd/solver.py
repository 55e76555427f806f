"""Host control flow of Algorithm 1: block selection (step 3), step sizes, the adaptive
probabilities of Sec. IV, and iteration of the GPU step.

Everything numeric inside an iteration runs in libri.so, including the block selection of
the batched form: block i is active when u[t, i] < p_i (Sec. III-B: each block
independently with probability p_i), with p from Eqs. 13-14 for the adaptive schedule,
drawn on the device from uniforms uploaded once (ri_sched_step).  The host only decides
which captured graph to replay.  The plain per-block form draws on the host.
"""
import dataclasses
import math

import numpy as np
import torch

from . import _lib as L
from ._lib import SCHED_ADAPTIVE, SCHED_DRAW, SCHED_REFRESH, SCHED_UPDATE
from .ops import PD, DeviceSchedule, Plan, Sara, probabilities, residual_energy


@dataclasses.dataclass
class Schedule:
    """How blocks are drawn (Sec. III-B, IV).

    kind "uniform": every p_i = p.  kind "fixed": the per-block probabilities p_vec (for
    instance 1 for the low-frequency blocks and 0 for the others).  kind "adaptive": Eq. 14
    from the c_i of Eq. 13 with sum_i p_i = n_nodes, p_min <= p_i <= p_max; c_i starts at
    x = 0, is updated after each step for the blocks that were active (from that step's
    residual, taken at x~), and, with refresh_every = K > 0, is recomputed for every block
    at the primal iterate x every K iterations (one forward FFT and residual pass).
    """

    kind: str = "uniform"
    p: float = 1.0
    n_nodes: float = 0.0
    p_min: float = 0.05
    p_max: float = 0.5
    p_vec: tuple = ()
    refresh_every: int = 0


@dataclasses.dataclass
class Reweight:
    """Reweighted SARA: every `every` iterations the weights of the weighted l1 prior become
    w = delta / (delta + |Psi^dagger x|) at the current x, with delta = delta0, delta0 beta,
    delta0 beta^2, ... (the first `every` iterations use w = 1, the plain prior)."""

    every: int
    delta0: float
    beta: float = 0.5

    def delta(self, t):
        """delta of the reweighting before iteration t, or None if t is not one."""
        if t <= 0 or t % self.every:
            return None
        return self.delta0 * self.beta ** (t // self.every - 1)


def step_sizes(psi_norm, phi_norm, tau=0.49):
    """Sec. V: sigma = 1/||Psi||^2, varsigma = 1/||Phi||^2, tau = 0.49."""
    return tau, 1.0 / psi_norm ** 2, 1.0 / phi_norm ** 2


class Solver:
    def __init__(self, plan: Plan, sara: Sara, y_plan, eps, psi_norm, phi_norm, tau=0.49, kappa=1e-3):
        self.plan, self.sara = plan, sara
        tau, sigma, varsigma = step_sizes(psi_norm, phi_norm, tau)
        self.pd = PD(plan, sara, y_plan, eps, tau, sigma, varsigma, kappa, psi_norm, phi_norm)
        self.eps = np.asarray(eps, dtype=np.float64)
        self.y_plan = y_plan
        self.mask_dev = torch.ones(plan.d, dtype=torch.uint8, device="cuda")
        self._mask_host = np.ones(plan.d, np.uint8)  # what mask_dev holds
        self.stats_dev = torch.zeros(plan.d, 2, dtype=torch.float64, device="cuda")
        self.res_dev = torch.zeros(plan.d, 2, dtype=torch.float64, device="cuda")
        self._graphs = {}

    def initial_energy(self):
        """Eq. 13 at x = 0 (the residual is the data itself)."""
        sq = self.plan.block_sumsq(self.y_plan).cpu().numpy()
        return residual_energy(np.sqrt(sq), self.eps)

    def energy(self):
        """Eq. 13 at the current primal iterate x, for every block."""
        sq = self.pd.residual().cpu().numpy()[:, 1]
        return residual_energy(np.sqrt(sq), self.eps)

    def _capture(self, fn):
        """Capture the kernels fn enqueues (without running them) into a graph."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        it = self.pd.iteration   # the library counts the captured step; restore it
        with torch.cuda.graph(g, stream=s):
            fn()
        torch.cuda.current_stream().wait_stream(s)
        self.pd.iteration = it
        return g

    def capture(self, all_blocks=False):
        """Capture one iteration into a graph for replay: reading self.mask_dev, or with
        every block active (no mask: the step rebuilds the grid sum from the new duals)."""
        mask = None if all_blocks else self.mask_dev
        self._graphs[all_blocks] = self._capture(lambda: self.pd.step(mask, self.stats_dev))
        return self._graphs[all_blocks]

    def _set_mask(self, mask_host):
        m = np.ones(self.plan.d, np.uint8) if mask_host is None else np.ascontiguousarray(mask_host, np.uint8)
        if not np.array_equal(m, self._mask_host):  # a copy only when the mask changes
            self.mask_dev.copy_(torch.from_numpy(m.copy()))
            self._mask_host = m.copy()

    def step(self, mask_host=None, graph=False, plain=False):
        """One iteration; mask_host None means every block active."""
        every = mask_host is None
        if not every:
            self._set_mask(mask_host)
        if plain:
            self.pd.step_plain(None if every else self._mask_host, self.stats_dev)
        elif graph:
            if every not in self._graphs:
                self.capture(every)
            self._graphs[every].replay()
            self.pd.iteration = self.pd.iteration + 1
        else:
            self.pd.step(None if every else self.mask_dev, self.stats_dev)

    def prepare(self, iterations, schedule: Schedule = Schedule(), uniforms=None, masks=None, graph=False,
                seed=0, reweight: Reweight = None):
        """A batched run of `iterations` steps, prepared but not started (see `run`): call
        its step() once per iteration, then history().  Nothing syncs with the host between
        steps."""
        return BatchedRun(self, iterations, schedule, uniforms, masks, graph, seed, reweight)

    def _start_weights(self, reweight):
        if reweight is not None and not self.pd.weighted:  # w = 1: the plain prior, same step
            n, b = self.plan.n, self.sara.b
            self.pd.set(L.RI_PD_W, torch.ones(b, n, n, dtype=torch.float32, device="cuda"))

    def run(self, iterations, schedule: Schedule = Schedule(), uniforms=None, masks=None, refresh=64,
            x_true=None, snr_every=0, graph=False, plain=False, callback=None, seed=0, reweight: Reweight = None):
        """Run `iterations` steps.  Masks come from `masks` (replayed), else from
        `uniforms` (T x d) against the schedule's probabilities, else from uniforms drawn
        here with np.random.default_rng(seed) (only p = 1 without either runs every block
        without drawing); with masks replayed, an adaptive schedule's probabilities are
        still computed and logged.  The batched form selects blocks on the device
        (ri_sched_step), so iterations follow each other without a host round trip; the
        plain form (per-block launches, which need the mask on the host) selects them on
        the host.  `refresh` rebuilds the running sum of G_i^dagger v_i every that many
        steps.  `reweight` runs reweighted SARA (weights refreshed every `every` steps).
        Returns a history dict (masks and probabilities per iteration, SNR)."""
        if plain:
            T = int(iterations)
            p_fixed, uniforms, masks, _ = _draws(self.plan.d, T, schedule, uniforms, masks, seed)
            return self._run_host(T, schedule, p_fixed, uniforms, masks, refresh, x_true, snr_every, callback,
                                  reweight)
        r = self.prepare(iterations, schedule, uniforms, masks, graph, seed, reweight)
        snrs = []
        for t in range(r.T):
            r.step()
            if refresh and (t + 1) % refresh == 0:
                self.pd.refresh()
            if x_true is not None and snr_every and ((t + 1) % snr_every == 0 or t + 1 == r.T):
                snrs.append((t + 1, snr(x_true, self.x())))
            if callback is not None:
                callback(t, self)
        h = r.history()
        h["snr"] = snrs
        return h

    def _run_host(self, T, schedule, p_fixed, uniforms, masks, refresh, x_true, snr_every, callback, reweight):
        """The plain form's loop: blocks drawn on the host, one step at a time."""
        d = self.plan.d
        adaptive = p_fixed is None
        c = self.initial_energy() if adaptive else None
        hist = {"masks": [], "p": [], "snr": []}
        self._start_weights(reweight)
        for t in range(T):
            if reweight is not None and reweight.delta(t) is not None:
                self.pd.reweight(reweight.delta(t))
            if adaptive and schedule.refresh_every and t > 0 and t % schedule.refresh_every == 0:
                c = self.energy()
            p = probabilities(c, schedule.n_nodes, schedule.p_min, schedule.p_max)[0] if adaptive else p_fixed
            if masks is not None:
                mask = masks[t]
            elif uniforms is not None:
                mask = (uniforms[t] < p).astype(np.uint8)
            else:
                mask = np.ones(d, np.uint8)
            self.step(mask, plain=True)
            if adaptive:
                st = self.stats_dev.cpu().numpy()
                act = np.flatnonzero(mask)
                if act.size:  # an empty active set leaves every c_i as it was
                    c[act] = residual_energy(np.sqrt(st[act, 1]), self.eps[act])
            if refresh and (t + 1) % refresh == 0:
                self.pd.refresh()
            hist["masks"].append(mask)
            hist["p"].append(p)
            if x_true is not None and snr_every and ((t + 1) % snr_every == 0 or t + 1 == T):
                hist["snr"].append((t + 1, snr(x_true, self.x())))
            if callback is not None:
                callback(t, self)
        return hist

    def x(self):
        return self.pd.get(0).cpu().numpy().astype(np.float64)


def _draws(d, T, schedule, uniforms, masks, seed):
    """(p_fixed or None for adaptive, uniforms, masks, every_block) of a run."""
    if schedule.kind == "fixed":
        p_fixed = np.asarray(schedule.p_vec, dtype=np.float64)
        if p_fixed.shape != (d,) or np.any(p_fixed < 0) or np.any(p_fixed > 1):
            raise ValueError("p_vec must hold d probabilities in [0, 1]")
    elif schedule.kind == "uniform":
        p_fixed = np.full(d, float(schedule.p))
    elif schedule.kind == "adaptive":
        p_fixed = None
    else:
        raise ValueError(f"unknown schedule kind {schedule.kind!r}")
    every_block = masks is None and uniforms is None and p_fixed is not None and bool(np.all(p_fixed >= 1.0))
    if masks is None and uniforms is None and not every_block:
        uniforms = np.random.default_rng(seed).random((T, d))
    if masks is not None:
        masks = np.asarray(masks, dtype=np.uint8)[:T]
        if masks.shape != (T, d):
            raise ValueError(f"masks must be ({T}, {d})")
    if uniforms is not None:
        uniforms = np.asarray(uniforms, dtype=np.float64)[:T]
        if uniforms.shape != (T, d):
            raise ValueError(f"uniforms must be ({T}, {d})")
    return p_fixed, uniforms, masks, every_block


class BatchedRun:
    """Iterations of the batched step with the block selection on the device.

    Each step() enqueues the draw of iteration t (ri_sched_step: Eq. 13 update from the
    last step's statistics and Eq. 14 for the adaptive schedule, then u[t, i] < p_i, or the
    replayed mask) and the step reading that mask; with refresh_every = K the draw of every
    K-th iteration is preceded by Eq. 13 at x for all blocks (ri_pd_residual).  With
    graph=True the two sequences are captured once each and replayed."""

    def __init__(self, solver, iterations, schedule, uniforms, masks, graph, seed, reweight=None):
        self.sol, self.T, self.graph = solver, int(iterations), graph
        self.reweight = reweight
        solver._start_weights(reweight)
        d = solver.plan.d
        p_fixed, uniforms, masks, every_block = _draws(d, self.T, schedule, uniforms, masks, seed)
        adaptive = p_fixed is None
        self.K = schedule.refresh_every if adaptive else 0
        self.sched = None
        if not every_block:
            self.sched = DeviceSchedule(d, self.T, solver.eps, solver.stats_dev, solver.res_dev,
                                        u=uniforms if masks is None else None, masks=masks, p_fixed=p_fixed,
                                        c0=solver.initial_energy() if adaptive else None, n_nodes=schedule.n_nodes,
                                        p_min=schedule.p_min, p_max=schedule.p_max)
        self.mask = self.sched.mask if self.sched is not None else None  # None: every block, no draw
        self.flags = SCHED_DRAW | ((SCHED_UPDATE | SCHED_ADAPTIVE) if adaptive else 0)
        if self.K:
            solver.pd.residual(solver.res_dev)  # its scratch is allocated outside any capture
        self.graphs = {}
        self.t = 0

    def _body(self):
        if self.sched is not None:
            self.sched.step(self.flags)
        self.sol.pd.step(self.mask, self.sol.stats_dev)

    def _body_refresh(self):  # Eq. 13 recomputed for every block at x before the draw
        self.sol.pd.residual(self.sol.res_dev)
        self.sched.step(SCHED_REFRESH | SCHED_ADAPTIVE | SCHED_DRAW)
        self.sol.pd.step(self.mask, self.sol.stats_dev)

    def step(self):
        if self.reweight is not None and self.reweight.delta(self.t) is not None:
            self.sol.pd.reweight(self.reweight.delta(self.t))  # between two steps, outside the graphs
        exact = bool(self.K) and self.t > 0 and self.t % self.K == 0
        fn = self._body_refresh if exact else self._body
        if self.graph:
            if exact not in self.graphs:
                self.graphs[exact] = self.sol._capture(fn)
            self.graphs[exact].replay()
            self.sol.pd.iteration = self.sol.pd.iteration + 1
        else:
            fn()
        self.t += 1

    def history(self):
        """Masks and probabilities of the iterations run so far (one copy to the host)."""
        d = self.sol.plan.d
        if self.sched is None:
            return {"masks": list(np.ones((self.t, d), np.uint8)), "p": list(np.ones((self.t, d)))}
        return {"masks": list(self.sched.mask_log.cpu().numpy()[:self.t]),
                "p": list(self.sched.p_log.cpu().numpy()[:self.t])}


def snr(x_true, x_hat):
    """Eq. 15 on the host (diagnostic)."""
    x_true = np.asarray(x_true, dtype=np.float64)
    err = np.linalg.norm(x_true - np.asarray(x_hat, dtype=np.float64))
    return float(20 * math.log10(np.linalg.norm(x_true) / err)) if err > 0 else float("inf")
