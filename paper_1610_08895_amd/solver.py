"""Host control flow of Algorithm 1: block selection (step 3), step sizes, the adaptive
probabilities of Sec. IV, and iteration of the GPU step.

Everything numeric inside an iteration runs in libri.so.  The host only turns uniform
variates into the active set (block i is active when u[t, i] < p_i, Sec. III-B: each
block independently with probability p_i), evaluates Eqs. 13-14 through the library's
host entry points, and moves the d-byte mask and the d x 2 block statistics.
"""
import dataclasses
import math

import numpy as np
import torch

from .ops import PD, Plan, Sara, probabilities, residual_energy


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
        self.stats_dev = torch.zeros(plan.d, 2, dtype=torch.float64, device="cuda")
        self._graph = None

    def initial_energy(self):
        """Eq. 13 at x = 0 (the residual is the data itself)."""
        sq = self.plan.block_sumsq(self.y_plan).cpu().numpy()
        return residual_energy(np.sqrt(sq), self.eps)

    def energy(self):
        """Eq. 13 at the current primal iterate x, for every block."""
        sq = self.pd.residual().cpu().numpy()[:, 1]
        return residual_energy(np.sqrt(sq), self.eps)

    def capture(self):
        """Capture one iteration (reading self.mask_dev) into a graph for replay."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        it = self.pd.iteration   # capture records the kernels without running them
        with torch.cuda.graph(g, stream=s):
            self.pd.step(self.mask_dev, self.stats_dev)
        torch.cuda.current_stream().wait_stream(s)
        self.pd.iteration = it
        self._graph = g
        return g

    def step(self, mask_host=None, graph=False, plain=False):
        if mask_host is not None:
            self.mask_dev.copy_(torch.from_numpy(np.ascontiguousarray(mask_host, dtype=np.uint8)))
        else:
            self.mask_dev.fill_(1)
        if plain:
            self.pd.step_plain(mask_host, self.stats_dev)
        elif graph:
            if self._graph is None:
                self.capture()
            self._graph.replay()
            self.pd.iteration = self.pd.iteration + 1
        else:
            self.pd.step(self.mask_dev, self.stats_dev)

    def run(self, iterations, schedule: Schedule = Schedule(), uniforms=None, masks=None, refresh=64,
            x_true=None, snr_every=0, graph=False, plain=False, callback=None):
        """Run `iterations` steps.  Masks come from `masks` (replayed), else from
        `uniforms` (T x d) against the schedule's probabilities; with masks replayed, an
        adaptive schedule's probabilities are still computed and logged.  `refresh` rebuilds
        the running sum of G_i^dagger v_i every that many steps.  Returns a history dict."""
        d = self.plan.d
        adaptive = schedule.kind == "adaptive"
        c = self.initial_energy() if adaptive else None
        if schedule.kind == "fixed":
            p_fixed = np.asarray(schedule.p_vec, dtype=np.float64)
            if p_fixed.shape != (d,) or np.any(p_fixed < 0) or np.any(p_fixed > 1):
                raise ValueError("p_vec must hold d probabilities in [0, 1]")
        elif schedule.kind not in ("uniform", "adaptive"):
            raise ValueError(f"unknown schedule kind {schedule.kind!r}")
        hist = {"masks": [], "p": [], "snr": []}
        for t in range(iterations):
            if adaptive and schedule.refresh_every and t > 0 and t % schedule.refresh_every == 0:
                c = self.energy()
            if adaptive:
                p, _ = probabilities(c, schedule.n_nodes, schedule.p_min, schedule.p_max)
            elif schedule.kind == "fixed":
                p = p_fixed
            else:
                p = np.full(d, schedule.p)
            if masks is not None:
                mask = np.asarray(masks[t], dtype=np.uint8)
            else:
                mask = (uniforms[t] < p).astype(np.uint8) if uniforms is not None else np.ones(d, np.uint8)
            self.step(mask, graph=graph, plain=plain)
            if adaptive:
                st = self.stats_dev.cpu().numpy()
                act = np.flatnonzero(mask)
                if act.size:  # an empty active set leaves every c_i as it was
                    c[act] = residual_energy(np.sqrt(st[act, 1]), self.eps[act])
            if refresh and (t + 1) % refresh == 0:
                self.pd.refresh()
            hist["masks"].append(mask)
            hist["p"].append(p)
            if x_true is not None and snr_every and ((t + 1) % snr_every == 0 or t + 1 == iterations):
                hist["snr"].append((t + 1, snr(x_true, self.x())))
            if callback is not None:
                callback(t, self)
        return hist

    def x(self):
        return self.pd.get(0).cpu().numpy().astype(np.float64)


def snr(x_true, x_hat):
    """Eq. 15 on the host (diagnostic)."""
    x_true = np.asarray(x_true, dtype=np.float64)
    err = np.linalg.norm(x_true - np.asarray(x_hat, dtype=np.float64))
    return float(20 * math.log10(np.linalg.norm(x_true) / err)) if err > 0 else float("inf")
