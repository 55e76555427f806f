"""Adaptive block probabilities against fixed ones (Sec. IV, and the experiment of Sec. V
with n = 4 nodes for d = 16 blocks): SNR against iterations for

* p_i = 1 (no randomisation, all 16 blocks every iteration);
* uniform p_i = 0.25 (4 blocks on average) and p_i = 0.4 (6.4 on average);
* Eq. 14 with sum_i p_i = 4, p_max = 0.5 and p_min in {0.05, 0.1, 0.2}, c_i of Eq. 13
  refreshed for every block at the primal iterate every K iterations;
* only the 4 lowest-frequency blocks (p_i = 1 there, 0 for the others);

on the synthetic problem of workload n256_m320k_d16 (256 x 256 sky, M = 5N Gaussian u-v
points cut into 16 equal radial blocks, 20 dB input SNR, radii at the chi-square 0.99
quantile).  With another workload the same ratios hold: n = d / 4 nodes, the lowest d / 4
blocks for the low-frequency run.  Every iteration runs in the library; the schedules
differ only in the masks, which are drawn from seeded uniforms.
`python -m paper_1610_08895_amd.study [--workload NAME]` prints one JSON line per schedule.
"""
import argparse
import json
import time

import numpy as np
import torch

import synth

from . import Plan, Sara
from .solver import Schedule, Solver, snr

WORKLOAD = "n256_m320k_d16"


def schedules(d, refresh_every=10):
    """The compared schedules, by label: n = d / 4 nodes on average, as 4 of 16 in Sec. V."""
    n = d / 4.0
    p_low = np.zeros(d)
    p_low[: d // 4] = 1.0  # blocks are radial and sorted by radius: the first ones are the low frequencies
    return {
        "p=1": Schedule("uniform", p=1.0),
        "uniform 0.25": Schedule("uniform", p=0.25),
        "uniform 0.4": Schedule("uniform", p=0.4),
        "adaptive pmin=0.05": Schedule("adaptive", n_nodes=n, p_min=0.05, p_max=0.5, refresh_every=refresh_every),
        "adaptive pmin=0.1": Schedule("adaptive", n_nodes=n, p_min=0.1, p_max=0.5, refresh_every=refresh_every),
        "adaptive pmin=0.2": Schedule("adaptive", n_nodes=n, p_min=0.2, p_max=0.5, refresh_every=refresh_every),
        "low frequencies only": Schedule("fixed", p_vec=tuple(p_low)),
    }


def setup(workload=WORKLOAD):
    """Plan, dictionary, noisy data and operator norm of the study's workload."""
    w = synth.WORKLOADS[workload]
    inp = synth.make_inputs(w)
    plan = Plan(w.n, inp.uv, inp.block_off)
    order = plan.order()
    x_true = torch.tensor(inp.x_true, dtype=torch.float32, device="cuda")
    y0 = plan.phi(x_true).cpu().numpy()
    y0_user = np.empty_like(y0)
    y0_user[order] = y0
    y_user, _, eps = synth.add_noise(w, y0_user.astype(np.complex128), inp.block_off)
    y_plan = torch.tensor(y_user[order], dtype=torch.complex64, device="cuda")
    sara = Sara(w.n, 4)
    x0 = torch.tensor(synth.power_start(w.n, w.seed(synth.SEED_POWER)), dtype=torch.float32, device="cuda")
    phi_norm, _ = plan.norm(x0, max_it=200, rtol=1e-6)
    return dict(w=w, inp=inp, plan=plan, sara=sara, y_plan=y_plan, eps=eps, phi_norm=phi_norm)


def run_schedule(S, sched, iterations, seed, snr_every=10):
    """One run: SNR trajectory, mean active blocks and visibilities per iteration."""
    plan, w = S["plan"], S["w"]
    sol = Solver(plan, S["sara"], S["y_plan"], S["eps"], 3.0, S["phi_norm"])
    u = synth.activity_uniforms(iterations, plan.d, seed)
    t0 = time.time()
    hist = sol.run(iterations, sched, uniforms=u, x_true=S["inp"].x_true, snr_every=snr_every)
    torch.cuda.synchronize()
    secs = time.time() - t0
    masks = np.array(hist["masks"], dtype=bool)
    sizes = np.diff(S["inp"].block_off)
    return {"snr": hist["snr"], "final_snr": snr(S["inp"].x_true, sol.x()),
            "mean_active": float(masks.sum(1).mean()),
            "mean_visibilities": float((masks * sizes[None, :]).sum(1).mean()),
            "seconds": secs}


def iterations_to(traj, level):
    """First recorded iteration whose SNR reaches `level` (None if never)."""
    for t, v in traj:
        if v >= level:
            return t
    return None


def run_study(iterations=600, seeds=(1,), labels=None, log=print, workload=WORKLOAD):
    S = setup(workload)
    out = {}
    for label, sched in schedules(S["plan"].d).items():
        if labels is not None and label not in labels:
            continue
        runs = [run_schedule(S, sched, iterations, 1000 + s) for s in seeds]
        ts = [t for t, _ in runs[0]["snr"]]
        mean = np.mean([[v for _, v in r["snr"]] for r in runs], axis=0)
        out[label] = {"snr": list(zip(ts, mean.tolist())), "final_snr": float(mean[-1]),
                      "mean_active": float(np.mean([r["mean_active"] for r in runs])),
                      "mean_visibilities": float(np.mean([r["mean_visibilities"] for r in runs])),
                      "seconds": float(np.mean([r["seconds"] for r in runs]))}
        if log:
            log(f"{label}: final SNR {out[label]['final_snr']:.2f} dB, "
                f"{out[label]['mean_active']:.2f} blocks per iteration")
    if "p=1" in out:
        ref = out["p=1"]["final_snr"]
        for r in out.values():
            r["iters_to"] = {f: iterations_to(r["snr"], f * ref) for f in (0.9, 0.95, 0.99)}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--iterations", type=int, default=600)
    ap.add_argument("--seeds", type=int, default=3, help="mask draws averaged per schedule")
    ap.add_argument("--workload", default=WORKLOAD, choices=sorted(synth.WORKLOADS))
    args = ap.parse_args()
    res = run_study(args.iterations, tuple(range(args.seeds)), log=lambda m: print(m, flush=True),
                    workload=args.workload)
    for label, r in res.items():
        print(json.dumps({"schedule": label, **{k: v for k, v in r.items() if k != "snr"},
                          "snr_every_10": [round(v, 3) for _, v in r["snr"]]}), flush=True)


if __name__ == "__main__":
    main()
