"""Writes the oracle's reference runs of Algorithm 1 used by the GPU SNR-parity tests.

Calls only the FP64 oracle and the seeded input generator.  For each workload it stores
the noise level, the l2-ball radii, ||Phi|| from a fixed number of power iterations, the
SNR trajectory, and for randomised schedules the block masks the oracle drew, so that the
GPU run can replay them.

    python tests/golden/make_pd_references.py n256_m128k_d16                  # both schedules, 500 it
    python tests/golden/make_pd_references.py n1024_m4m_d64 200 p1            # p = 1, 200 iterations
    python tests/golden/make_pd_references.py n1024_m4m_d64 200 adaptive16    # Eq. 14, sum p = 16

With labels given, only those schedules run, and their records are merged into the
workload's file (under a lock, so several labels can run as separate processes); each
record carries its own iteration count.
"""
import fcntl
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import pd as opd  # noqa: E402
from oracle.measurement import Measurement  # noqa: E402
from oracle.metrics import snr  # noqa: E402
from oracle.power import phi_norm  # noqa: E402
from oracle.wavelets import Sara  # noqa: E402

POWER_ITERS = 30
OUT = os.path.dirname(os.path.abspath(__file__))


def pack_masks(masks):
    return ["".join("1" if b else "0" for b in row) for row in np.asarray(masks, bool)]


def main(name, iterations=None, labels=None):
    w = synth.WORKLOADS[name]
    T = iterations or w.iterations
    inp = synth.make_inputs(w)
    meas = Measurement(inp.uv, inp.block_off, (w.n, w.n))
    sara = Sara(w.n)
    t0 = time.time()
    y, sig, eps = synth.add_noise(w, meas.phi(inp.x_true), inp.block_off)
    fn, _ = phi_norm(meas, synth.power_start(w.n, w.seed(synth.SEED_POWER)), tol=0.0, max_it=POWER_ITERS)
    prm = opd.default_params(3.0, fn)
    print(f"{name}: setup {time.time() - t0:.0f}s ||Phi||={fn:.6f}", flush=True)
    runs = {}
    for label, kind, kw in w.prob_schemes:
        if labels and label not in labels:
            continue
        t1 = time.time()
        rec = {"kind": kind, "params": kw, "snr": [], "iterations": T}
        every = 10

        def cb(st, stats, r):
            if r["t"] % every == 0 or r["t"] == T:
                rec["snr"].append([r["t"], r["snr"]])
                print(f"  {label} t={r['t']} snr={r['snr']:.4f} ({time.time() - t1:.0f}s)", flush=True)

        if kind == "uniform" and kw["p"] >= 1.0:
            masks = np.ones((T, meas.d), bool)
            opd.run(meas, sara, y, eps, prm, masks, x_true=inp.x_true, callback=cb)
        elif kind == "uniform":
            u = synth.activity_uniforms(T, meas.d, w.seed(synth.SEED_MASKS))
            masks = u < kw["p"]
            rec["masks"] = pack_masks(masks)
            opd.run(meas, sara, y, eps, prm, masks, x_true=inp.x_true, callback=cb)
        else:
            u = synth.activity_uniforms(T, meas.d, w.seed(synth.SEED_MASKS))
            st, hist, masks, probs = opd.run_adaptive(meas, sara, y, eps, prm, u, kw["n_nodes"], kw["p_min"],
                                                      kw["p_max"], x_true=inp.x_true)
            rec["snr"] = [[h["t"], h["snr"]] for h in hist if h["t"] % every == 0 or h["t"] == T]
            rec["masks"] = pack_masks(masks)
            rec["p_first"] = probs[0].tolist()
        runs[label] = rec
    out = {
        "_source": "written by tests/golden/make_pd_references.py from the FP64 oracle (oracle/) and synth",
        "workload": name, "iterations": T, "sigma_n": sig, "eps": eps.tolist(), "phi_norm": fn,
        "power_iterations": POWER_ITERS, "psi_norm": 3.0, "tau": prm.tau, "kappa": prm.kappa, "runs": runs,
    }
    path = os.path.join(OUT, f"pd_reference_{name}.json")
    with open(path + ".lock", "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        if labels and os.path.exists(path):
            with open(path) as f:
                old = json.load(f)
            for k in ("sigma_n", "phi_norm"):
                assert abs(old[k] - out[k]) <= 1e-12 * abs(out[k]), f"{k} differs from the stored file"
            old["runs"].update(runs)
            old["iterations"] = max(r.get("iterations", old["iterations"]) for r in old["runs"].values())
            out = old
        with open(path, "w") as f:
            json.dump(out, f)
    os.remove(path + ".lock")
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else None, sys.argv[3:] or None)
