"""Writes the oracle's reference gradient of unrolled Algorithm 1 for the GPU test.

Calls only the FP64 oracle and the seeded input generator.  For the 512 x 512 workload
(M = 2^20 in 32 blocks, p = 1, 20 iterations) it stores the noise level, the l2-ball
radii, ||Phi|| from a fixed number of power iterations, and SNR(x^(20)) with its
derivatives with respect to tau and sigma from the reverse sweep, together with central
differences (h = 1e-6) of the same quantity as a check.

    python tests/golden/make_grad_reference.py
"""
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import grad as og  # noqa: E402
from oracle import pd as opd  # noqa: E402
from oracle.measurement import Measurement  # noqa: E402
from oracle.power import phi_norm  # noqa: E402
from oracle.wavelets import Sara  # noqa: E402

NAME = "n512_m1m_d32"
POWER_ITERS = 30
OUT = os.path.dirname(os.path.abspath(__file__))


def main():
    w = synth.WORKLOADS[NAME]
    inp = synth.make_inputs(w)
    meas = Measurement(inp.uv, inp.block_off, (w.n, w.n))
    sara = Sara(w.n)
    t0 = time.time()
    y, sig, eps = synth.add_noise(w, meas.phi(inp.x_true), inp.block_off)
    fn, _ = phi_norm(meas, synth.power_start(w.n, w.seed(synth.SEED_POWER)), tol=0.0, max_it=POWER_ITERS)
    prm = opd.default_params(3.0, fn)
    masks = np.ones((w.iterations, meas.d), bool)
    print(f"setup {time.time() - t0:.0f}s ||Phi||={fn:.6f}", flush=True)
    s_T, dtau, dsig = og.unrolled_gradient(meas, sara, y, eps, prm, masks, inp.x_true)
    print(f"reverse sweep {time.time() - t0:.0f}s: SNR {s_T:.6f} dtau {dtau:.8g} dsigma {dsig:.8g}", flush=True)
    f_tau = lambda t: og.unrolled_snr(meas, sara, y, eps, dataclasses.replace(prm, tau=t), masks, inp.x_true)  # noqa
    f_sig = lambda q: og.unrolled_snr(meas, sara, y, eps, dataclasses.replace(prm, sigma=q), masks, inp.x_true)  # noqa
    fd_tau = og.central_difference(f_tau, prm.tau)
    fd_sig = og.central_difference(f_sig, prm.sigma)
    print(f"central differences {time.time() - t0:.0f}s: dtau {fd_tau:.8g} dsigma {fd_sig:.8g}", flush=True)
    out = {
        "_source": "written by tests/golden/make_grad_reference.py from the FP64 oracle (oracle/) and synth",
        "workload": NAME, "iterations": w.iterations, "sigma_n": sig, "eps": eps.tolist(), "phi_norm": fn,
        "power_iterations": POWER_ITERS, "psi_norm": 3.0, "tau": prm.tau, "sigma": prm.sigma,
        "varsigma": prm.varsigma, "kappa": prm.kappa, "snr": s_T, "dsnr_dtau": dtau, "dsnr_dsigma": dsig,
        "fd_dsnr_dtau": fd_tau, "fd_dsnr_dsigma": fd_sig, "fd_step": 1e-6,
    }
    path = os.path.join(OUT, f"grad_reference_{NAME}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
