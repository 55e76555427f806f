"""Quality and convergence diagnostics (oracle, FP64).

* snr: Eq. 15, 20 log10(||x|| / ||x - x_hat||).
* l1_analysis: ||Psi^dagger x||_1, the objective of Eq. 4.
* ball_ratio: ||Phi_i x - y_i|| / eps_i per block, the feasibility of Eq. 6's B_i.
"""
import numpy as np


def snr(x_true, x_hat):
    x_true = np.asarray(x_true, dtype=np.float64)
    err = np.linalg.norm(x_true - np.asarray(x_hat, dtype=np.float64))
    return float(20.0 * np.log10(np.linalg.norm(x_true) / err)) if err > 0 else float("inf")


def l1_analysis(sara, x):
    return float(np.abs(sara.adj(x)).sum())


def ball_ratio(meas, x, y, eps):
    grid = meas.F(meas.Z(x))
    out = np.empty(meas.d)
    for i in range(meas.d):
        lo, hi = meas.block_range(i)
        out[i] = np.linalg.norm(meas.degrid(i, grid) - y[lo:hi]) / eps[i]
    return out
