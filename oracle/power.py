"""Power method for spectral norms (oracle, FP64).

Sec. V sets sigma = 1/||Psi||_S^2 and varsigma = 1/||Phi||_S^2, with all operator
norms computed beforehand by the power method.  For a linear map A, ||A||_S^2 is the
largest eigenvalue of the self-adjoint A^dagger A; iterating x <- A^dagger A x / ||.||
from a generic start converges to it.  For Phi acting on real images the map iterated
is x -> Re Phi^dagger Phi x, the operator Algorithm 1 actually applies.

Pin: agreement with numpy's SVD of explicitly assembled small matrices.
"""
import numpy as np


def power_method(apply_normal, x0, tol: float = 1e-10, max_it: int = 1000):
    """Return (||A||_S, iterations) given x -> A^dagger A x and a start vector."""
    x = np.asarray(x0, dtype=np.float64)
    x = x / np.linalg.norm(x)
    lam_prev = 0.0
    it = 0
    for it in range(1, max_it + 1):
        y = apply_normal(x)
        lam = float(np.linalg.norm(y))
        if lam == 0.0:
            return 0.0, it
        x = y / lam
        if abs(lam - lam_prev) <= tol * lam:
            break
        lam_prev = lam
    return float(np.sqrt(lam)), it


def phi_norm(meas, x0, **kw):
    return power_method(lambda x: meas.phi_adj_real(meas.phi(x)), x0, **kw)


def psi_norm(sara, x0, **kw):
    return power_method(lambda x: sara.fwd(sara.adj(x)), x0, **kw)
