"""Proximity operators of Sec. III (oracle, FP64).

* proj_l2ball : Eq. 10, projection onto B_i = {z : ||z - y_i||_2 <= eps_i}.
* soft        : Eq. 11, soft-thresholding S_alpha (complex-safe, 0 at z = 0).
* proj_pos    : Eq. 12, projection onto the positive orthant, keeping the real part.

Algorithm 1 uses them through the Moreau decomposition (Sec. III):
step 8 is z - P_B(z) and step 13 is z - S_alpha(z); ``data_dual_update`` and
``sparsity_dual_update`` write those forms literally.

Pins: variational characterisations (the projection inequality, brute-force
minimisation of the prox objectives), idempotence, nonexpansiveness, and the
closed forms z - P_B(z) = (z - y)(1 - eps/||z - y||)_+ and z - S_a(z) = clip(z, +-a).
"""
import numpy as np


def proj_l2ball(z, y, eps):
    r = z - y
    nr = np.linalg.norm(r)
    if nr > eps:
        return eps * r / nr + y
    return np.array(z, copy=True)


def soft(z, alpha):
    """S_alpha(z); alpha a scalar or one threshold per entry (the weighted l1 norm)."""
    z = np.asarray(z)
    mag = np.abs(z)
    out = np.zeros_like(z)
    nz = mag > 0
    a = np.broadcast_to(np.asarray(alpha, dtype=np.float64), z.shape)[nz]
    out[nz] = z[nz] * np.maximum(mag[nz] - a, 0.0) / mag[nz]
    return out


def proj_pos(z):
    return np.maximum(np.real(z), 0.0)


def data_dual_update(v, Gb, y, eps):
    """Algorithm 1 step 8: v + G b - P_B(v + G b)."""
    z = v + Gb
    return z - proj_l2ball(z, y, eps)


def sparsity_dual_update(s, w, alpha):
    """Algorithm 1 step 13: (s + w) - S_alpha(s + w), w = Psi^dagger x~.  With alpha an array
    of per-coefficient thresholds this is the step for the weighted l1 prior."""
    z = s + w
    return z - soft(z, alpha)
