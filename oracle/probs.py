"""Adaptive block-selection probabilities, Sec. IV (oracle, FP64).

Eq. 13: c_i = max(||Phi_i x - y_i||_2 - eps_i, 0)^2 / eps_i^2.

Eq. 14: p_i = p_min + min((n - d p_min) c_i / sum_j c_j + a, p_max - p_min), with
a >= 0 raised until sum_i p_i = n (a = 0 when nothing saturates), and p_i = n / d for
all i when sum c = 0.  Requires p_min <= n/d <= p_max.

``adaptive_probabilities`` solves for a exactly: with w_i = (n - d p_min) c_i / sum c
sorted in decreasing order, if the k largest saturate then
a = (R - k cap - sum_{i>=k} w_i) / (d - k), R = n - d p_min, cap = p_max - p_min; the
right k is the smallest one for which the next entry does not saturate.

Pins: sum p = n, p_min <= p <= p_max, monotone in c, uniform for c = 0, and a equal to
an independent bisection on sum_i min(w_i + a, cap) = R.
"""
import numpy as np


def residual_energy(resid_norm, eps):
    """Eq. 13 from ||Phi_i x - y_i||_2 and eps_i."""
    resid_norm = np.asarray(resid_norm, dtype=np.float64)
    eps = np.asarray(eps, dtype=np.float64)
    return np.maximum(resid_norm - eps, 0.0) ** 2 / eps ** 2


def adaptive_probabilities(c, n_nodes, p_min, p_max):
    """Eq. 14.  Returns (p, a)."""
    c = np.asarray(c, dtype=np.float64)
    d = c.size
    if not (0.0 < p_min <= n_nodes / d <= p_max):
        raise ValueError("need 0 < p_min <= n/d <= p_max")
    total = c.sum()
    if total == 0.0:
        return np.full(d, n_nodes / d), 0.0
    R = n_nodes - d * p_min
    cap = p_max - p_min
    w = R * c / total
    ws = np.sort(w)[::-1]
    a = 0.0
    if ws[0] > cap:  # something saturates at a = 0, so a > 0 is needed
        suffix = np.concatenate([np.cumsum(ws[::-1])[::-1], [0.0]])
        for k in range(1, d + 1):
            if k == d:
                a = cap  # everything saturates: then d * cap == R
                break
            a_k = (R - k * cap - suffix[k]) / (d - k)
            if ws[k] + a_k <= cap:
                a = a_k
                break
    return p_min + np.minimum(w + a, cap), a
