"""Pins of the oracle's Eq. 13 and Eq. 14."""
import numpy as np
import pytest
from scipy.optimize import brentq

from oracle.probs import adaptive_probabilities, residual_energy


def test_residual_energy_closed_form():
    c = residual_energy([3.0, 1.0, 2.0], [2.0, 2.0, 2.0])
    assert c.tolist() == [0.25, 0.0, 0.0]


def _bisection_a(c, n, pmin, pmax):
    d = c.size
    w = (n - d * pmin) * c / c.sum()
    cap = pmax - pmin
    f = lambda a: np.minimum(w + a, cap).sum() - (n - d * pmin)
    if f(0.0) >= -1e-15:
        return 0.0
    return brentq(f, 0.0, cap, xtol=1e-15, rtol=1e-15)


@pytest.mark.parametrize("seed", range(6))
def test_eq14_constraints_and_independent_solve(seed):
    rng = np.random.default_rng(seed)
    d = 16
    c = rng.lognormal(0, 2, d) * (rng.uniform(size=d) < 0.8)
    n, pmin, pmax = 4.0, 0.05, 0.5
    p, a = adaptive_probabilities(c, n, pmin, pmax)
    assert p.sum() == pytest.approx(n, abs=1e-12)
    assert np.all(p >= pmin - 1e-15) and np.all(p <= pmax + 1e-15)
    assert a == pytest.approx(_bisection_a(c, n, pmin, pmax), abs=1e-12)
    order = np.argsort(c)
    assert np.all(np.diff(p[order]) >= -1e-15)                      # monotone in c


def test_eq14_special_cases():
    p, a = adaptive_probabilities(np.zeros(8), 2.0, 0.05, 0.9)
    assert np.allclose(p, 0.25) and a == 0.0
    # nothing saturates: a = 0 and p is affine in c
    c = np.array([1.0, 1.0, 2.0, 0.0])
    p, a = adaptive_probabilities(c, 2.0, 0.1, 1.0)
    assert a == 0.0
    assert np.allclose(p, 0.1 + 1.6 * c / 4.0)
    # p_max = n/d forces uniform probabilities
    p, _ = adaptive_probabilities(np.array([5.0, 0.1, 0.0, 1.0]), 2.0, 0.1, 0.5)
    assert np.allclose(p, 0.5)
    # one dominant block saturates, the rest share the remainder evenly
    p, a = adaptive_probabilities(np.array([100.0, 0.0, 0.0, 0.0, 0.0]), 2.0, 0.1, 0.6)
    assert p[0] == pytest.approx(0.6) and np.allclose(p[1:], 0.35)
    with pytest.raises(ValueError):
        adaptive_probabilities(np.ones(4), 3.0, 0.1, 0.5)       # n/d > p_max
