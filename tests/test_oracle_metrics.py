"""Pins of the oracle's Eq. 15, SNR = 20 log10(||x|| / ||x - x_hat||), against closed values.

Each case fixes the ratio of the two norms exactly, with ||x|| far from 1 and x spread over
many entries, so a wrong numerator (||x||^2, ||x||_1), a 10 log10 in place of 20 log10, or
a swapped ratio all fail."""
import math

import numpy as np
import pytest

from oracle.metrics import snr


@pytest.fixture
def x(rng):
    v = np.abs(rng.standard_normal((32, 32))) + 0.1
    return 7.3 * v / np.linalg.norm(v)  # ||x|| = 7.3, 1024 nonzero entries


@pytest.mark.parametrize("scale,db", [(0.9, 20.0), (0.99, 40.0), (1.1, 20.0), (0.999, 60.0), (0.0, 0.0), (2.0, 0.0)])
def test_snr_of_scaled_estimates(x, scale, db):
    """x_hat = s x: ||x - x_hat|| = |1 - s| ||x||, so SNR = -20 log10 |1 - s|."""
    assert snr(x, scale * x) == pytest.approx(db, abs=1e-9)


def test_snr_of_random_error(x, rng):
    """x_hat = x +- e with ||e|| = ||x|| / 100 gives 40 dB whatever the direction of e."""
    e = rng.standard_normal(x.shape)
    e *= (np.linalg.norm(x) / 100.0) / np.linalg.norm(e)
    assert snr(x, x + e) == pytest.approx(40.0, abs=1e-9)
    assert snr(x, x - e) == pytest.approx(40.0, abs=1e-9)


def test_snr_is_scale_invariant_and_exact_fit_is_infinite(x):
    assert snr(3.0 * x, 3.0 * 0.9 * x) == pytest.approx(snr(x, 0.9 * x), abs=1e-12)
    assert math.isinf(snr(x, x))
    # 20 log10(||x|| / ||x - x_hat||) with the two norms given directly
    xh = x.copy()
    xh[0, 0] += 0.73  # ||x - x_hat|| = 0.73 = ||x|| / 10
    assert snr(x, xh) == pytest.approx(20.0, abs=1e-9)
