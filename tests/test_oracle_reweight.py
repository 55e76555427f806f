"""Pins of the oracle's reweighted SARA (weighted l1 prior, oracle/reweight.py)."""
import numpy as np
import pytest

import synth
from oracle import pd as opd
from oracle.measurement import Measurement
from oracle.metrics import snr
from oracle.prox import soft, sparsity_dual_update
from oracle.reweight import run_reweighted, weights
from oracle.wavelets import Sara


def test_weighted_soft_threshold_is_the_prox(rng):
    """S_{alpha w}(u)_k minimises 1/2 (z - u_k)^2 + alpha w_k |z| (brute force over a fine grid)."""
    u = rng.standard_normal(40) * 2.0
    thr = rng.uniform(0.0, 1.5, 40)
    got = soft(u, thr)
    grid = np.linspace(-6, 6, 240001)
    for k in range(40):
        f = 0.5 * (grid - u[k]) ** 2 + thr[k] * np.abs(grid)
        assert got[k] == pytest.approx(grid[np.argmin(f)], abs=1e-4)


def test_unit_weights_give_the_plain_step(rng):
    s = rng.uniform(-1e-3, 1e-3, (3, 8, 8))
    a = rng.standard_normal((3, 8, 8)) * 1e-3
    alpha = 3e-3
    assert np.array_equal(sparsity_dual_update(s, a, alpha), sparsity_dual_update(s, a, alpha * np.ones_like(s)))
    # the Moreau form with per-coefficient thresholds is the clip to +- alpha w
    w = rng.uniform(0.1, 1.0, s.shape)
    assert np.allclose(sparsity_dual_update(s, a, alpha * w), np.clip(s + a, -alpha * w, alpha * w), atol=1e-18)


def test_weights_are_the_log_penalty_derivative(rng):
    """w = d/d|c| [delta log(delta + |c|)], checked by central differences; w(0) = 1 and
    w = 1/2 where |c| = delta."""
    n = 16
    sara = Sara(n, 2)
    x = rng.standard_normal((n, n))
    delta = 0.3
    w = weights(sara, x, delta)
    c = np.abs(sara.adj(x))
    h = 1e-6
    fd = delta * (np.log(delta + c + h) - np.log(delta + c - h)) / (2 * h)
    assert np.allclose(w, fd, rtol=1e-7, atol=0)
    assert np.all((w > 0) & (w <= 1))
    z = np.zeros((n, n))
    assert np.array_equal(weights(sara, z, delta), np.ones((sara.b, n, n)))
    # a Dirac coefficient of exactly delta gets weight 1/2
    z[3, 5] = delta
    assert weights(sara, z, delta)[0, 3, 5] == pytest.approx(0.5, abs=1e-15)
    with pytest.raises(ValueError):
        weights(sara, x, 0.0)


def test_reweighted_run_without_reweighting_is_the_plain_run(rng):
    """`every` beyond the run length keeps w = 1: the plain Algorithm 1 bitwise; with
    reweighting the invariants still hold (|s| <= alpha w, x >= 0)."""
    n, M, d = 32, 3000, 3
    x = synth.sky(n, 3, 5, rng)
    uv, off, _ = synth.partition(synth.uv_coverage(M, rng), d, "equal")
    meas = Measurement(uv, off, (n, n))
    sara = Sara(n, 3)
    y = meas.phi(x) + 0.02 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    eps = synth.l2_ball_radii(off, 0.02 * np.sqrt(2))
    prm = opd.default_params(3.0, 60.0)
    masks = np.ones((12, d), bool)
    a, _ = opd.run(meas, sara, y, eps, prm, masks)
    b, _, deltas = run_reweighted(meas, sara, y, eps, prm, masks, every=100, delta0=0.1, beta=0.5)
    assert deltas == [] and np.array_equal(a.x, b.x) and np.array_equal(a.s, b.s)
    c, hist, deltas = run_reweighted(meas, sara, y, eps, prm, masks, every=4, delta0=0.1, beta=0.5, x_true=x)
    assert deltas == [0.1, 0.05]
    assert np.all(np.abs(c.s) <= prm.alpha * c.w * (1 + 1e-9))
    assert np.all(c.x >= 0)
    assert np.isfinite(hist[-1]["snr"])
