"""Pins of the oracle's proximity operators (Eqs. 10-12) and the Moreau forms of steps 8, 13."""
import numpy as np
import pytest

from oracle.prox import data_dual_update, proj_l2ball, proj_pos, soft, sparsity_dual_update


def _cplx(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def test_ball_projection_properties():
    rng = np.random.default_rng(1)
    y = _cplx(rng, 50)
    eps = 2.0
    for scale in (0.1, 0.5, 3.0, 10.0):
        z = y + scale * _cplx(rng, 50) / np.sqrt(50)
        p = proj_l2ball(z, y, eps)
        assert np.linalg.norm(p - y) <= eps * (1 + 1e-14)
        assert np.allclose(proj_l2ball(p, y, eps), p, atol=1e-14)            # idempotent
        if np.linalg.norm(z - y) <= eps:
            assert np.array_equal(p, z)
        # projection inequality: Re <z - P(z), w - P(z)> <= 0 for every w in the ball
        for _ in range(20):
            w = y + eps * rng.uniform() * (lambda u: u / np.linalg.norm(u))(_cplx(rng, 50))
            assert np.vdot(z - p, w - p).real <= 1e-12
    # nonexpansive
    z1, z2 = y + 5 * _cplx(rng, 50), y + 5 * _cplx(rng, 50)
    assert np.linalg.norm(proj_l2ball(z1, y, eps) - proj_l2ball(z2, y, eps)) <= np.linalg.norm(z1 - z2)


def test_step8_moreau_form():
    rng = np.random.default_rng(2)
    y = _cplx(rng, 40)
    for eps in (0.5, 5.0, 50.0):
        v, Gb = _cplx(rng, 40), y + _cplx(rng, 40)
        r = v + Gb - y
        ref = r * max(0.0, 1.0 - eps / np.linalg.norm(r))
        assert np.allclose(data_dual_update(v, Gb, y, eps), ref, atol=1e-13)


def test_soft_threshold_is_the_prox_of_l1_by_brute_force():
    rng = np.random.default_rng(3)
    alpha = 0.7
    grid = np.linspace(-4, 4, 80001)
    for z in rng.uniform(-3, 3, 25):
        obj = 0.5 * (grid - z) ** 2 + alpha * np.abs(grid)
        assert soft(np.array([z]), alpha)[0] == pytest.approx(grid[np.argmin(obj)], abs=2e-4)
    # complex: shrink the modulus, keep the phase; exactly 0 at 0
    z = np.array([3 + 4j, 0.1 + 0.1j, 0j])
    assert np.allclose(soft(z, 1.0), [2.4 + 3.2j, 0, 0], atol=1e-15)


def test_step13_moreau_form_is_a_clip():
    rng = np.random.default_rng(4)
    s, w = rng.standard_normal(1000), rng.standard_normal(1000)
    a = 0.3
    assert np.allclose(sparsity_dual_update(s, w, a), np.clip(s + w, -a, a), atol=1e-15)


def test_positive_projection_by_brute_force():
    rng = np.random.default_rng(5)
    grid = np.linspace(0, 4, 40001)
    for z in rng.uniform(-2, 2, 10) + 1j * rng.uniform(-2, 2, 10):
        best = grid[np.argmin(np.abs(grid - z) ** 2)]
        assert proj_pos(np.array([z]))[0] == pytest.approx(best, abs=1e-4)
