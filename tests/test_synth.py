"""Checks of the seeded workload generator (inputs only)."""
import numpy as np
import pytest
from scipy.stats import chi2

import synth


def test_sky_is_nonnegative_with_unit_peak_and_seeded():
    a = synth.sky(64, 5, 10, np.random.default_rng(1))
    b = synth.sky(64, 5, 10, np.random.default_rng(1))
    assert np.array_equal(a, b)
    assert a.min() >= 0.0 and a.max() == pytest.approx(1.0)


def test_uv_band_and_spread():
    uv = synth.uv_coverage(200000, np.random.default_rng(2))
    assert uv.dtype == np.float32
    assert np.all(np.abs(uv) < np.float32(np.pi))
    assert np.std(uv.astype(np.float64)) == pytest.approx(np.pi / 4, rel=0.02)
    uo = synth.uv_coverage(100000, np.random.default_rng(3), outlier_frac=0.1)
    # uniform outliers push a visible tail beyond 3 sigma: 0.1 * (1 - 3/4) + 0.9 * 0.0027
    frac = np.mean(np.abs(uo[:, 0]) > 3 * np.pi / 4)
    assert 0.022 < frac < 0.034


@pytest.mark.parametrize("scheme,d", [("equal", 4), ("annuli", 16), ("lognormal", 64)])
def test_partitions_are_radial_and_complete(scheme, d):
    M = 1 << 16
    uv = synth.uv_coverage(M, np.random.default_rng(4))
    uvs, off, order = synth.partition(uv, d, scheme, np.random.default_rng(5))
    assert off[0] == 0 and off[-1] == M and np.all(np.diff(off) > 0)
    assert np.array_equal(uvs, uv[order])
    r = np.hypot(uvs[:, 0].astype(np.float64), uvs[:, 1].astype(np.float64))
    assert np.all(np.diff(r) >= 0)
    if scheme == "lognormal":
        assert np.diff(off).min() >= 256 and len(off) == d + 1


def test_noise_level_and_radii_coverage():
    rng = np.random.default_rng(6)
    y0 = rng.standard_normal(4096) + 1j * rng.standard_normal(4096)
    s = synth.noise_sigma(y0, 20.0)
    assert s ** 2 == pytest.approx(np.mean(np.abs(y0) ** 2) / 100.0)
    off = np.array([0, 100, 1100, 4096])
    eps = synth.l2_ball_radii(off, s)
    assert eps[1] == pytest.approx(s / np.sqrt(2) * np.sqrt(chi2.ppf(0.99, 2000)))
    # Monte-Carlo: the noise falls inside the ball 99% of the time
    inside, trials = 0, 2000
    for _ in range(trials):
        nz = synth.complex_noise(4096, s, rng)
        inside += np.linalg.norm(nz[100:1100]) <= eps[1]
    sd = np.sqrt(0.99 * 0.01 / trials)
    assert abs(inside / trials - 0.99) < 4 * sd


def test_workload_table_matches_sizes():
    w = synth.WORKLOADS["n1024_m4m_d64"]
    assert (w.n, w.M, w.d) == (1024, 1 << 22, 64)
    inp = synth.make_inputs(synth.WORKLOADS["n64_m8k_d4"])
    assert inp.uv.shape == (8192, 2) and inp.block_off.tolist() == [0, 2048, 4096, 6144, 8192]
