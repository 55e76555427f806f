"""Pins of the oracle's DDE-aware measurement operator (oracle/dde.py)."""
import numpy as np
import pytest

import synth
from oracle.dde import DDEMeasurement, nudft_dde
from oracle.measurement import Measurement, nudft


def _uv(rng, M):
    return rng.uniform(-np.pi, np.pi, (M, 2)).astype(np.float32)


def test_delta_dde_is_the_plain_operator(rng):
    n, M = 16, 300
    uv = _uv(rng, M)
    meas = Measurement(uv, [0, M], (n, n))
    d = np.zeros((M, 5, 5), complex)
    d[:, 2, 2] = 1.0
    dm = DDEMeasurement(meas, d)
    x = rng.standard_normal((n, n))
    assert np.allclose(dm.phi(x), meas.phi(x), rtol=0, atol=1e-13 * np.abs(meas.phi(x)).max())
    y = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    assert np.allclose(dm.phi_adj(y), meas.phi_adj(y), atol=1e-12 * np.abs(meas.phi_adj(y)).max())


def test_unit_shift_dde_is_a_shifted_frequency(rng):
    """d = 1 at (p, q) = (1, 0) measures the plain visibility at u + 2 pi / K (the x axis),
    and at (p, q) = (0, -2) the one at v - 4 pi / K."""
    n, M = 16, 200
    K = 2 * n
    uv = rng.uniform(-2.5, 2.5, (M, 2))
    meas = Measurement(uv, [0, M], (n, n))
    x = rng.standard_normal((n, n))
    for (p, q) in [(1, 0), (0, -2)]:
        d = np.zeros((M, 5, 5), complex)
        d[:, 2 + q, 2 + p] = 1.0
        shifted = uv + np.array([2 * np.pi * p / K, 2 * np.pi * q / K])
        ref = Measurement(shifted, [0, M], (n, n)).phi(x)
        got = DDEMeasurement(meas, d).phi(x)
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-9


@pytest.mark.parametrize("jd", [1, 3, 5])
def test_dde_operator_against_direct_nudft(rng, jd):
    """The DDE-aware Phi against the discretised Eq. 1 with the DDE, summed directly: the
    error is the interpolation's (J = 8), far below the DDE's own effect."""
    n, M = 16, 150
    K = 2 * n
    uv = synth.uv_coverage(M, rng)
    x = rng.standard_normal((n, n))
    d = synth.dde_taps(M, jd, rng, strength=0.3)
    meas = Measurement(uv, [0, M], (n, n))
    got = DDEMeasurement(meas, d).phi(x)
    ref = nudft_dde(x, uv, d, K)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < 2e-6, err
    if jd > 1:  # the DDE changes the data by far more than that
        assert np.linalg.norm(ref - nudft(x, uv)) / np.linalg.norm(ref) > 1e-2


def test_dde_adjoint_identity(rng):
    n, M, d_blocks = 32, 2000, 3
    uv, off, _ = synth.partition(synth.uv_coverage(M, rng), d_blocks, "equal")
    meas = Measurement(uv, off, (n, n))
    dm = DDEMeasurement(meas, synth.dde_taps(M, 5, rng))
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    y = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    g = meas.F(meas.Z(x))
    lhs = np.vdot(dm.degrid(g), y)
    rhs = np.vdot(x, dm.phi_adj(y))
    assert abs(lhs - rhs) / abs(lhs) < 1e-12
    # the real restriction used by Algorithm 1
    xr = x.real
    assert abs(np.vdot(dm.phi(xr), y).real - np.sum(xr * dm.phi_adj_real(y))) < 1e-10 * abs(lhs)
    # per-block adjoints sum to the whole one
    parts = sum(dm.phi_adj(y, blocks=[i]) for i in range(d_blocks))
    assert np.allclose(parts, dm.phi_adj(y), atol=1e-12 * np.abs(parts).max())


def test_dde_taps_generator(rng):
    d = synth.dde_taps(1000, 5, rng, strength=0.2)
    assert d.shape == (1000, 5, 5)
    assert abs(np.mean(d[:, 2, 2]) - 1.0) < 0.03
    assert np.std(d[:, 0, 0]) < np.std(d[:, 2, 1])  # decays away from the centre
    with pytest.raises(ValueError):
        synth.dde_taps(3, 4, rng)


def test_dde_block_interface_and_pd_iteration(rng):
    """The block form (M_i, G_i, G_i^H) agrees with the whole operator, and Algorithm 1 runs on
    the DDE operator with a delta DDE exactly as on the plain one."""
    from oracle import pd as opd
    from oracle.wavelets import Sara

    n, M, d = 32, 2500, 3
    uv, off, _ = synth.partition(synth.uv_coverage(M, rng), d, "equal")
    meas = Measurement(uv, off, (n, n))
    dm = DDEMeasurement(meas, synth.dde_taps(M, 3, rng))
    x = rng.standard_normal((n, n))
    g = meas.F(meas.Z(x))
    whole = dm.degrid(g)
    for i in range(d):
        lo, hi = meas.block_range(i)
        assert np.allclose(dm.Gi(i, dm.Mi(i, g)), whole[lo:hi], rtol=0, atol=1e-12 * np.abs(whole).max())
    y = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    acc = np.zeros(meas.Ky * meas.Kx, complex)
    for i in range(d):
        lo, hi = meas.block_range(i)
        acc[dm.cells(i)] += dm.GiH(i, y[lo:hi])
    assert np.allclose(acc.reshape(meas.Ky, meas.Kx), dm.grid_adj(y), atol=1e-12 * np.abs(acc).max())
    delta = np.zeros((M, 3, 3), complex)
    delta[:, 1, 1] = 1.0
    sara = Sara(n, 3)
    yb = meas.phi(x) + 0.01 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    prm = opd.default_params(3.0, 60.0)
    masks = rng.uniform(size=(4, d)) < 0.7
    a, _ = opd.run(meas, sara, yb, np.full(d, 0.3), prm, masks)
    b, _ = opd.run(DDEMeasurement(meas, delta), sara, yb, np.full(d, 0.3), prm, masks)
    assert np.allclose(a.x, b.x, rtol=0, atol=1e-12)
