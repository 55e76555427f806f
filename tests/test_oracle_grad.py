"""Pins of the oracle's derivatives (oracle/grad.py) against central differences.

Each VJP is checked against finite differences of its own forward map with complex
values taken as pairs of reals; the data-fit gradient against finite differences of
1/2 ||Phi x - y||^2; the unrolled d SNR / d(tau, sigma) against finite differences of the
unrolled SNR (FP64, h = 1e-6), away from the kinks of the proximity operators.
"""
import numpy as np
import pytest

import synth
from helpers import problem
from oracle import grad as og
from oracle import pd as opd
from oracle.measurement import Measurement
from oracle.power import phi_norm
from oracle.prox import data_dual_update, sparsity_dual_update
from oracle.wavelets import Sara


def _fd_jacobian_c(f, z, h=1e-7):
    """Real Jacobian of f: C^n -> C^m, columns over (Re z_k, Im z_k)."""
    cols = []
    for k in range(z.size):
        for unit in (1.0, 1j):
            dz = np.zeros_like(z)
            dz[k] = unit * h
            cols.append((f(z + dz) - f(z - dz)) / (2 * h))
    return cols  # list of complex vectors, one per real input coordinate


@pytest.mark.parametrize("outside", [True, False])
def test_ball_shrink_vjp_matches_finite_differences(outside):
    rng = np.random.default_rng(1 if outside else 2)
    r = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    eps = 0.5 * np.linalg.norm(r) if outside else 2.0 * np.linalg.norm(r)
    g = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    # the step-8 map through its Moreau form, as the oracle's iteration uses it
    f = lambda z: data_dual_update(np.zeros_like(z), z, np.zeros_like(z), eps)  # noqa: E731
    cols = _fd_jacobian_c(f, r)
    want = np.array([np.real(np.vdot(c, g)) for c in cols])  # g^T J, per real coordinate
    got_c = og.vjp_ball_shrink(r, eps, g)
    got = np.ravel(np.column_stack([got_c.real, got_c.imag]))
    assert np.allclose(got, want, rtol=1e-7, atol=1e-9)


def test_clip_and_positivity_vjps_match_finite_differences():
    rng = np.random.default_rng(3)
    alpha = 0.3
    a = rng.uniform(-1, 1, 50)
    a = a[np.abs(np.abs(a) - alpha) > 1e-3]          # away from the kinks
    g = rng.standard_normal(a.size)
    f = lambda z: sparsity_dual_update(np.zeros_like(z), z, alpha)  # noqa: E731
    h = 1e-7
    fd = np.array([(f(a + h * e)[k] - f(a - h * e)[k]) / (2 * h) for k, e in enumerate(np.eye(a.size))])
    assert np.allclose(og.vjp_clip(a, alpha, g), fd * g, atol=1e-8)
    z = rng.standard_normal(40)
    z = z[np.abs(z) > 1e-3]
    gz = rng.standard_normal(z.size)
    fdz = np.array([(opd.proj_pos(z + h * e)[k] - opd.proj_pos(z - h * e)[k]) / (2 * h)
                    for k, e in enumerate(np.eye(z.size))])
    assert np.allclose(og.vjp_pos(z, gz), fdz * gz, atol=1e-8)


def test_data_fit_gradient_matches_finite_differences():
    n, M = 16, 300
    x, uv, off = problem(n, M, 2, "equal", 4)
    meas = Measurement(uv, off, (n, n))
    rng = np.random.default_rng(5)
    y = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    f = lambda xx: 0.5 * np.linalg.norm(meas.phi(xx) - y) ** 2  # noqa: E731
    gr = og.data_fit_grad(meas, x, y)
    for k in range(4):
        d = rng.standard_normal((n, n))
        fd = (f(x + 1e-6 * d) - f(x - 1e-6 * d)) / 2e-6
        assert np.sum(gr * d) == pytest.approx(fd, rel=1e-6)


def test_snr_gradient_matches_finite_differences():
    rng = np.random.default_rng(6)
    xt, x = rng.standard_normal(30), rng.standard_normal(30)
    from oracle.metrics import snr

    gr = og.snr_grad(xt, x)
    for k in range(3):
        d = rng.standard_normal(30)
        fd = (snr(xt, x + 1e-6 * d) - snr(xt, x - 1e-6 * d)) / 2e-6
        assert np.dot(gr, d) == pytest.approx(fd, rel=1e-6)


def _unrolled_case(seed=7, T=10):
    n, M, d = 16, 500, 3
    x, uv, off = problem(n, M, d, "equal", seed)
    meas = Measurement(uv, off, (n, n))
    sara = Sara(n)
    y0 = meas.phi(x)
    sig = synth.noise_sigma(y0, 25.0)
    y = y0 + synth.complex_noise(M, sig, np.random.default_rng(seed + 1))
    eps = synth.l2_ball_radii(off, sig)
    phin, _ = phi_norm(meas, synth.power_start(n, seed), tol=0.0, max_it=60)
    prm = opd.default_params(3.0, phin)
    masks = np.random.default_rng(seed + 2).uniform(size=(T, d)) < 0.7
    masks[0] = True
    return meas, sara, x, y, eps, prm, masks


def test_unrolled_gradient_matches_finite_differences():
    """Algorithm 1 unrolled for 10 iterations with fixed random masks (p = 0.7)."""
    meas, sara, x, y, eps, prm, masks = _unrolled_case()
    s, dtau, dsig = og.unrolled_gradient(meas, sara, y, eps, prm, masks, x)
    assert s == pytest.approx(og.unrolled_snr(meas, sara, y, eps, prm, masks, x), abs=1e-12)
    import dataclasses

    f_tau = lambda t: og.unrolled_snr(meas, sara, y, eps, dataclasses.replace(prm, tau=t), masks, x)  # noqa: E731
    f_sig = lambda q: og.unrolled_snr(meas, sara, y, eps, dataclasses.replace(prm, sigma=q), masks, x)  # noqa: E731
    fd_tau = og.central_difference(f_tau, prm.tau)
    fd_sig = og.central_difference(f_sig, prm.sigma)
    print(f"dSNR/dtau {dtau:.8g} (FD {fd_tau:.8g}), dSNR/dsigma {dsig:.8g} (FD {fd_sig:.8g})")
    assert abs(dtau) > 1e-3 and abs(dsig) > 1e-6
    assert dtau == pytest.approx(fd_tau, rel=1e-4)
    assert dsig == pytest.approx(fd_sig, rel=1e-4)


def test_stored_512_gradient_agrees_with_its_central_differences():
    """The stored oracle gradient at 512^2 (M = 2^20, 20 iterations) against the central
    differences the same script computed (h = 1e-6)."""
    import json
    import os

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "grad_reference_n512_m1m_d32.json")
    if not os.path.exists(path):
        pytest.skip("no stored reference gradient")
    ref = json.load(open(path))
    assert ref["dsnr_dtau"] == pytest.approx(ref["fd_dsnr_dtau"], rel=1e-5)
    assert ref["dsnr_dsigma"] == pytest.approx(ref["fd_dsnr_dsigma"], rel=1e-5)
