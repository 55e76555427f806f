"""Pins of the oracle's measurement operator (Eqs. 1-3, 8) against independent references."""
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import i0

from oracle.kaiser_bessel import kb, kb_ft
from oracle.measurement import Measurement, nudft


def test_kb_shape():
    J, beta = 8, 18.72
    t = np.linspace(-4, 4, 101)
    v = kb(t, J, beta)
    assert np.allclose(v, v[::-1], rtol=1e-13, atol=0)
    assert kb(np.array([0.0]), J, beta)[0] == pytest.approx(1.0, abs=1e-15)
    # edge of the support: I0(0) / I0(beta)
    assert kb(np.array([4.0]), J, beta)[0] == pytest.approx(1.0 / i0(beta), rel=1e-14)
    assert kb(np.array([4.0001, -5.0]), J, beta).tolist() == [0.0, 0.0]


@pytest.mark.parametrize("f", [0.0, 0.05, 0.125, 0.2, 0.25])
def test_kb_fourier_transform_closed_form_vs_quadrature(f):
    J, beta = 8, 18.72
    q, _ = quad(lambda t: kb(np.array([t]), J, beta)[0] * np.cos(2 * np.pi * f * t), -J / 2, J / 2,
                epsabs=1e-15, epsrel=1e-13, limit=400)
    assert kb_ft(f, J, beta) == pytest.approx(q, rel=1e-10)


def test_F_is_the_textbook_dft():
    rng = np.random.default_rng(1)
    K = 12
    z = rng.standard_normal((K, K)) + 1j * rng.standard_normal((K, K))
    k = np.arange(K)
    W = np.exp(-2j * np.pi * np.outer(k, k) / K)
    ref = W @ z @ W.T
    m = Measurement(np.zeros((1, 2), np.float32), [0, 1], (K // 2, K // 2))
    assert np.abs(m.F(z) - ref).max() <= 1e-12 * np.abs(ref).max()
    # F^dagger F = K^2 I
    assert np.abs(m.FH(m.F(z)) - K * K * z).max() <= 1e-11 * K * K * np.abs(z).max()


@pytest.mark.parametrize("n", [16, 32])
def test_phi_matches_direct_nudft_and_improves_with_J(n):
    rng = np.random.default_rng(n)
    M = 400
    uv = rng.uniform(-np.pi, np.pi, (M, 2)).astype(np.float32)
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    ref = nudft(x, uv)
    errs = []
    for J in (4, 6, 8):
        y = Measurement(uv, [0, 150, M], (n, n), J=J).phi(x)
        errs.append(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    assert errs[2] < 1e-6
    assert errs[0] > errs[1] > errs[2]


def test_nudft_brute_force_single_pixel():
    # one pixel at centred coordinate (l_x, l_y) = (3, -2): y = exp(-i (3u - 2v))
    n = 8
    x = np.zeros((n, n))
    x[n // 2 - 2, n // 2 + 3] = 1.0
    uv = np.array([[0.3, -1.1], [2.0, 0.5]])
    ref = np.exp(-1j * (3 * uv[:, 0] - 2 * uv[:, 1]))
    assert np.allclose(nudft(x, uv), ref, atol=1e-14)


def test_integer_grid_coordinates_and_band_edges():
    # u-v exactly on grid points and at the band edge still interpolate accurately
    n = 16
    K = 2 * n
    uv = np.array([[0.0, 0.0], [2 * np.pi * 3 / K, -2 * np.pi * 5 / K],
                   [np.nextafter(np.float32(np.pi), 0), -np.pi]], dtype=np.float32)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((n, n))
    y = Measurement(uv, [0, 3], (n, n)).phi(x)
    ref = nudft(x, uv)
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 1e-6


def test_adjoint_dot_products():
    rng = np.random.default_rng(3)
    n, M = 16, 300
    uv = rng.uniform(-np.pi, np.pi, (M, 2)).astype(np.float32)
    m = Measurement(uv, [0, 100, 220, M], (n, n))
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    y = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    lhs = np.vdot(y, m.phi(x))
    rhs = np.vdot(m.phi_adj(y), x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    xr = x.real
    assert np.vdot(y, m.phi(xr)).real == pytest.approx(np.vdot(m.phi_adj_real(y), xr).real, rel=1e-12)


def test_adjoint_as_explicit_matrix():
    # assemble Phi column by column and compare Phi^dagger with the conjugate transpose
    rng = np.random.default_rng(4)
    n, M = 8, 40
    uv = rng.uniform(-np.pi, np.pi, (M, 2)).astype(np.float32)
    m = Measurement(uv, [0, 13, M], (n, n))
    E = np.eye(n * n)
    P = np.stack([m.phi(e.reshape(n, n)) for e in E], axis=1)
    y = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    assert np.abs(m.phi_adj(y).ravel() - P.conj().T @ y).max() < 1e-12 * np.abs(P).max() * M


def test_block_stacking_and_cell_sets():
    rng = np.random.default_rng(5)
    n, M = 16, 256
    uv = rng.uniform(-np.pi, np.pi, (M, 2)).astype(np.float32)
    off = [0, 60, 61, 200, M]
    m = Measurement(uv, off, (n, n))
    x = rng.standard_normal((n, n))
    y = m.phi(x)
    grid = m.F(m.Z(x))
    for i in range(m.d):
        lo, hi = m.block_range(i)
        assert np.allclose(m.phi_block(i, x), y[lo:hi], rtol=0, atol=1e-12)
        # G_i acting on M_i b~ equals the direct gather from the full grid
        assert np.allclose(m.Gi(i, m.Mi(i, grid)), y[lo:hi], atol=1e-12)
        # every tap of the block lies in its cell set, and nothing else does
        flat, _ = m.footprint(lo, hi)
        assert np.array_equal(np.unique(flat), m.cells(i))
    v = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    acc = sum(m.MiH(i, m.GiH(i, v[off[i]:off[i + 1]])) for i in range(m.d))
    assert np.allclose(m.ZH(m.FH(acc)), m.phi_adj(v), atol=1e-10)
