"""Pins of the oracle's Daubechies filters and SARA dictionary (Sec. III)."""
import math
import os

import numpy as np
import pytest

from oracle.power import psi_norm
from oracle.wavelets import Sara, daubechies, dwt2, highpass, idwt2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "daubechies_closed_forms.txt")


def _closed_forms():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, taps = line.split(":", 1)
        out[name.strip()] = np.array([eval(t, {"sqrt": math.sqrt}) for t in taps.split(",")])
    return out


@pytest.mark.parametrize("name", ["db1", "db2", "db3"])
def test_filters_match_published_closed_forms(name):
    ref = _closed_forms()[name]
    h = daubechies(int(name[2:]))
    assert h.shape == ref.shape
    assert np.abs(h - ref).max() < 1e-14


@pytest.mark.parametrize("N", range(1, 9))
def test_filter_conditions(N):
    h = daubechies(N)
    assert h.size == 2 * N
    assert h.sum() == pytest.approx(math.sqrt(2), abs=1e-14)
    # double-shift orthonormality: sum_k h_k h_{k+2l} = delta_l
    for l in range(N):
        assert np.dot(h[: h.size - 2 * l], h[2 * l:]) == pytest.approx(1.0 if l == 0 else 0.0, abs=1e-12)
    # N vanishing moments of the highpass
    g = highpass(h)
    k = np.arange(h.size, dtype=np.float64)
    for p in range(N):
        assert abs(np.dot(g, k ** p)) < 1e-9 * max(1.0, (2 * N) ** p)
    # minimum phase: the zeros left after removing (1 + z^-1)^N lie inside the unit circle
    q, rem = np.polydiv(h, np.poly([-1.0] * N))
    assert np.abs(rem).max() < 1e-10
    assert np.all(np.abs(np.roots(q)) < 1.0)


def _matrix(fn, n):
    return np.stack([fn(e.reshape(n, n)).ravel() for e in np.eye(n * n)], axis=1)


@pytest.mark.parametrize("N", [1, 2, 5, 8])
def test_2d_transform_is_orthogonal_brute_force(N):
    # 16 x 16 with 4 levels: the coarsest level is 2 x 2, far shorter than db8's 16 taps
    n, L = 16, 4
    h = daubechies(N)
    Q = _matrix(lambda x: dwt2(x, h, L), n)
    assert np.abs(Q.T @ Q - np.eye(n * n)).max() < 1e-12
    R = _matrix(lambda c: idwt2(c, h, L), n)
    assert np.abs(R - Q.T).max() < 1e-12


def test_haar_coefficients_are_block_sums():
    rng = np.random.default_rng(7)
    n, L = 16, 4
    x = rng.standard_normal((n, n))
    c = dwt2(x, daubechies(1), L)
    # coarsest approximation: sum over 16x16 blocks / 2^L
    assert c[0, 0] == pytest.approx(x.sum() / 16.0, abs=1e-12)
    # level-1 diagonal detail at (i, j): (a - b - c + d)/2 on the 2x2 block
    i, j = 3, 5
    blk = x[2 * i:2 * i + 2, 2 * j:2 * j + 2]
    assert c[n // 2 + i, n // 2 + j] == pytest.approx((blk[0, 0] - blk[0, 1] - blk[1, 0] + blk[1, 1]) / 2, abs=1e-12)
    # level-1 low-y / high-x detail: rows summed, columns differenced
    assert c[i, n // 2 + j] == pytest.approx((blk[0, 0] - blk[0, 1] + blk[1, 0] - blk[1, 1]) / 2, abs=1e-12)
    # level-1 high-y / low-x detail
    assert c[n // 2 + i, j] == pytest.approx((blk[0, 0] + blk[0, 1] - blk[1, 0] - blk[1, 1]) / 2, abs=1e-12)
    # level-2 approximation lives at [0:n/4, 0:n/4] only transiently; level-2 LL of block (1,2)
    c2 = dwt2(x, daubechies(1), 2)
    assert c2[1, 2] == pytest.approx(x[4:8, 8:12].sum() / 4, abs=1e-12)


@pytest.mark.parametrize("N", range(1, 9))
def test_constant_image_has_no_details(N):
    n, L = 32, 4
    c = dwt2(np.full((n, n), 2.5), daubechies(N), L)
    m = n >> L
    # each level multiplies a constant by sqrt(2)^2 = 2
    assert np.allclose(c[:m, :m], 2.5 * 2 ** L, atol=1e-12)
    d = c.copy()
    d[:m, :m] = 0
    assert np.abs(d).max() < 1e-12


def test_sara_frame_identity_and_norm():
    rng = np.random.default_rng(8)
    n = 32
    s = Sara(n)
    assert s.b == 9
    x = rng.standard_normal((n, n))
    assert np.abs(s.fwd(s.adj(x)) - 9 * x).max() < 1e-12
    # adjoint pair: <Psi^dagger x, c> = <x, Psi c>
    c = rng.standard_normal((9, n, n))
    assert np.vdot(s.adj(x), c) == pytest.approx(np.vdot(x, s.fwd(c)), rel=1e-12)
    # Dirac basis is the identity
    assert np.array_equal(s.adj(x)[0], x)
    nrm, _ = psi_norm(s, rng.standard_normal((n, n)))
    assert nrm == pytest.approx(3.0, rel=1e-9)


def test_sara_rejects_bad_size():
    with pytest.raises(ValueError):
        Sara(24, levels=4)
