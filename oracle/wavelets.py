"""Daubechies filters and the SARA sparsity dictionary (oracle, FP64).

Sec. III takes Psi in C^{N x bN} as a collection of b bases (the SARA bases of
Carrillo et al. 2012).  The reading used here: b = 9, the Dirac basis plus the
Daubechies wavelets db1..db8, each a 4-level periodic separable 2D discrete wavelet
transform, concatenated without normalisation, so Psi Psi^dagger = 9 I and
||Psi||_S = 3.

Filters (textbook construction, Daubechies 1988): the squared response of the
length-2N lowpass is |H(w)|^2 = 2 cos^{2N}(w/2) P(sin^2(w/2)) with
P(y) = sum_{k<N} C(N-1+k, k) y^k.  Each root y_k of P gives the zeros z of
z^2 - (2 - 4 y_k) z + 1 = 0; keeping the one inside the unit circle (minimum phase),
H(z) = c (1 + z^-1)^N prod_k (1 - z_k z^-1), scaled so that sum h = sqrt 2.  The
highpass is g_j = (-1)^j h_{2N-1-j}.

One analysis level along an axis of length m (m even) is
    a[k] = sum_j h[j] x[(2k + j) mod m],   d[k] = sum_j g[j] x[(2k + j) mod m],
for k < m/2; synthesis is its transpose.  In 2D, x (columns) is filtered first,
then y (rows), and the level's m x m region is overwritten in Mallat layout:
    [0:m/2, 0:m/2]  low-y  low-x  (recursed on)
    [0:m/2, m/2:m]  low-y  high-x
    [m/2:m, 0:m/2]  high-y low-x
    [m/2:m, m/2:m]  high-y high-x
Coefficients of basis b occupy s[b] (n x n); basis 0 is the Dirac basis (s[0] = x).

Pins: db1 and the closed forms of db2, db3; for every N, sum h = sqrt 2, unit norm,
double-shift orthogonality, N vanishing moments and minimum phase; brute-force
orthogonality of each 2D transform as a matrix; Haar coefficients as block sums;
Psi Psi^dagger = 9 I and ||Psi|| = 3 by the power method.
"""
import math

import numpy as np

from .parallel import pmap


def daubechies(N: int) -> np.ndarray:
    """Minimum-phase Daubechies lowpass filter with N vanishing moments (length 2N)."""
    if N < 1:
        raise ValueError("N >= 1")
    # P(y), coefficients highest degree first for numpy.roots
    p = [math.comb(N - 1 + k, k) for k in range(N)][::-1]
    ys = np.roots(p) if N > 1 else np.zeros(0)
    zs = []
    for y in ys:
        # z + 1/z = 2 - 4y  ->  z^2 - (2 - 4y) z + 1 = 0
        r = np.roots([1.0, -(2.0 - 4.0 * y), 1.0])
        zs.append(r[np.argmin(np.abs(r))])
    h = np.array([1.0 + 0j])
    for _ in range(N):
        h = np.convolve(h, [1.0, 1.0])
    for z in zs:
        h = np.convolve(h, [1.0, -z])
    h = h.real
    return h * (math.sqrt(2.0) / h.sum())


def highpass(h: np.ndarray) -> np.ndarray:
    L = h.size
    return np.array([(-1) ** j * h[L - 1 - j] for j in range(L)])


def _analysis_axis(x, f, axis):
    """c[k] = sum_j f[j] x[(2k + j) mod m] along ``axis``."""
    x = np.moveaxis(x, axis, -1)
    m = x.shape[-1]
    k = np.arange(m // 2)
    out = np.zeros(x.shape[:-1] + (m // 2,), dtype=x.dtype)
    for j in range(f.size):
        out += f[j] * x[..., (2 * k + j) % m]
    return np.moveaxis(out, -1, axis)


def _synthesis_axis(c, f, axis, m):
    """Transpose of _analysis_axis: x[(2k + j) mod m] += f[j] c[k]."""
    c = np.moveaxis(c, axis, -1)
    k = np.arange(m // 2)
    out = np.zeros(c.shape[:-1] + (m,), dtype=c.dtype)
    for j in range(f.size):
        out[..., (2 * k + j) % m] += f[j] * c
    return np.moveaxis(out, -1, axis)


def dwt2(x, h, levels):
    """Periodic separable 2D DWT in Mallat layout (same shape as x)."""
    g = highpass(h)
    c = np.array(x, dtype=np.float64, copy=True)
    m = c.shape[0]
    for _ in range(levels):
        region = c[:m, :m]
        lo_x, hi_x = _analysis_axis(region, h, 1), _analysis_axis(region, g, 1)
        row = np.concatenate([lo_x, hi_x], axis=1)
        lo_y, hi_y = _analysis_axis(row, h, 0), _analysis_axis(row, g, 0)
        c[:m, :m] = np.concatenate([lo_y, hi_y], axis=0)
        m //= 2
    return c


def idwt2(c, h, levels):
    """Adjoint (= inverse, the filter bank being orthonormal) of dwt2."""
    g = highpass(h)
    x = np.array(c, dtype=np.float64, copy=True)
    n = x.shape[0]
    for lev in reversed(range(levels)):
        m = n >> lev
        region = x[:m, :m]
        row = _synthesis_axis(region[: m // 2], h, 0, m) + _synthesis_axis(region[m // 2:], g, 0, m)
        x[:m, :m] = _synthesis_axis(row[:, : m // 2], h, 1, m) + _synthesis_axis(row[:, m // 2:], g, 1, m)
    return x


class Sara:
    """Psi = [I, W_db1^T, ..., W_db8^T] (N x 9N); Psi^dagger x stacks 9 coefficient images."""

    def __init__(self, n: int, levels: int = 4, wavelets=tuple(range(1, 9)), dirac: bool = True):
        if n % (1 << levels):
            raise ValueError("n must be divisible by 2^levels")
        self.n, self.levels, self.dirac = n, levels, dirac
        self.filters = [daubechies(N) for N in wavelets]
        self.b = len(self.filters) + (1 if dirac else 0)

    def adj(self, x):
        """Psi^dagger x -> (b, n, n)."""
        out = [np.array(x, dtype=np.float64)] if self.dirac else []
        out += pmap(lambda h: dwt2(x, h, self.levels), self.filters)
        return np.stack(out)

    def fwd(self, s):
        """Psi s = sum over bases of the synthesis of s[b] -> (n, n)."""
        k = 0
        acc = np.zeros((self.n, self.n))
        if self.dirac:
            acc += s[0]
            k = 1
        for part in pmap(lambda kh: idwt2(s[kh[0]], kh[1], self.levels), list(enumerate(self.filters, start=k))):
            acc += part  # summed in basis order
        return acc
