"""Direction-dependent effects in the interpolation G (oracle, FP64).

Eq. 1 writes a visibility as the Fourier transform of the sky times the DDE term D(l, u),
and Sec. II folds those effects into G: each row of G becomes a kernel of compact support
(the DDE's Fourier transform) convolved with the interpolation kernel.  Reading used here:
the DDE of visibility m is band limited on the oversampled grid,

    D_m(l) = sum_{p, q = -h..h} d_m[q, p] exp(-2 pi i (p l_x + q l_y) / K),

so its visibility is sum_{p,q} d_m[q, p] times the plain visibility at (u + 2 pi p / K,
v + 2 pi q / K), and the plain interpolation at a frequency shifted by whole cells is the
same kernel on shifted cells.  Row m of the DDE-aware G is therefore

    G_dde[m, k] = sum_{p,q} d_m[q, p] G[m, k - (q, p)]     (cell indices mod K),

supported on (J + 2h)^2 cells.  Phi_dde = G_dde F Z (with Z's pre-compensation), and
Phi_dde^dagger uses the conjugate weights.  Written as the sum over (p, q) of shifted
copies of the plain footprint, so duplicate cells simply add.

Pins: a delta DDE (d = 1 at p = q = 0) gives the plain Phi; d = 1 at (p, q) = (1, 0) gives
the plain Phi at u + 2 pi / K; a direct non-uniform DFT of the DDE-modulated sky
(the discretised Eq. 1 with D_m); the complex adjoint identity.
"""
import numpy as np

_CHUNK = 1 << 13


class DDEMeasurement:
    """Phi_dde for a plain measurement operator `meas` and taps d (M, jd, jd) complex.

    Offers the block interface of Measurement (cells, Mi, Gi, GiH, F, Z and their
    adjoints), so Algorithm 1 in oracle/pd.py runs on it unchanged."""

    def __init__(self, meas, d):
        d = np.asarray(d, dtype=np.complex128)
        if d.ndim != 3 or d.shape[0] != meas.M or d.shape[1] != d.shape[2] or d.shape[1] % 2 == 0:
            raise ValueError("d must be (M, jd, jd) with jd odd")
        self.meas, self.taps = meas, d
        self.h = d.shape[1] // 2
        self.M, self.d, self.ny, self.nx = meas.M, meas.d, meas.ny, meas.nx
        self.Ky, self.Kx = meas.Ky, meas.Kx
        self.F, self.FH, self.Z, self.ZH = meas.F, meas.FH, meas.Z, meas.ZH
        self.block_range = meas.block_range
        self._cells = {}

    def footprint(self, lo, hi):
        """Flat cell indices and complex weights of visibilities lo..hi-1: (m, jd^2 J^2)."""
        meas, h = self.meas, self.h
        flat, w = meas.footprint(lo, hi)              # plain taps, (m, J^2)
        ky, kx = flat // meas.Kx, flat % meas.Kx
        idx, wt = [], []
        for q in range(-h, h + 1):
            for p in range(-h, h + 1):
                idx.append(((ky + q) % meas.Ky) * meas.Kx + (kx + p) % meas.Kx)
                wt.append(w * self.taps[lo:hi, h + q, h + p][:, None])
        return np.concatenate(idx, axis=1), np.concatenate(wt, axis=1)

    # ---- the block interface (Eq. 8): M_i is the set of cells block i's kernels touch ----
    def cells(self, i):
        if i not in self._cells:
            lo, hi = self.block_range(i)
            parts = [np.unique(self.footprint(a, min(hi, a + _CHUNK))[0]) for a in range(lo, hi, _CHUNK)]
            self._cells[i] = np.unique(np.concatenate(parts)) if parts else np.zeros(0, np.int64)
        return self._cells[i]

    def Mi(self, i, grid):
        return grid.reshape(-1)[self.cells(i)]

    def Gi(self, i, b_i):
        cells = self.cells(i)
        lo, hi = self.block_range(i)
        out = np.empty(hi - lo, dtype=np.complex128)
        for a in range(lo, hi, _CHUNK):
            b = min(hi, a + _CHUNK)
            flat, w = self.footprint(a, b)
            out[a - lo:b - lo] = np.sum(w * b_i[np.searchsorted(cells, flat)], axis=1)
        return out

    def GiH(self, i, v_i):
        cells = self.cells(i)
        lo, hi = self.block_range(i)
        acc_r = np.zeros(cells.size)
        acc_i = np.zeros(cells.size)
        for a in range(lo, hi, _CHUNK):
            b = min(hi, a + _CHUNK)
            flat, w = self.footprint(a, b)
            loc = np.searchsorted(cells, flat).reshape(-1)
            c = (np.conj(w) * v_i[a - lo:b - lo, None]).reshape(-1)
            acc_r += np.bincount(loc, weights=c.real, minlength=cells.size)
            acc_i += np.bincount(loc, weights=c.imag, minlength=cells.size)
        return acc_r + 1j * acc_i

    def degrid(self, grid, lo=0, hi=None):
        hi = self.meas.M if hi is None else hi
        g = grid.reshape(-1)
        out = np.empty(hi - lo, dtype=np.complex128)
        for a in range(lo, hi, _CHUNK):
            b = min(hi, a + _CHUNK)
            flat, w = self.footprint(a, b)
            out[a - lo:b - lo] = np.sum(w * g[flat], axis=1)
        return out

    def grid_adj(self, y, lo=0, hi=None):
        """G_dde^H y over visibilities lo..hi-1, as a full K x K grid."""
        meas = self.meas
        hi = meas.M if hi is None else hi
        acc_r = np.zeros(meas.Ky * meas.Kx)
        acc_i = np.zeros(meas.Ky * meas.Kx)
        for a in range(lo, hi, _CHUNK):
            b = min(hi, a + _CHUNK)
            flat, w = self.footprint(a, b)
            c = (np.conj(w) * np.asarray(y)[a - lo:b - lo, None]).reshape(-1)
            f = flat.reshape(-1)
            acc_r += np.bincount(f, weights=c.real, minlength=acc_r.size)
            acc_i += np.bincount(f, weights=c.imag, minlength=acc_i.size)
        return (acc_r + 1j * acc_i).reshape(meas.Ky, meas.Kx)

    def phi(self, x):
        meas = self.meas
        return self.degrid(meas.F(meas.Z(x)))

    def phi_adj(self, y, blocks=None):
        """Complex image Phi_dde^dagger y (over the given blocks, default all)."""
        meas = self.meas
        acc = np.zeros((meas.Ky, meas.Kx), dtype=np.complex128)
        for i in range(meas.d) if blocks is None else blocks:
            lo, hi = meas.block_range(i)
            acc += self.grid_adj(np.asarray(y)[lo:hi], lo, hi)
        return meas.ZH(meas.FH(acc))

    def phi_adj_real(self, y, blocks=None):
        return self.phi_adj(y, blocks).real


def nudft_dde(x, uv, d, K):
    """Direct y_m = sum_l x_l D_m(l) exp(-i (u_m l_x + v_m l_y)) with D_m from the taps d
    (the discretised Eq. 1 with DDEs); O(M N jd^2), tiny inputs only."""
    ny, nx = x.shape
    ly = (np.arange(ny) - ny // 2)[:, None]
    lx = (np.arange(nx) - nx // 2)[None, :]
    h = d.shape[1] // 2
    uv = np.asarray(uv, dtype=np.float64)
    out = np.empty(uv.shape[0], dtype=np.complex128)
    for m in range(uv.shape[0]):
        D = np.zeros((ny, nx), dtype=np.complex128)
        for q in range(-h, h + 1):
            for p in range(-h, h + 1):
                D += d[m, h + q, h + p] * np.exp(-2j * np.pi * (p * lx + q * ly) / K)
        out[m] = np.sum(x * D * np.exp(-1j * (uv[m, 0] * lx + uv[m, 1] * ly)))
    return out
