"""Blocked measurement operator Phi = G M F Z and its adjoint (oracle, FP64).

Follows Sec. II (Eqs. 2-3) and the block split of Sec. III (Eq. 8):

    Phi_i = G_i M_i F Z,     y = [y_1; ...; y_d],

with these discretisation conventions (the paper leaves them open):

* pixel p of an ny x nx image sits at centred coordinate l = p - n/2, and a
  visibility at (u, v) rad/px measures sum_p x_p exp(-i (u l_x + v l_y)) (the sign of
  Eq. 1, exp(-2 i pi u.l));
* Z zero-pads onto a K = 2n grid per axis (2x oversampling per axis, i.e. k = 4 grid
  points per pixel as in Sec. V), placing pixel l at grid index l mod K, and
  pre-compensates the interpolation by S = 1 / (phi_hat(l_y/K_y) phi_hat(l_x/K_x));
* F is the unnormalised 2D DFT exp(-2 pi i k q / K) (numpy's fft2);
* G interpolates from the J x J grid taps k_j = floor(kappa) - J/2 + 1 + j,
  kappa = u K / (2 pi), weight phi(kappa - k_j) per axis, indices mod K;
* M_i selects the grid cells that block i's footprints touch (kN_i of them), so
  G_i acts on b_i = M_i F Z x only.

The image-side adjoint is complex; Algorithm 1 step 17 keeps its real part.

Pins: direct NUDFT (the discretised Eq. 1) on small problems with error falling as J
grows; <Phi x, y> = <x, Phi^dagger y>; F against an explicit DFT matrix; block
stacking Phi x = [Phi_1 x; ...; Phi_d x].
"""
import numpy as np

from .kaiser_bessel import kb, kb_beta, kb_ft

_CHUNK = 1 << 15


class Measurement:
    def __init__(self, uv, block_off, shape, J: int = 8, beta: float | None = None, osf: int = 2):
        self.ny, self.nx = shape
        self.Ky, self.Kx = osf * self.ny, osf * self.nx
        self.J = J
        self.beta = kb_beta(J) if beta is None else beta
        self.uv = np.asarray(uv, dtype=np.float64)
        self.block_off = np.asarray(block_off, dtype=np.int64)
        self.d = len(self.block_off) - 1
        self.M = int(self.block_off[-1])
        assert self.uv.shape == (self.M, 2)
        ly = np.arange(self.ny) - self.ny // 2
        lx = np.arange(self.nx) - self.nx // 2
        self.rows = ly % self.Ky
        self.cols = lx % self.Kx
        self.sy = 1.0 / kb_ft(ly / self.Ky, J, self.beta)
        self.sx = 1.0 / kb_ft(lx / self.Kx, J, self.beta)
        self._cells = {}

    # ---- Z (with the pre-compensation S), F and their adjoints: Eq. 3 -------------
    def Z(self, x):
        g = np.zeros((self.Ky, self.Kx), dtype=np.complex128)
        g[np.ix_(self.rows, self.cols)] = x * self.sy[:, None] * self.sx[None, :]
        return g

    def ZH(self, g):
        return g[np.ix_(self.rows, self.cols)] * self.sy[:, None] * self.sx[None, :]

    @staticmethod
    def F(z):
        return np.fft.fft2(z)

    def FH(self, b):
        return np.fft.ifft2(b) * (self.Ky * self.Kx)

    # ---- G: Kaiser-Bessel interpolation footprints --------------------------------
    def block_range(self, i):
        return int(self.block_off[i]), int(self.block_off[i + 1])

    def footprint(self, lo, hi):
        """Flat grid indices and weights of the J x J taps of visibilities lo..hi-1."""
        J = self.J
        ku = self.uv[lo:hi, 0] * self.Kx / (2.0 * np.pi)
        kv = self.uv[lo:hi, 1] * self.Ky / (2.0 * np.pi)
        j = np.arange(J)
        kx = np.floor(ku).astype(np.int64)[:, None] - J // 2 + 1 + j
        ky = np.floor(kv).astype(np.int64)[:, None] - J // 2 + 1 + j
        wx = kb(ku[:, None] - kx, J, self.beta)
        wy = kb(kv[:, None] - ky, J, self.beta)
        flat = (ky % self.Ky)[:, :, None] * self.Kx + (kx % self.Kx)[:, None, :]
        w = wy[:, :, None] * wx[:, None, :]
        m = hi - lo
        return flat.reshape(m, J * J), w.reshape(m, J * J)

    def _chunks(self, i):
        lo, hi = self.block_range(i)
        for a in range(lo, hi, _CHUNK):
            b = min(hi, a + _CHUNK)
            yield a - lo, b - lo, self.footprint(a, b)

    # ---- M_i: cell index set of block i (Eq. 8) ------------------------------------
    def cells(self, i):
        if i not in self._cells:
            parts = [np.unique(flat) for _, _, (flat, _) in self._chunks(i)]
            self._cells[i] = np.unique(np.concatenate(parts)) if parts else np.zeros(0, np.int64)
        return self._cells[i]

    def Mi(self, i, grid):
        """b_i = M_i b~ : the kN_i grid values block i needs."""
        return grid.reshape(-1)[self.cells(i)]

    def MiH(self, i, vals):
        """M_i^dagger: embed kN_i values into an otherwise zero K_y x K_x grid."""
        g = np.zeros(self.Ky * self.Kx, dtype=np.complex128)
        g[self.cells(i)] = vals
        return g.reshape(self.Ky, self.Kx)

    def Gi(self, i, b_i):
        """G_i b_i: degrid block i's visibilities from its kN_i cells."""
        cells = self.cells(i)
        lo, hi = self.block_range(i)
        out = np.empty(hi - lo, dtype=np.complex128)
        for a, b, (flat, w) in self._chunks(i):
            loc = np.searchsorted(cells, flat)
            out[a:b] = np.sum(w * b_i[loc], axis=1)
        return out

    def GiH(self, i, v_i):
        """G_i^dagger v_i: grid block i's visibilities onto its kN_i cells."""
        cells = self.cells(i)
        acc_r = np.zeros(cells.size)
        acc_i = np.zeros(cells.size)
        for a, b, (flat, w) in self._chunks(i):
            loc = np.searchsorted(cells, flat).reshape(-1)
            c = (w * v_i[a:b, None]).reshape(-1)
            acc_r += np.bincount(loc, weights=c.real, minlength=cells.size)
            acc_i += np.bincount(loc, weights=c.imag, minlength=cells.size)
        return acc_r + 1j * acc_i

    # ---- whole operators -----------------------------------------------------------
    def degrid(self, i, grid):
        """G_i M_i grid for block i, gathering straight from the full grid."""
        lo, hi = self.block_range(i)
        g = grid.reshape(-1)
        out = np.empty(hi - lo, dtype=np.complex128)
        for a, b, (flat, w) in self._chunks(i):
            out[a:b] = np.sum(w * g[flat], axis=1)
        return out

    def grid_adj(self, i, v_i):
        """M_i^dagger G_i^dagger v_i as a full K_y x K_x grid."""
        acc_r = np.zeros(self.Ky * self.Kx)
        acc_i = np.zeros(self.Ky * self.Kx)
        for a, b, (flat, w) in self._chunks(i):
            c = (w * v_i[a:b, None]).reshape(-1)
            f = flat.reshape(-1)
            acc_r += np.bincount(f, weights=c.real, minlength=acc_r.size)
            acc_i += np.bincount(f, weights=c.imag, minlength=acc_i.size)
        return (acc_r + 1j * acc_i).reshape(self.Ky, self.Kx)

    def phi_block(self, i, x):
        return self.degrid(i, self.F(self.Z(x)))

    def phi(self, x):
        """y = Phi x (complex, length M, blocks stacked as in Eq. 8)."""
        grid = self.F(self.Z(x))
        return np.concatenate([self.degrid(i, grid) for i in range(self.d)])

    def phi_adj(self, y, blocks=None):
        """Phi^dagger y = Z^dagger F^dagger sum_i M_i^dagger G_i^dagger y_i (complex image)."""
        acc = np.zeros((self.Ky, self.Kx), dtype=np.complex128)
        for i in range(self.d) if blocks is None else blocks:
            lo, hi = self.block_range(i)
            acc += self.grid_adj(i, y[lo:hi])
        return self.ZH(self.FH(acc))

    def phi_adj_real(self, y, blocks=None):
        """Re Phi^dagger y, the adjoint of Phi restricted to real images."""
        return self.phi_adj(y, blocks).real


def nudft(x, uv):
    """Direct non-uniform DFT y_m = sum_p x_p exp(-i (u_m l_x + v_m l_y)), l = p - n/2.

    The discretised Eq. 1 without direction-dependent effects; O(M N), tiny inputs only.
    """
    ny, nx = x.shape
    ly = np.arange(ny) - ny // 2
    lx = np.arange(nx) - nx // 2
    uv = np.asarray(uv, dtype=np.float64)
    ph = uv[:, 0:1, None] * lx[None, None, :] + uv[:, 1:2, None] * ly[None, :, None]
    return np.sum(np.exp(-1j * ph) * x[None, :, :], axis=(1, 2))
