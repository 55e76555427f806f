"""Kaiser-Bessel interpolation kernel (oracle, FP64).

The measurement operator of Eq. 3 interpolates an oversampled FFT grid with a
compactly supported kernel (the paper uses 8 x 8 kernels after Fessler & Sutton 2003)
and Z pre-compensates that interpolation.  The kernel here is the Kaiser-Bessel
window

    phi(t) = I0(beta sqrt(1 - (2 t / J)^2)) / I0(beta),   |t| <= J/2,  0 otherwise,

with J = 8 taps and beta = 2.34 J (the shape commonly used for 2x oversampling).
Its continuous Fourier transform, phi_hat(f) = int phi(t) exp(-2 pi i f t) dt, has the
closed form

    phi_hat(f) = J sinh(sqrt(beta^2 - (pi J f)^2)) / (sqrt(beta^2 - (pi J f)^2) I0(beta)),

valid while pi J |f| < beta (always true for |f| <= 1/4, the band of a 2x grid).

Pins: phi_hat against numerical quadrature of phi; phi symmetric, phi(0) = 1.
"""
import numpy as np
from scipy.special import i0


def kb_beta(J: int) -> float:
    return 2.34 * J


def kb(t, J: int = 8, beta: float | None = None):
    """phi(t), elementwise."""
    if beta is None:
        beta = kb_beta(J)
    t = np.asarray(t, dtype=np.float64)
    arg = 1.0 - (2.0 * t / J) ** 2
    out = np.zeros_like(t)
    inside = arg >= 0.0
    out[inside] = i0(beta * np.sqrt(arg[inside])) / i0(beta)
    return out


def kb_ft(f, J: int = 8, beta: float | None = None):
    """phi_hat(f), elementwise, for pi J |f| < beta."""
    if beta is None:
        beta = kb_beta(J)
    f = np.asarray(f, dtype=np.float64)
    z = np.sqrt(beta * beta - (np.pi * J * f) ** 2)
    return J * np.sinh(z) / (z * i0(beta))
