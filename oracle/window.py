"""Kaiser-Bessel window pair for the oracle NFFT (O2).

The paper leaves the window open (Remark 2.2 lists families); this oracle uses
the Kaiser-Bessel pair of the NFFT literature. In grid units t = M_sigma * x,
with shape parameter b = pi (2 - 1/sigma):

    phi(t)     = (1/pi) sinh(b sqrt(m^2 - t^2)) / sqrt(m^2 - t^2),   |t| <= m,
    phi_hat(k) = (1/M_sigma) I_0(m sqrt(b^2 - (2 pi k / M_sigma)^2)).

phi_hat is the continuous Fourier transform of the *untruncated* window
w(x) = phi(M_sigma x) (the section on the NFFT defines hat w as the integral
over R^d); the truncated w_m keeps the closed cube |t| <= m, including the
edge value b/pi (definition of w_m, and the closed inequality of the index
set (2.12)). The d-variate window is the tensor product.

The Fourier pair itself is pinned in the tests by numerical quadrature of the
inverse transform of phi_hat over its compact support.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special


def oversampled_size(M: int, sigma: float) -> int:
    """M_sigma = 2 * ceil(ceil(sigma M) / 2) (the definition before (2.9))."""
    return 2 * math.ceil(math.ceil(sigma * M) / 2)


def shape_b(sigma: float) -> float:
    return math.pi * (2.0 - 1.0 / sigma)


# pi and b in the platform's extended precision
_PI_X = np.longdouble("3.14159265358979323846264338327950288419716939937510")


def phi(t, m: int, sigma: float) -> np.ndarray:
    """Truncated 1-D window w_m in grid units; zero for |t| > m.

    Evaluated in extended precision and rounded once to float64: in float64
    the argument b z of sinh carries the rounding of b and z, and sinh passes
    its relative error on multiplied by b z (up to b m, about 19 at m = 4 and
    28 at m = 6), which the weighted sums of a badly conditioned reconstruction
    then amplify further."""
    t = np.asarray(t, dtype=np.float64)
    tx = t.astype(np.longdouble)
    b = _PI_X * (np.longdouble(2) - np.longdouble(1) / np.longdouble(sigma))
    s = np.longdouble(m) * np.longdouble(m) - tx * tx
    inside = s >= 0
    z = np.sqrt(np.where(inside, s, np.longdouble(0)))
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        val = np.where(z > 0, np.sinh(b * z) / np.where(z > 0, z, np.longdouble(1)), b)
    return np.where(inside, val / _PI_X, np.longdouble(0)).astype(np.float64)


def phi_full(t, m: int, sigma: float) -> np.ndarray:
    """Untruncated 1-D window (sinh branch inside, sin branch outside)."""
    t = np.asarray(t, dtype=np.float64)
    b = shape_b(sigma)
    s = m * m - t * t
    out = np.empty_like(t)
    pos = s > 0
    zp = np.sqrt(s[pos])
    out[pos] = np.sinh(b * zp) / zp / math.pi
    neg = s < 0
    zn = np.sqrt(-s[neg])
    out[neg] = np.sin(b * zn) / zn / math.pi
    out[s == 0] = b / math.pi
    return out


def phi_hat(k, m: int, sigma: float, Ms: int) -> np.ndarray:
    """Continuous Fourier transform of w(x) = phi(Ms x) at frequency k."""
    k = np.asarray(k, dtype=np.float64)
    b = shape_b(sigma)
    a = 2.0 * math.pi * k / Ms
    s = b * b - a * a
    out = np.empty_like(k)
    pos = s >= 0
    out[pos] = special.i0(m * np.sqrt(s[pos]))
    out[~pos] = special.j0(m * np.sqrt(-s[~pos]))
    return out / Ms


def phi_hat_d(kvec: np.ndarray, m: int, sigma: float, Ms: int) -> np.ndarray:
    """Tensor-product transform hat w(k) = prod_t phi_hat(k_t); kvec is (K, d)."""
    out = np.ones(kvec.shape[0])
    for t in range(kvec.shape[1]):
        out = out * phi_hat(kvec[:, t], m, sigma, Ms)
    return out
