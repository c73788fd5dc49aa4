"""Ray directions and frequency quadratures (inputs of the formal solve).

* ``healpix_ring``: centres of the 12 Nside^2 equal-area HEALPix pixels in the RING
  numbering, from the pixel-to-angle relations of Gorski et al. (2005); the paper uses
  these as its 3-D ray set (Sec. 3.1.3).
* ``uniform_grid``: the frequency grid used by the synthetic workloads, 31 points
  evenly spaced over +-4 local Doppler widths with weights proportional to e^{-x^2},
  end weights halved (trapezoid) and normalised to sum to one.
* ``gauss_hermite``: the Gauss-Hermite rule the paper writes in Sec. 3.1.2, i.e.
  numpy's physicists' Hermite rule with the weights divided by sqrt(pi) so that they
  sum to one against the normalised Gaussian profile.

Every rule returned here is symmetric: x[n] == -x[N-1-n] exactly and w[n] == w[N-1-n].
"""
from __future__ import annotations

import math

import numpy as np


def healpix_ring(nside: int) -> np.ndarray:
    if nside < 1:
        raise ValueError("nside must be >= 1")
    npix = 12 * nside * nside
    ncap = 2 * nside * (nside - 1)
    out = np.empty((npix, 3), dtype=np.float64)
    for p in range(npix):
        if p < ncap:  # north polar cap, ring index counted from the pole
            i = (1 + math.isqrt(1 + 2 * p)) >> 1
            j = p + 1 - 2 * i * (i - 1)
            z = 1.0 - i * i / (3.0 * nside * nside)
            phi = (j - 0.5) * (0.5 * math.pi) / i
        elif p < npix - ncap:  # equatorial belt
            q = p - ncap
            i = q // (4 * nside) + nside
            j = q % (4 * nside) + 1
            shift = 1.0 if ((i + nside) & 1) else 0.5
            z = (2 * nside - i) * 2.0 / (3.0 * nside)
            phi = (j - shift) * math.pi / (2.0 * nside)
        else:  # south polar cap, ring index counted from the south pole
            q = npix - p
            i = (1 + math.isqrt(2 * q - 1)) >> 1
            j = 4 * i + 1 - (q - 2 * i * (i - 1))
            z = -1.0 + i * i / (3.0 * nside * nside)
            phi = (j - 0.5) * (0.5 * math.pi) / i
        st = math.sqrt(max(0.0, (1.0 - z) * (1.0 + z)))
        out[p] = (st * math.cos(phi), st * math.sin(phi), z)
    return out


def axis_pair() -> np.ndarray:
    """Two antipodal rays along +-x (the paper's 1-D test set)."""
    return np.array([[1.0, 0.0, 0.0], [-1.0, 0.0, 0.0]])


def _symmetrise(x: np.ndarray, w: np.ndarray):
    n = x.shape[0]
    x = x.copy()
    w = w.copy()
    for k in range(n // 2):
        x[n - 1 - k] = -x[k]
        w[n - 1 - k] = w[k]
    if n % 2:
        x[n // 2] = 0.0
    return x, w


def uniform_grid(n: int = 31, half_width: float = 4.0):
    k = np.arange(n, dtype=np.float64)
    x = -half_width + 2.0 * half_width * k / (n - 1)
    w = np.exp(-x * x)
    w[0] *= 0.5
    w[-1] *= 0.5
    x, w = _symmetrise(x, w)
    w = w / w.sum()
    x, w = _symmetrise(x, w)
    return x, w


def gauss_hermite(n: int):
    x, w = np.polynomial.hermite.hermgauss(n)
    w = w / math.sqrt(math.pi)
    x, w = _symmetrise(x, w)
    return x, w
