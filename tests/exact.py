"""Exact reference potentials for the paper's analytic test densities (test helpers).

Independent of the oracle: these evaluate the paper's closed forms in extended precision
(mpmath) or integrate the real-space Green's function by adaptive quadrature.
"""

from __future__ import annotations

import math

import mpmath as mp
import numpy as np
from scipy import integrate

mp.mp.dps = 40


def gaussian_1d_closed(z, z0: float, lz: float, H: float = 1.0) -> np.ndarray:
    """Sect. 3.1 closed form divided by 4 pi G, for a Gaussian of scale height H truncated to
    [-Lz/2, Lz/2] (the paper prints H = 1; general H by substituting z/H, z0/H and scaling by H^2).
    The integration constant is zero, as in the paper."""
    out = []
    r2 = mp.sqrt(2)
    H = mp.mpf(H)
    zh0 = mp.mpf(z0) / H
    lh = mp.mpf(lz) / H
    a = -mp.mpf(1) / 2 * mp.sqrt(mp.pi / 2) * (mp.erf((-lh / 2 - zh0) / r2) + mp.erf((lh / 2 - zh0) / r2))
    for zz in np.atleast_1d(z):
        zh = mp.mpf(float(zz)) / H
        u = zh - zh0
        v = mp.sqrt(mp.pi / 2) * u * mp.erf(u / r2) + mp.e ** (-u * u / 2) + a * zh
        out.append(float(v * H * H))
    return np.array(out)


def gaussian_1d_quad(z, z0: float, lz: float, H: float = 1.0) -> np.ndarray:
    """The same potential (over 4 pi G) as the convolution with the 1-D Green's function
    |z - z'|/2 of Sect. 2.3 over the box, by adaptive quadrature.  This fixes the additive
    constant that the closed form leaves free (VGF convolves with exactly this kernel)."""
    out = []
    for zz in np.atleast_1d(z):
        zz = float(zz)
        f = lambda zp: 0.5 * abs(zz - zp) * math.exp(-0.5 * ((zp - z0) / H) ** 2)  # noqa: E731
        v1, _ = integrate.quad(f, -0.5 * lz, zz, epsabs=1e-15, epsrel=1e-13, limit=200)
        v2, _ = integrate.quad(f, zz, 0.5 * lz, epsabs=1e-15, epsrel=1e-13, limit=200)
        out.append(v1 + v2)
    return np.array(out)


def cos_gauss_bracket(z, k: float, H: float, lz: float) -> np.ndarray:
    """Sect. 3.2 closed form: the bracket [2a cosh(kz) + F+ + F-] for one horizontal mode of
    wavenumber k, i.e. Phi/(4 pi G) per unit horizontal amplitude.  Evaluated in 40-digit
    arithmetic because the printed form cancels badly for large kH."""
    k = mp.mpf(k)
    H = mp.mpf(H)
    lz = mp.mpf(lz)
    r2 = mp.sqrt(2)
    a = -mp.sqrt(mp.pi / 2) * (H / (2 * k)) * mp.e ** ((k * H) ** 2 / 2) * mp.erf((k * H + lz / (2 * H)) / r2)
    out = []
    for zz in np.atleast_1d(z):
        zz = mp.mpf(float(zz))

        def F(sg):
            return mp.sqrt(mp.pi / 2) * (H / (2 * k)) * mp.e ** ((k * H / 2) * (k * H + sg * 2 * zz / H)) * mp.erf(
                (k * H + sg * zz / H) / r2
            )

        out.append(float(2 * a * mp.cosh(k * zz) + F(1) + F(-1)))
    return np.array(out)


def screened_quad(z, k: float, H: float, lz: float) -> np.ndarray:
    """Same bracket as cos_gauss_bracket, as the convolution of the truncated Gaussian with the
    screened Green's function -exp(-k|z-z'|)/(2k) of Sect. 2.3, by adaptive quadrature."""
    out = []
    for zz in np.atleast_1d(z):
        zz = float(zz)
        f = lambda zp: -math.exp(-k * abs(zz - zp)) / (2 * k) * math.exp(-0.5 * (zp / H) ** 2)  # noqa: E731
        v1, _ = integrate.quad(f, -0.5 * lz, zz, epsabs=1e-15, epsrel=1e-13, limit=200)
        v2, _ = integrate.quad(f, zz, 0.5 * lz, epsabs=1e-15, epsrel=1e-13, limit=200)
        out.append(v1 + v2)
    return np.array(out)


def shifted_rel_err(num: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Pointwise error of Sect. 3.1 after shifting both potentials to minimum 1 (Sect. 3.1, 3.2)."""
    a = num - num.min() + 1.0
    b = ref - ref.min() + 1.0
    return np.abs((a - b) / b)


def paper_norm(num: np.ndarray, ref: np.ndarray) -> float:
    """||eps||_2 = sqrt(sum eps^2)/N of Sect. 3.3, N = number of cells."""
    e = shifted_rel_err(num, ref)
    return math.sqrt(float((e * e).sum())) / e.size
