"""Pins for the oracle's Green's functions (Sect. 2.3, App. A; Eq. (2) for SASHA).

The transformed kernel is checked against direct numerical integration of the real-space
truncated kernel, against its small-kz expansion and its infinite-box limit.
"""

import math

import numpy as np
import pytest
from scipy import integrate

from oracle import green_sasha, green_vgf


def quad_green(k, kz, L):
    """int_{-L}^{L} G_k(z) exp(i kz z) dz with G_k of Sect. 2.3 (real since G_k is even)."""
    if k == 0.0:
        f = lambda z: 0.5 * abs(z) * math.cos(kz * z)  # noqa: E731
    else:
        f = lambda z: -math.exp(-k * abs(z)) / (2.0 * k) * math.cos(kz * z)  # noqa: E731
    # integrate each half separately: the kernel has a kink at z = 0
    pts = max(50, int(abs(kz) * L / math.pi) * 4 + 50)
    v1, _ = integrate.quad(f, -L, 0.0, epsabs=1e-14, epsrel=1e-12, limit=pts)
    v2, _ = integrate.quad(f, 0.0, L, epsabs=1e-14, epsrel=1e-12, limit=pts)
    return v1 + v2


@pytest.mark.parametrize("L", [0.7, 1.0, 6.0, 6.6])
@pytest.mark.parametrize("k", [0.0, 0.05, 1.0, 2.5, 9.0])
@pytest.mark.parametrize("kz", [0.0, 0.3, 1.0, -2.7, 13.0])
def test_green_vgf_matches_quadrature(k, kz, L):
    g = float(green_vgf(k, kz, L))
    ref = quad_green(k, kz, L)
    scale = max(abs(ref), L * L * 1e-3 if k == 0 else 1e-3 / (k * k + kz * kz + 1e-30))
    assert abs(g - ref) <= 1e-9 * scale + 1e-13, (g, ref)


def test_green_vgf_k0_small_kz_expansion():
    # int_0^L z cos(kz z) dz = L^2/2 - kz^2 L^4/8 + kz^4 L^6/144 - ...
    L = 1.3
    for kz in [1e-2, 3e-3]:
        g = float(green_vgf(0.0, kz, L))
        series = L**2 / 2 - kz**2 * L**4 / 8 + kz**4 * L**6 / 144
        assert abs(g - series) < 1e-9
    assert float(green_vgf(0.0, 0.0, L)) == L * L / 2


def test_green_vgf_infinite_box_limit():
    # L -> infinity: the screened kernel transforms to the free-space -1/(k^2 + kz^2)
    for k, kz in [(1.0, 0.0), (2.0, 3.0), (0.5, -1.5)]:
        g = float(green_vgf(k, kz, 60.0))
        assert abs(g + 1.0 / (k * k + kz * kz)) < 1e-12


def test_green_vgf_even_in_kz_and_vectorised():
    k = np.array([0.0, 0.0, 1.5, 3.0])
    kz = np.array([0.0, 2.0, 1.0, 7.5])
    a = green_vgf(k, kz, 2.0)
    b = green_vgf(k, -kz, 2.0)
    assert np.array_equal(a, b)
    for i in range(4):
        assert a[i] == float(green_vgf(k[i], kz[i], 2.0))


def test_green_sasha():
    assert float(green_sasha(0.0, 0.0)) == 0.0
    assert float(green_sasha(3.0, 4.0)) == pytest.approx(-1.0 / 25.0, rel=1e-15)
    assert float(green_sasha(0.0, 2.0)) == pytest.approx(-0.25, rel=1e-15)
