"""Pins of the oracle's linear-interpolation remap (the real-space variant of the mapping to
the periodic frame named in Sect. 2.1, next to the spectral one):

* at t = 0 nothing moves, so it equals the spectral remap;
* when every row's shift s x_i is a whole number of y cells, linear interpolation is an exact
  cyclic shift, and so is the spectral phase: the two remaps agree (the spectral one is itself
  pinned by the brute-force definition and the closed forms);
* for a smooth sheared wave its difference from the spectral remap falls at second order in
  the y spacing (linear interpolation error), with the physics fixed.
"""

import math

import numpy as np
import pytest

from oracle import Box, Shear, solve
from oracle.shearing_poisson import cell_centres


def _pair(box_kw, rho, shear):
    a = solve(rho, Box(**box_kw, remap="spectral"), shear)
    b = solve(rho, Box(**box_kw, remap="linear"), shear)
    return a, b


@pytest.mark.parametrize("method", ["vgf", "sasha"])
def test_linear_equals_spectral_at_t0(method):
    rng = np.random.default_rng(3)
    rho = rng.standard_normal((8, 12, 6)) + 0.3
    kw = dict(nx=8, ny=12, nz=6, lx=1.0, ly=1.5, lz=1.0, method=method)
    a, b = _pair(kw, rho, Shear(q=1.5, omega=1.0, t=0.0, G=1.0))
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


@pytest.mark.parametrize(
    "case",
    [
        # nx, ny, nz, lx, ly, lz, q, omega, t: s (i + 1/2) dx/dy is an odd integer for every row
        (8, 32, 4, 1.0, 4.0, 1.0, 2.0, 1.0, 1.0),  # s = 2, dx = dy
        (4, 16, 6, 2.0, 4.0, 1.0, 1.0, 1.0, 1.0),  # s = 1, dx = 2 dy
    ],
)
@pytest.mark.parametrize("method", ["vgf", "sasha"])
def test_linear_equals_spectral_for_whole_cell_shifts(case, method):
    nx, ny, nz, lx, ly, lz, q, om, t = case
    s = math.fmod(q * om * lx * t, ly) / lx
    x = (np.arange(nx) + 0.5) * lx / nx
    shifts = s * x / (ly / ny)
    assert np.allclose(shifts, np.round(shifts), atol=1e-12) and np.all(np.round(shifts) != 0)
    rng = np.random.default_rng(nx + ny)
    rho = rng.standard_normal((nx, ny, nz)) + 0.5
    kw = dict(nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz, method=method)
    a, b = _pair(kw, rho, Shear(q=q, omega=om, t=t, G=0.8))
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_linear_remap_converges_at_second_order():
    # sheared plane wave cos(Kx x) cos(Ky (y + s x)) exp(-z^2/2H^2) at a fractional shift
    errs = []
    for ny in (16, 32, 64, 128):
        kw = dict(nx=8, ny=ny, nz=8, lx=1.0, ly=1.0, lz=1.0)
        box = Box(**kw)
        x, y, z = cell_centres(box)
        sh = Shear(q=1.5, omega=1.0, t=0.37, G=1.0)
        s = math.fmod(sh.q * sh.omega * box.lx * sh.t, box.ly) / box.lx
        X, Y, Z = np.meshgrid(x, y, z, indexing="ij")
        rho = np.cos(2 * math.pi * X) * np.cos(2 * math.pi * (Y + s * X)) * np.exp(-0.5 * (Z / 0.2) ** 2)
        a, b = _pair(kw, rho, sh)
        errs.append(np.linalg.norm(a - b) / np.linalg.norm(a))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert errs[0] > 1e-4  # the linear remap is not the spectral one at fractional shifts
    assert min(orders) > 1.8 and max(orders) < 2.3, (errs, orders)
