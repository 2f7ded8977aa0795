"""Pins of the oracle's output for the hydrodynamics: vertical ghost cells (Sect. 2.4: in the
ghost cells the vertical gradient of Phi equals that of the last active cell) and the
acceleration -grad Phi by centred differences with shear-periodic x, periodic y and the ghost
layers in z.  The differences are checked against exact derivatives of a smooth shear-periodic
potential at their orders of accuracy, so a wrong neighbour, sign, spacing or shear direction
at the x edges shows up as an O(1) error."""

import math

import numpy as np
import pytest

from oracle import Box, Shear, fill_ghosts, gravity
from oracle.shearing_poisson import cell_centres, shear_offset


def test_ghosts_continue_the_last_gradient():
    rng = np.random.default_rng(1)
    phi = rng.standard_normal((3, 4, 6))
    for ng in (1, 2, 3):
        g = fill_ghosts(phi, ng)
        assert g.shape == (3, 4, 6 + 2 * ng)
        assert np.array_equal(g[:, :, ng:ng + 6], phi)
        d_lo = phi[:, :, 1] - phi[:, :, 0]
        d_hi = phi[:, :, 5] - phi[:, :, 4]
        for k in range(ng):
            assert np.allclose(g[:, :, k + 1] - g[:, :, k], d_lo, rtol=0, atol=1e-12)
            assert np.allclose(g[:, :, ng + 6 + k] - g[:, :, ng + 5 + k], d_hi, rtol=0, atol=1e-12)
    # a potential linear in z is continued exactly
    z = np.arange(6, dtype=float)
    lin = np.broadcast_to(0.3 + 1.7 * z, (2, 2, 6))
    g = fill_ghosts(lin, 2)
    assert np.allclose(g[0, 0], 0.3 + 1.7 * np.arange(-2, 8), atol=1e-12)


def _analytic(box, s, X, Y, Z):
    """A smooth shear-periodic potential (a plane wave in the shearing frame y + s x, times a
    Gaussian in z) and its exact gradient."""
    kx, ky = 2 * math.pi / box.lx, 4 * math.pi / box.ly
    u = kx * X + ky * (Y + s * X)
    ez = np.exp(-0.5 * Z * Z)
    phi = np.cos(u) * ez
    dx = -np.sin(u) * (kx + ky * s) * ez
    dy = -np.sin(u) * ky * ez
    dz = -Z * np.cos(u) * ez
    return phi, -dx, -dy, -dz


@pytest.mark.parametrize("t", [0.0, 0.41])
def test_gravity_second_order(t):
    errs = {"x": [], "xb": [], "y": [], "z": [], "zb": []}
    for n in (16, 32, 64):
        box = Box(n, n, n, 1.0, 1.5, 4.0)
        sh = Shear(q=1.5, omega=1.0, t=t, G=1.0)
        s = shear_offset(sh.q, sh.omega, box.lx, box.ly, sh.t) / box.lx
        x, y, z = cell_centres(box)
        X, Y, Z = np.meshgrid(x, y, z, indexing="ij")
        phi, gx, gy, gz = _analytic(box, s, X, Y, Z)
        ax, ay, az = gravity(fill_ghosts(phi, 2), box, sh, 2)
        sc = np.abs(gx).max()
        errs["x"].append(np.abs(ax - gx)[1:-1].max() / sc)  # interior rows
        # edge rows: the neighbour beyond the edge is interpolated in y (O(dy^2) error over 2 dx)
        errs["xb"].append(np.abs(ax - gx)[[0, -1]].max() / sc)
        errs["y"].append(np.abs(ay - gy).max() / sc)
        errs["z"].append(np.abs(az - gz)[:, :, 1:-1].max() / sc)      # interior: centred
        errs["zb"].append(np.abs(az - gz)[:, :, [0, -1]].max() / sc)  # edge cells: one-sided
    bounds = [("x", 1.8, 2.3), ("y", 1.8, 2.3), ("z", 1.8, 2.3), ("zb", 0.8, 1.3)]
    bounds.append(("xb", 0.8, 2.3) if t else ("xb", 1.8, 2.3))  # t = 0: nothing is interpolated
    for key, lo, hi in bounds:
        e = errs[key]
        orders = [math.log2(e[i] / e[i + 1]) for i in range(len(e) - 1)]
        assert min(orders) > lo and max(orders) < hi, (key, e, orders)
