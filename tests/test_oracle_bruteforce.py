"""Brute-force pin of the oracle's transform pipeline on tiny grids.

The discrete operator the method applies is written out as explicit sums over Fourier modes
with physical coordinates (no FFTs, no separable steps): the sheared mode
exp(i[Kx x + Ky (y + s x) + kz z]) of Sect. 2.1, the Green's function of Sect. 2.3 at the
sheared wave vector, zero padding of z to P*Nz cells, the real-field half-spectrum sum over
Ky >= 0 with the Nyquist row excluded, and the 4 pi G normalisation.  Any slip in the
oracle's index maps, phase signs, padding, extraction or scaling breaks agreement.
"""

import math

import numpy as np
import pytest

from oracle import Box, Shear, green_sasha, green_vgf, solve


def brute_force(rho, lx, ly, lz, pad, alpha, method, q, omega, t, G):
    nx, ny, nz = rho.shape
    M = pad * nz
    L = (alpha if alpha > 0 else pad / 2.0) * lz
    dy0 = (q * omega * lx * t) % ly
    s = dy0 / lx
    xs = (np.arange(nx) + 0.5) * lx / nx
    ys = (np.arange(ny) + 0.5) * ly / ny
    zs = -lz / 2 + (np.arange(M) + 0.5) * lz / nz  # extended through the padding
    X, Y, Z = np.meshgrid(xs, ys, zs[:nz], indexing="ij")
    cells = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    rv = rho.ravel()
    phi = np.zeros(nx * ny * nz)
    for mx in range(nx):
        ix = mx if mx < nx // 2 else mx - nx
        Kx = 2 * math.pi * ix / lx
        for my in range(ny // 2):
            Ky = 2 * math.pi * my / ly
            k = math.sqrt((Kx + s * Ky) ** 2 + Ky**2)
            w = 1.0 if my == 0 else 2.0
            for mz in range(M):
                iz = mz if mz < M // 2 else mz - M
                kz = 2 * math.pi * iz / (pad * lz)
                arg = Kx * cells[0] + Ky * (cells[1] + s * cells[0]) + kz * cells[2]
                e = np.exp(1j * arg)
                rhat = np.sum(rv * np.conj(e))
                if method == "vgf":
                    g = float(green_vgf(k, kz, L))
                else:
                    g = float(green_sasha(k, kz))
                phi += w * np.real(g * rhat * e)
    phi *= 4 * math.pi * G / (nx * ny * M)
    phi = phi.reshape(nx, ny, nz)
    if method == "sasha":
        tot = rho.sum()
        if tot != 0:
            mean = tot / (nx * ny * M)
            zc = zs[:nz]
            z0 = (rho.sum(axis=(0, 1)) * zc).sum() / tot
            phi += 4 * math.pi * G * mean * zc * (zc / 2 - z0)
    return phi


CASES = [
    # nx, ny, nz, lx, ly, lz, pad, alpha, method, t
    (8, 8, 4, 1.0, 1.0, 1.0, 2, 0.0, "vgf", 0.3),
    (6, 8, 4, 1.5, 2.0, 0.8, 2, 0.0, "vgf", 0.3),
    (4, 6, 4, 1.0, 3.0, 2.0, 4, 1.1, "vgf", 1.7),
    (8, 4, 6, 2.0, 1.0, 1.0, 2, 0.0, "sasha", 0.45),
    (4, 8, 4, 1.0, 1.0, 1.0, 4, 0.0, "sasha", 0.0),
]


@pytest.mark.parametrize("case", CASES)
def test_oracle_equals_brute_force(case):
    nx, ny, nz, lx, ly, lz, pad, alpha, method, t = case
    rng = np.random.default_rng(7 + nx * 100 + ny * 10 + nz)
    rho = rng.standard_normal((nx, ny, nz)) + 0.5
    q, omega, G = 1.5, 0.9, 1.3
    ref = brute_force(rho, lx, ly, lz, pad, alpha, method, q, omega, t, G)
    box = Box(nx, ny, nz, lx, ly, lz, pad=pad, alpha=alpha, method=method)
    got = solve(rho, box, Shear(q=q, omega=omega, t=t, G=G))
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < 1e-13, err
