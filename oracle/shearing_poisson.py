"""Plain FP64 CPU oracle for the shearing-box Poisson solve with vertical vacuum boundaries.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link this
module: only the tests, the smoke check and the CPU-baseline leg of the benchmark use it.
It shares no code with the HIP library and never reads anything the HIP library wrote.

It computes, slowly and obviously, what the paper's method computes (Rendon Restrepo &
Gressel, "An efficient spectral Poisson solver for the NIRVANA code: the shearing-box case
with vertical vacuum boundary conditions"):

  1. map the density to the fully periodic (shearing) frame, Sect. 2.1: a y-shift by
     -Delta_y0(t) x / Lx, either spectral (the Fourier-interpolation, SAFI, variant) or by
     linear interpolation between neighbouring y cells (the other variant the section names);
  2. Hockney zero padding of z from Nz to M = P*Nz cells, Sect. 2.2 and Sect. 2.4;
  3. forward transform in y (real half spectrum), x and z;
  4. multiply by the Green's function evaluated at the sheared wave vector
     k(t) = (Kx + (Delta_y0/Lx) Ky, Ky, kz) of Sect. 2.1:
       - VGF-HybridBC: the regularised transform G^L(k, kz) of Sect. 2.3
         (equation "Green's function regularized in Fourier", derived in App. A);
       - SASHA: the classical spectral kernel -1/|k|^2 of Eq. (2), with the zero mode
         removed (mean subtraction, Sect. 2.2) and the analytic Phi_0(z) added back;
  5. inverse transforms, scaled by 4 pi G (Sect. 2.3, Phi = 4 pi G F^-1(G rho));
  6. keep the first Nz cells, undo the y-shift, inverse y transform to real space.

numpy's FFT serves as the transform primitive.  Step order and notation follow the paper;
there is no fusion, blocking or reordering beyond the library calls.

Readings taken where the paper is silent (each listed in the design notes):
  * shear sign: lab fields satisfy f(x+Lx, y) = f(x, y+Delta_y0); the remap multiplies the
    y spectrum by exp(-i Ky s x), s = Delta_y0/Lx, the un-remap by exp(+i Ky s x);
  * q is a parameter (the paper fixes q = 3/2); Delta_y0 = fmod(q Omega Lx t, Ly) in [0, Ly);
  * cell-centred grids x_i = (i+1/2) Lx/Nx, y_j = (j+1/2) Ly/Ny, z_k = -Lz/2 + (k+1/2) Lz/Nz;
  * the y-Nyquist plane is dropped (a sheared real field has no real Nyquist component);
    x and z mode numbers follow numpy's fftfreq (Nyquist counted negative);
  * discrete normalisation: Phi = 4 pi G * IDFT(G * DFT(rho_pad)), no cell-volume factor;
  * truncation length L = alpha * Lz with default alpha = P/2, i.e. L is half the padded
    period, so the periodic images of the truncated kernel never overlap the box;
  * SASHA mean <rho> is taken over the padded periodic domain, m = sum(rho)/(Nx Ny M), and
    z0 = sum(z rho)/sum(rho) (z0 = 0 and Phi_0 = 0 if sum(rho) = 0).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

FOUR_PI = 4.0 * math.pi


@dataclass(frozen=True)
class Box:
    """Grid and domain of one shearing box (oracle-side description)."""

    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    pad: int = 2            # P: z is padded from Nz to P*Nz cells
    alpha: float = 0.0      # L = alpha*Lz; 0 selects alpha = P/2
    method: str = "vgf"     # "vgf" (VGF-HybridBC) or "sasha"
    remap: str = "spectral"  # map to the periodic frame: "spectral" (Fourier shift) or "linear"

    @property
    def m(self) -> int:
        return self.pad * self.nz

    @property
    def trunc_len(self) -> float:
        a = self.alpha if self.alpha > 0.0 else 0.5 * self.pad
        return a * self.lz


@dataclass(frozen=True)
class Shear:
    """Per-solve parameters: shear rate q, rotation Omega, time t, gravitational constant G."""

    q: float = 1.5
    omega: float = 1.0
    t: float = 0.0
    G: float = 1.0


def shear_offset(q: float, omega: float, lx: float, ly: float, t: float) -> float:
    """Delta_y0(t) = mod(q Omega Lx t, Ly), wrapped into [0, Ly) (Sect. 2.1, q = 3/2 there)."""
    d = math.fmod(q * omega * lx * t, ly)
    if d < 0.0:
        d += ly
    if d >= ly:
        d = 0.0
    return d


def mode_numbers(n: int) -> np.ndarray:
    """Signed DFT mode numbers 0..n/2-1, -n/2..-1 (Nyquist counted negative)."""
    m = np.arange(n, dtype=np.int64)
    m[m >= n // 2] -= n
    return m


def green_vgf(k, kz, L: float) -> np.ndarray:
    """Fourier transform of the truncated screened Green's function, G^L(k, kz).

    Sect. 2.3, equation "Green's function regularized in Fourier" (derived in App. A):
      L^2/2                                              if k = 0, kz = 0
      (kz L sin(kz L) + cos(kz L) - 1) / kz^2            if k = 0, kz != 0
      -(exp(-k L) ((kz/k) sin(kz L) - cos(kz L)) + 1) / (k^2 + kz^2)   otherwise
    Written exactly as printed (no rearrangement).
    """
    k, kz = np.broadcast_arrays(np.asarray(k, dtype=np.float64), np.asarray(kz, dtype=np.float64))
    out = np.empty(k.shape, dtype=np.float64)
    k0 = k == 0.0
    kz0 = kz == 0.0
    c1 = k0 & kz0
    c2 = k0 & ~kz0
    c3 = ~k0
    out[c1] = L * L / 2.0
    q = kz[c2]
    out[c2] = (q * L * np.sin(q * L) + np.cos(q * L) - 1.0) / (q * q)
    kk, q = k[c3], kz[c3]
    out[c3] = -(np.exp(-kk * L) * ((q / kk) * np.sin(q * L) - np.cos(q * L)) + 1.0) / (kk * kk + q * q)
    return out


def green_sasha(k, kz) -> np.ndarray:
    """Periodic spectral kernel of Eq. (2), -1/|k|^2, with the zero mode removed (Sect. 2.2)."""
    k, kz = np.broadcast_arrays(np.asarray(k, dtype=np.float64), np.asarray(kz, dtype=np.float64))
    k2 = k * k + kz * kz
    out = np.zeros(k.shape, dtype=np.float64)
    nz = k2 != 0.0
    out[nz] = -1.0 / k2[nz]
    return out


def cell_centres(box: Box):
    x = (np.arange(box.nx) + 0.5) * (box.lx / box.nx)
    y = (np.arange(box.ny) + 0.5) * (box.ly / box.ny)
    z = -0.5 * box.lz + (np.arange(box.nz) + 0.5) * (box.lz / box.nz)
    return x, y, z


def sheared_wavenumbers(box: Box, s: float):
    """Physical horizontal wavenumber k = |(Kx + s Ky, Ky)| for every (mx, my<Ny/2) (Sect. 2.1),
    and the padded vertical wavenumbers kz.  k is exactly 0 only at mx = my = 0."""
    Kx = (2.0 * math.pi / box.lx) * mode_numbers(box.nx)
    Ky = (2.0 * math.pi / box.ly) * np.arange(box.ny // 2)
    kx = Kx[:, None] + s * Ky[None, :]
    k = np.sqrt(kx * kx + Ky[None, :] ** 2)
    kz = (2.0 * math.pi / (box.pad * box.lz)) * mode_numbers(box.m)
    return k, kz, Ky


def sasha_phi0(rho: np.ndarray, box: Box, G: float) -> np.ndarray:
    """Phi_0(z) = 4 pi G <rho> z (z/2 - z0), z0 = <z rho>/<rho> (Sect. 2.2), as a length-Nz profile."""
    _, _, z = cell_centres(box)
    col = rho.sum(axis=(0, 1))
    total = col.sum()
    if total == 0.0:
        return np.zeros(box.nz)
    mean = total / (box.nx * box.ny * box.m)
    z0 = (z * col).sum() / total
    return FOUR_PI * G * mean * z * (0.5 * z - z0)


def shift_y_linear(f: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Sample f[i, :, :] at the fractional y index j + d[i] by linear interpolation between the
    two neighbouring cells (periodic in y): the real-space remap of Sect. 2.1 (linear variant)."""
    ny = f.shape[1]
    out = np.empty_like(f)
    j = np.arange(ny)
    for i in range(f.shape[0]):
        m = math.floor(d[i])
        w = d[i] - m
        out[i] = (1.0 - w) * f[i, (j + m) % ny, :] + w * f[i, (j + m + 1) % ny, :]
    return out


def solve(rho: np.ndarray, box: Box, shear: Shear) -> np.ndarray:
    """Potential Phi on the Nx x Ny x Nz box for density rho (C order [x][y][z]), in FP64."""
    rho = np.asarray(rho, dtype=np.float64)
    if rho.shape != (box.nx, box.ny, box.nz):
        raise ValueError(f"rho shape {rho.shape} != box {(box.nx, box.ny, box.nz)}")
    nx, ny, nz, M = box.nx, box.ny, box.nz, box.m
    dy0 = shear_offset(shear.q, shear.omega, box.lx, box.ly, shear.t)
    s = dy0 / box.lx
    x, _, _ = cell_centres(box)
    k, kz, Ky = sheared_wavenumbers(box, s)

    # 1. Map to the periodic frame (Sect. 2.1): the periodic field at (x, y) is the lab field at
    #    (x, y - s x).  Spectral: multiply the y spectrum by exp(-i Ky s x).  Linear: sample the
    #    lab field at y - s x by linear interpolation in y.  Then drop the y-Nyquist.
    if box.remap == "spectral":
        rt = np.fft.rfft(rho, axis=1)[:, : ny // 2, :]
        remap = np.exp(-1j * s * np.outer(x, Ky))
        rt = rt * remap[:, :, None]
    elif box.remap == "linear":
        cells = s * x / (box.ly / ny)  # shift s x in y cells
        rt = np.fft.rfft(shift_y_linear(rho, -cells), axis=1)[:, : ny // 2, :]
    else:
        raise ValueError(box.remap)

    # 2. Zero padding of z to M = P*Nz (Hockney).
    rp = np.zeros((nx, ny // 2, M), dtype=np.complex128)
    rp[:, :, :nz] = rt

    # 3. Remaining forward transforms (x, z).
    rh = np.fft.fft(np.fft.fft(rp, axis=0), axis=2)

    # 4. Green's function at the sheared wave vector.
    if box.method == "vgf":
        g = green_vgf(k[:, :, None], kz[None, None, :], box.trunc_len)
    elif box.method == "sasha":
        g = green_sasha(k[:, :, None], kz[None, None, :])
    else:
        raise ValueError(box.method)
    ph = g * rh

    # 5. Inverse transforms (z, x) and extraction of the physical cells.
    ph = np.fft.ifft(np.fft.ifft(ph, axis=2), axis=0)[:, :, :nz]

    # 6. Reverse mapping and inverse y transform; scale by 4 pi G.  The lab potential at (x, y)
    #    is the periodic one at (x, y + s x).
    if box.remap == "spectral":
        ph = ph * np.conj(remap)[:, :, None]
    full = np.zeros((nx, ny // 2 + 1, nz), dtype=np.complex128)
    full[:, : ny // 2, :] = ph
    phi = np.fft.irfft(full, n=ny, axis=1) * (FOUR_PI * shear.G)
    if box.remap == "linear":
        phi = shift_y_linear(phi, cells)

    if box.method == "sasha":
        phi = phi + sasha_phi0(rho, box, shear.G)[None, None, :]
    return phi


# ------------------------------------------------------------------------------------------
# Output for the hydrodynamics: vertical ghost cells and the gravitational acceleration.


def fill_ghosts(phi: np.ndarray, ng: int) -> np.ndarray:
    """Potential with ng ghost layers below and above the box (Sect. 2.4): in the ghost cells
    the vertical gradient equals that of the last active cell, i.e. Phi continues linearly
    with the slope between the two outermost active cells.  Returns [nx][ny][nz + 2 ng]."""
    nx, ny, nz = phi.shape
    out = np.empty((nx, ny, nz + 2 * ng))
    out[:, :, ng:ng + nz] = phi
    lo = phi[:, :, 1] - phi[:, :, 0]
    hi = phi[:, :, nz - 1] - phi[:, :, nz - 2]
    for g in range(1, ng + 1):
        out[:, :, ng - g] = phi[:, :, 0] - g * lo
        out[:, :, ng + nz - 1 + g] = phi[:, :, nz - 1] + g * hi
    return out


def gravity(phi_g: np.ndarray, box: Box, shear: Shear, ng: int):
    """Acceleration g = -grad Phi at the cell centres by second-order centred differences,
    from the potential with ng >= 1 ghost layers in z (as filled by fill_ghosts).

    y is periodic.  x is shear-periodic: the lab field satisfies f(x + Lx, y) = f(x, y + Dy0),
    so the neighbour beyond the last x row is the first row sampled at y + Dy0 and the one
    before the first row is the last row sampled at y - Dy0, both by linear interpolation in y
    (the real-space shift used by the linear remap).  z uses the ghost layers."""
    if ng < 1:
        raise ValueError("the z difference needs at least one ghost layer")
    nx, ny, nz = box.nx, box.ny, box.nz
    phi = phi_g[:, :, ng:ng + nz]
    dx, dy, dz = box.lx / nx, box.ly / ny, box.lz / nz
    cells = shear_offset(shear.q, shear.omega, box.lx, box.ly, shear.t) / dy
    first = shift_y_linear(phi[:1], np.array([cells]))       # row 0 at y + Dy0
    last = shift_y_linear(phi[-1:], np.array([-cells]))      # row nx-1 at y - Dy0
    ext = np.concatenate([last, phi, first], axis=0)
    gx = -(ext[2:] - ext[:-2]) / (2.0 * dx)
    gy = -(np.roll(phi, -1, axis=1) - np.roll(phi, 1, axis=1)) / (2.0 * dy)
    gz = -(phi_g[:, :, ng + 1:ng + nz + 1] - phi_g[:, :, ng - 1:ng + nz - 1]) / (2.0 * dz)
    return gx, gy, gz
