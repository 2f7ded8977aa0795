"""Physics pins for the oracle: the paper's analytic tests, its printed error levels and
convergence orders, exact invariants of the discrete operator, and the Poisson equation
itself in the box interior."""

import json
import math
import os

import numpy as np
import pytest

from oracle import Box, Shear, cell_centres, sasha_phi0, shear_offset, solve

from .exact import (
    cos_gauss_bracket,
    gaussian_1d_closed,
    gaussian_1d_quad,
    paper_norm,
    screened_quad,
    shifted_rel_err,
)

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_accuracy.json")))
FOUR_PI = 4 * math.pi


def column_density(box, profile):
    return np.broadcast_to(profile[None, None, :], (box.nx, box.ny, box.nz)).copy()


# ----------------------------------------------------------------------------------------
# Sect. 3.1: 1-D vertical Gaussian


def test_exact_1d_references_agree_up_to_constant():
    z = np.linspace(-2.9, 2.9, 13)
    for z0 in (0.0, 2.0):
        c = gaussian_1d_closed(z, z0, 6.0)
        q = gaussian_1d_quad(z, z0, 6.0)
        d = c - q
        assert np.ptp(d) < 1e-11  # the closed form equals the convolution plus a constant


@pytest.mark.parametrize("pad,alpha", [(2, 0.0), (4, 1.1)])
def test_1d_gaussian_paper_levels(pad, alpha):
    g_s, g_c = GOLDEN["one_d_shifted"], GOLDEN["one_d_centred"]
    n, L = g_s["n"], g_s["L"]
    box = Box(4, 4, n, L, L, L, pad=pad, alpha=alpha)
    _, _, z = cell_centres(box)
    for z0, g in ((g_s["z0"], g_s), (g_c["z0"], g_c)):
        rho = column_density(box, np.exp(-0.5 * (z - z0) ** 2))
        phi = solve(rho, box, Shear(t=0.37))
        col = phi[1, 2] / FOUR_PI
        ref = gaussian_1d_closed(z, z0, L)
        eps = shifted_rel_err(col, ref)
        if "eps_high" in g:
            assert eps.max() <= g["eps_high"]
            assert np.median(eps) >= 0.1 * g["eps_low"]
        elif alpha == 0.0:
            # alpha = P/2 reproduces the paper's "~1e-7": the printed level is read as within a
            # factor of two either way (measured 1.18e-7), and, as printed, only 4 points come
            # near it (above 0.3x the level); all others agree to better than 4e-8.  The prose
            # places those points near the midplane; here they are the two outermost cells at
            # each end, where the truncated kernel's cut matters most.
            assert 0.5 * g["eps_max"] <= eps.max() <= 2.0 * g["eps_max"]
            assert int((eps > 0.3 * g["eps_max"]).sum()) == g["n_points_near_eps_max"]
        else:
            # the literal alpha = 1.1 with 4x padding is an order of magnitude worse (1.13e-6: its
            # truncated kernel is discontinuous once periodised), which is why alpha = P/2 is the
            # default reading; bounded at 15x the printed level
            assert eps.max() <= 15.0 * g["eps_max"]
        # all columns identical: a z-only density has only the k = 0 mode
        assert np.abs(phi - phi[1:2, 2:3]).max() <= 1e-12 * np.abs(phi).max()


def test_1d_vgf_fixes_the_constant():
    # VGF convolves with exactly |z-z'|/2 on the truncated support: no free constant.
    n, L = 128, 6.0
    box = Box(2, 2, n, L, L, L, pad=2)
    _, _, z = cell_centres(box)
    for z0 in (0.0, 2.0):
        phi = solve(column_density(box, np.exp(-0.5 * (z - z0) ** 2)), box, Shear())[0, 0] / FOUR_PI
        ref = gaussian_1d_quad(z, z0, L)
        assert np.abs(phi - ref).max() <= 5e-5 * np.abs(ref).max()


def test_1d_padding_reading():
    # Padding by 2 with alpha = 1.1 lets periodic images of the kernel overlap the box;
    # alpha = P/2 avoids it.  The paper's 4x padding with alpha = 1.1 is also accurate.
    n, L, z0 = 128, 6.0, 2.0
    errs = {}
    for pad, alpha in ((2, 1.1), (2, 0.0), (4, 1.1)):
        box = Box(2, 2, n, L, L, L, pad=pad, alpha=alpha)
        _, _, z = cell_centres(box)
        phi = solve(column_density(box, np.exp(-0.5 * (z - z0) ** 2)), box, Shear())[0, 0] / FOUR_PI
        ref = gaussian_1d_quad(z, z0, L)
        errs[(pad, alpha)] = np.abs(phi - ref).max() / np.abs(ref).max()
    assert errs[(2, 0.0)] < 1e-4 and errs[(4, 1.1)] < 2e-4
    assert errs[(2, 1.1)] > 1e-2


def test_1d_scale_height_substitution():
    # General H via z/H substitution; checks the oracle's Lz and z0 handling for H != 1.
    n, L, H, z0 = 96, 3.0, 0.4, 0.3
    box = Box(2, 4, n, 1.0, 1.0, L, pad=2)
    _, _, z = cell_centres(box)
    phi = solve(column_density(box, np.exp(-0.5 * ((z - z0) / H) ** 2)), box, Shear())[1, 3] / FOUR_PI
    ref = gaussian_1d_quad(z, z0, L, H)
    assert np.abs(phi - ref).max() <= 1e-4 * np.abs(ref).max()


# ----------------------------------------------------------------------------------------
# Sect. 3.2: 3-D cos x cos x Gaussian, also sheared (Sect. 2.1)


def sheared_cos_case(nx, ny, nz, lx, ly, lz, H, mxk, myk, t, q=1.5, omega=1.0, method="vgf", pad=2, alpha=0.0):
    box = Box(nx, ny, nz, lx, ly, lz, pad=pad, alpha=alpha, method=method)
    s = ((q * omega * lx * t) % ly) / lx  # written out here, independent of the oracle
    x, y, z = cell_centres(box)
    Kx, Ky = 2 * math.pi * mxk / lx, 2 * math.pi * myk / ly
    X, Y, Z = np.meshgrid(x, y, z, indexing="ij")
    # shear-periodic density: a plane wave in the shearing frame y' = y + s x
    rho = np.cos(Kx * X) * np.cos(Ky * (Y + s * X)) * np.exp(-0.5 * (Z / H) ** 2)
    phi = solve(rho, box, Shear(q=q, omega=omega, t=t))
    k1 = math.hypot(Kx + s * Ky, Ky)
    k2 = math.hypot(Kx - s * Ky, Ky)
    b1 = cos_gauss_bracket(z, k1, H, lz)
    b2 = cos_gauss_bracket(z, k2, H, lz)
    ref = FOUR_PI * 0.5 * (
        np.cos((Kx + s * Ky) * X + Ky * Y) * b1[None, None, :] + np.cos((Kx - s * Ky) * X - Ky * Y) * b2[None, None, :]
    )
    return phi, ref, z


def test_closed_form_matches_quadrature():
    z = np.linspace(-2.5, 2.5, 7)
    for k, H in ((1.48, 1.0), (2.2, 0.3)):
        a = cos_gauss_bracket(z, k, H, 6.0)
        b = screened_quad(z, k, H, 6.0)
        assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max()


@pytest.mark.parametrize("H,key", [(1.0, "three_d_H1"), (3.0, "three_d_H3")])
def test_3d_paper_levels(H, key):
    # Sect. 3.2 at the paper's size: 128^3, L = 6, kx = ky = 2 pi/Lx, t = 0.
    g = GOLDEN[key]
    n, L = g["n"], g["L"]
    phi, ref, _ = sheared_cos_case(n, n, n, L, L, L, H, 1, 1, 0.0)
    col = shifted_rel_err(phi[0, 0], ref[0, 0])  # column nearest x = y = 0
    # the paper gives an order of magnitude ("about"); allow a factor 5
    assert col.max() <= 5.0 * g["eps_max"]
    # largest at the vertical boundaries, tiny at the midplane
    assert np.argmax(col) in (0, 1, n - 2, n - 1)
    assert col[n // 2 - 1 : n // 2 + 1].max() <= 1e-3 * col.max() + 1e-15


def test_3d_overall_level():
    n, L = 64, 6.0
    phi, ref, _ = sheared_cos_case(n, n, n, L, L, L, 1.0, 1, 1, 0.0)
    assert np.abs(phi - ref).max() / np.abs(ref).max() <= GOLDEN["three_d_overall"]["eps_max"] * 3


@pytest.mark.parametrize("t", [0.3, 2.9])
def test_sheared_closed_form(t):
    phi, ref, _ = sheared_cos_case(32, 32, 32, 1.0, 1.0, 1.0, 0.1, 1, 1, t)
    assert np.linalg.norm(phi - ref) / np.linalg.norm(ref) < 2e-6


def test_sheared_closed_form_non_cubic():
    # Lx != Ly, Nx != Ny, higher modes: a transposed Lx/Ly or Nx/Ny would fail this.
    phi, ref, _ = sheared_cos_case(24, 48, 32, 2.0, 3.0, 1.5, 0.2, 2, 3, 0.71, q=2.0, omega=0.8)
    assert np.linalg.norm(phi - ref) / np.linalg.norm(ref) < 1e-5


def test_wrong_shear_sign_is_detected():
    # A remap with the opposite sign would produce the potential of the mirrored shear.
    phi, ref, _ = sheared_cos_case(32, 32, 32, 1.0, 1.0, 1.0, 0.1, 1, 1, 0.3)
    phi_m, _, _ = sheared_cos_case(32, 32, 32, 1.0, 1.0, 1.0, 0.1, 1, 1, -0.3)
    assert np.linalg.norm(phi_m - ref) / np.linalg.norm(ref) > 1e-2


def test_sasha_3d_less_accurate_than_vgf():
    g = GOLDEN["sasha_vs_vgf"]
    n, L = 32, 6.0
    errs = {}
    for method in ("vgf", "sasha"):
        phi, ref, _ = sheared_cos_case(n, n, n, L, L, L, 1.0, 1, 1, 0.3, method=method)
        errs[method] = paper_norm(phi, ref)
    ratio = errs["sasha"] / errs["vgf"]
    assert g["ratio_min"] <= ratio <= g["ratio_max"], ratio


# ----------------------------------------------------------------------------------------
# Sect. 3.3: convergence


def _orders(errs):
    return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


def test_convergence_vgf_3d():
    g = GOLDEN["convergence_vgf"]
    L = 6.0
    worst = []
    for H in (1.0, 3.0):
        errs = []
        for n in (16, 32, 64):
            phi, ref, _ = sheared_cos_case(n, n, n, L, L, L, H, 1, 1, 0.0)
            errs.append(paper_norm(phi, ref))
        assert min(_orders(errs)) >= g["order_min"], errs
        worst.append(errs[0])
    assert max(worst) <= 3 * g["n16_worst"]
    assert min(worst) >= 0.1 * g["n16_best"]


@pytest.mark.parametrize("method", ["vgf", "sasha"])
def test_convergence_1d(method):
    L, z0 = 6.0, 2.0
    errs = []
    for n in (16, 32, 64):
        # cubic grids as in the paper: its norm divides by the total cell count N = n^3
        box = Box(n, n, n, L, L, L, pad=2, method=method)
        _, _, z = cell_centres(box)
        phi = solve(column_density(box, np.exp(-0.5 * (z - z0) ** 2)), box, Shear())
        ref = FOUR_PI * gaussian_1d_closed(z, z0, L)
        errs.append(paper_norm(phi, np.broadcast_to(ref, phi.shape)))
    need = GOLDEN["convergence_vgf"]["order_min"] if method == "vgf" else GOLDEN["convergence_sasha"]["order_1d_min"]
    assert min(_orders(errs)) >= need, errs


def test_convergence_sasha_3d():
    L = 6.0
    errs = []
    for n in (16, 32, 64):
        phi, ref, _ = sheared_cos_case(n, n, n, L, L, L, 1.0, 1, 1, 0.0, method="sasha")
        errs.append(paper_norm(phi, ref))
    assert min(_orders(errs)) >= GOLDEN["convergence_sasha"]["order_3d_min"], errs


# ----------------------------------------------------------------------------------------
# SASHA's analytic part (Sect. 2.2)


def test_sasha_phi0_solves_its_equation():
    box = Box(2, 2, 64, 1.0, 1.0, 3.0, pad=2, method="sasha")
    _, _, z = cell_centres(box)
    rng = np.random.default_rng(3)
    rho = np.abs(rng.standard_normal((2, 2, 64))) + 0.1
    p0 = sasha_phi0(rho, box, 0.7)
    dz = z[1] - z[0]
    mean = rho.sum() / (2 * 2 * box.m)
    lap = (p0[2:] - 2 * p0[1:-1] + p0[:-2]) / dz**2  # exact for a parabola
    assert np.allclose(lap, FOUR_PI * 0.7 * mean, rtol=1e-10)
    z0 = (rho.sum(axis=(0, 1)) * z).sum() / rho.sum()
    # vertex at the centre of mass: dPhi0/dz = 4 pi G <rho> (z - z0)
    grad = np.gradient(p0, dz)[1:-1]
    assert np.allclose(grad, FOUR_PI * 0.7 * mean * (z[1:-1] - z0), rtol=1e-9, atol=1e-12)
    assert np.all(sasha_phi0(rho * 0.0, box, 1.0) == 0.0)


def test_sasha_1d_matches_closed_form_up_to_constant():
    n, L, z0 = 128, 6.0, 2.0
    box = Box(2, 2, n, L, L, L, pad=2, method="sasha")
    _, _, z = cell_centres(box)
    phi = solve(column_density(box, np.exp(-0.5 * (z - z0) ** 2)), box, Shear())[0, 0]
    ref = FOUR_PI * gaussian_1d_closed(z, z0, L)
    d = phi - ref
    assert np.ptp(d) <= 1e-4 * np.ptp(ref)  # Sect. 3.1 level, free additive constant
    assert shifted_rel_err(phi, ref).max() <= GOLDEN["one_d_shifted"]["eps_high"]


# ----------------------------------------------------------------------------------------
# Exact invariants of the discrete operator


def _noise_box(method="vgf", shape=(16, 12, 8), pad=2):
    box = Box(*shape, 1.3, 0.9, 0.7, pad=pad, method=method)
    rng = np.random.default_rng(11)
    return box, rng.standard_normal(shape) + 1.0, rng.standard_normal(shape)


@pytest.mark.parametrize("method", ["vgf", "sasha"])
def test_linearity(method):
    box, a, b = _noise_box(method)
    sh = Shear(t=0.41)
    lhs = solve(2.0 * a - 0.5 * b, box, sh)
    rhs = 2.0 * solve(a, box, sh) - 0.5 * solve(b, box, sh)
    if method == "sasha":
        # Phi_0 is not linear in rho (z0 is a ratio); compare the periodic parts
        lhs = lhs - sasha_phi0(2.0 * a - 0.5 * b, box, 1.0)
        rhs = rhs - 2.0 * sasha_phi0(a, box, 1.0) + 0.5 * sasha_phi0(b, box, 1.0)
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


def test_y_shift_commutes():
    box, a, _ = _noise_box()
    sh = Shear(t=0.23)
    assert np.allclose(solve(np.roll(a, 3, axis=1), box, sh), np.roll(solve(a, box, sh), 3, axis=1), atol=1e-12)


def test_z_only_density_is_shear_independent():
    box, a, _ = _noise_box()
    prof = a[0, 0]
    rho = np.broadcast_to(prof, a.shape).copy()
    p1 = solve(rho, box, Shear(t=0.0))
    p2 = solve(rho, box, Shear(q=2.0, omega=3.0, t=0.77))
    assert np.abs(p1 - p2).max() <= 1e-12 * np.abs(p1).max()
    assert np.abs(p1 - p1[:1, :1]).max() <= 1e-12 * np.abs(p1).max()


def test_y_independent_density_is_shear_independent():
    box, a, _ = _noise_box()
    rho = np.broadcast_to(a[:, :1, :], a.shape).copy()
    p1 = solve(rho, box, Shear(t=0.0))
    p2 = solve(rho, box, Shear(t=0.63))
    assert np.abs(p1 - p2).max() <= 1e-12 * np.abs(p1).max()


def test_shear_period_in_time():
    # t and t + Ly/(q Omega Lx) give the same Delta_y0 (Sect. 2.1)
    box, a, _ = _noise_box()
    q, om = 1.5, 1.0
    t0 = 0.2
    t1 = t0 + box.ly / (q * om * box.lx)
    assert shear_offset(q, om, box.lx, box.ly, t0) == pytest.approx(shear_offset(q, om, box.lx, box.ly, t1), abs=1e-14)
    p0 = solve(a, box, Shear(q=q, omega=om, t=t0))
    p1 = solve(a, box, Shear(q=q, omega=om, t=t1))
    assert np.abs(p0 - p1).max() <= 1e-10 * np.abs(p0).max()


def test_shear_offset_wraps_into_box():
    assert shear_offset(1.5, 1.0, 1.0, 1.0, 0.3) == pytest.approx(0.45)
    assert shear_offset(1.5, 1.0, 2.0, 1.0, 0.5) == pytest.approx(0.5)
    d = shear_offset(1.5, 1.0, 1.0, 1.0, -0.3)
    assert 0.0 <= d < 1.0 and d == pytest.approx(0.55)


@pytest.mark.parametrize("method", ["vgf", "sasha"])
def test_z_mirror(method):
    # rho(-z) gives Phi(-z) at t = 0: the kernel is even in z
    box, a, _ = _noise_box(method)
    p = solve(a, box, Shear(t=0.0))
    pm = solve(a[:, :, ::-1], box, Shear(t=0.0))
    assert np.abs(pm[:, :, ::-1] - p).max() <= 1e-11 * np.abs(p).max()


def test_interior_poisson_residual():
    # Spectral horizontal Laplacian in the shearing frame + 4th-order d2/dz2 on interior cells.
    nx = ny = nz = 32
    lx = ly = lz = 1.0
    H, t = 0.1, 0.3
    box = Box(nx, ny, nz, lx, ly, lz)
    s = ((1.5 * 1.0 * lx * t) % ly) / lx
    x, y, z = cell_centres(box)
    X, Y, Z = np.meshgrid(x, y, z, indexing="ij")
    Kx, Ky = 2 * math.pi / lx, 2 * math.pi / ly
    rho = (1.0 + 0.5 * np.cos(Kx * X) * np.cos(Ky * (Y + s * X))) * np.exp(-0.5 * (Z / H) ** 2)
    phi = solve(rho, box, Shear(t=t))
    dz = lz / nz
    # horizontal part: each term is a sheared plane wave, Laplacian = -k^2 * term
    ph_hat_y = np.fft.rfft(phi, axis=1)
    lap = np.zeros_like(phi)
    # k = 0 part (Ky = 0, x-mean) has no horizontal Laplacian; the cos-cos part has Ky = +-2pi
    mean = phi.mean(axis=(0, 1), keepdims=True)
    pert = phi - mean
    k1sq = (Kx + s * Ky) ** 2 + Ky**2
    k2sq = (Kx - s * Ky) ** 2 + Ky**2
    # split pert into its two sheared plane-wave families by projection
    c1 = np.cos((Kx + s * Ky) * X + Ky * Y)
    s1 = np.sin((Kx + s * Ky) * X + Ky * Y)
    c2 = np.cos((Kx - s * Ky) * X - Ky * Y)
    s2 = np.sin((Kx - s * Ky) * X - Ky * Y)
    basis = [c1, s1, c2, s2]
    ksq = [k1sq, k1sq, k2sq, k2sq]
    for b, kk in zip(basis, ksq):
        coef = (pert * b).sum(axis=(0, 1), keepdims=True) / (b * b).sum(axis=(0, 1), keepdims=True)
        lap -= kk * coef * b
    del ph_hat_y
    d2 = (-phi[:, :, 4:] + 16 * phi[:, :, 3:-1] - 30 * phi[:, :, 2:-2] + 16 * phi[:, :, 1:-3] - phi[:, :, :-4]) / (12 * dz * dz)
    res = lap[:, :, 2:-2] + d2 - FOUR_PI * rho[:, :, 2:-2]
    assert np.abs(res).max() <= 5e-3 * np.abs(FOUR_PI * rho).max()
