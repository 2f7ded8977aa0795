"""Helpers for GPU tests: run the HIP solve through the C ABI and compare with the oracle."""

from __future__ import annotations

import numpy as np

import oracle


def rel_l2(a, b) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_solve(box: dict, rhos, shears, precision: str, **plan_kw):
    """box: dict(nx, ny, nz, lx, ly, lz, pad, alpha, method) or a list of them; rhos: float64
    numpy arrays (rounded to the plan precision here); returns float64 numpy results."""
    import torch

    from paper_2510_10070_amd import Box, Plan, Shear

    boxes = box if isinstance(box, list) else [box]
    rhos = rhos if isinstance(rhos, list) else [rhos]
    shears = shears if isinstance(shears, list) else [shears]
    dt = torch.float64 if precision == "fp64" else torch.float32
    plan = Plan([Box(**b) for b in boxes], precision=precision, **plan_kw)
    r_t = [torch.tensor(r, dtype=dt, device="cuda:0") for r in rhos]
    p_t = [torch.empty_like(r) for r in r_t]
    plan.solve(r_t, p_t, [Shear(*s) for s in shears])
    torch.cuda.synchronize()
    out = [p.double().cpu().numpy() for p in p_t]
    used = [r.double().cpu().numpy() for r in r_t]
    plan.close()
    return out, used


def oracle_solve(box: dict, rho, shear):
    b = oracle.Box(**box)
    return oracle.solve(rho, b, oracle.Shear(*shear))


def per_mode_error(got, ref, zchunk: int = 64, floor: float = 1e-2) -> float:
    """Worst horizontal-mode error of a potential, normalised mode by mode.

    Both fields are transformed in x and y (lab frame, per z plane); for every horizontal mode
    (mx, my) the z profile of the difference is compared with that of the reference:
        e(mx, my) = |dPhi_hat(mx, my, :)| / (|Phi_hat_ref(mx, my, :)| + floor * max)
    where max is the largest |Phi_hat_ref(mx, my, :)| over modes.  A global rel-L2 weighs a mode
    by its share of the total norm, and a stratified potential is dominated by its horizontal mean,
    so an error confined to any other mode hides there; here e <= tol holds every mode to tol
    relative to its own amplitude, plus an absolute tol * floor * max.  That floor is set by the
    float arithmetic itself: every transform of a field carries rounding of its largest mode into
    all the others, about 2.4e-8 of max per mode for a float pipeline on the stratified test
    densities, so tol = 1e-5 with floor = 1e-2 (1e-7 of max) leaves a factor of four."""
    nx, ny, nz = ref.shape
    d2 = np.zeros((nx, ny))
    r2 = np.zeros((nx, ny))
    for z0 in range(0, nz, zchunk):
        sl = slice(z0, min(nz, z0 + zchunk))
        r = np.fft.fft2(ref[:, :, sl], axes=(0, 1))
        r2 += (np.abs(r) ** 2).sum(axis=2)
        del r
        d = np.fft.fft2(np.asarray(got[:, :, sl], dtype=np.float64) - ref[:, :, sl], axes=(0, 1))
        d2 += (np.abs(d) ** 2).sum(axis=2)
        del d
    rn = np.sqrt(r2)
    return float((np.sqrt(d2) / (rn + floor * rn.max())).max())


def condition_tolerance(rho, box: dict, shear, precision: str, seed: int = 5) -> float:
    """Relative error a solve in the given precision can be held to on this input.

    Rounding in the forward transforms spreads an error of about eps |rho| over every mode, which
    the Green's function then weighs by its own value there; an input whose potential comes from
    weak (high-|k|) modes alone is therefore ill-conditioned.  kappa = (|Phi(xi)|/|xi|) /
    (|Phi(rho)|/|rho|), with xi white noise, measures that amplification with the oracle.  A float
    pipeline's error measured c * eps * kappa with c <= 6.2 (eps = 2^-24) on the top-mode test
    waves; the bound takes c = 20, and never less than the plain tolerance (1e-5 / 1e-12)."""
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal(np.shape(rho))
    gn = np.linalg.norm(oracle_solve(box, xi, shear)) / np.linalg.norm(xi)
    gs = np.linalg.norm(oracle_solve(box, rho, shear)) / np.linalg.norm(rho)
    eps = 2.0 ** -24 if precision == "fp32" else 2.0 ** -53
    return max(1e-5 if precision == "fp32" else 1e-12, 20.0 * eps * gn / gs)


def max_pointwise_error(got, ref) -> float:
    """max |Phi_gpu - Phi_ref| / max |Phi_ref|."""
    return float(np.abs(np.asarray(got, dtype=np.float64) - ref).max() / np.abs(ref).max())


def seed_tune_cache(path, precision: str, choices) -> None:
    """Write an autotuner cache that makes plans created with autotune=True take the given tile
    variants without measuring: choices = [(kind, len, aux, variant)], kind 5 = fused pass A,
    7 = fused pass C (len = Ny, aux = Nx); 0-4 = the five streaming passes."""
    import torch

    arch = torch.cuda.get_device_properties(0).gcnArchName
    prec = 1 if precision == "fp32" else 0
    with open(path, "w") as f:
        for kind, n, aux, v in choices:
            f.write(f"{arch} {prec} {kind} {n} {aux} {v}\n")
