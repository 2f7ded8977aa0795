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
