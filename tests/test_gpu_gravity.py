"""Parity of the hydrodynamics outputs (vertical ghost layers, acceleration -grad Phi) with the
oracle, through the C ABI: on the same potential values, and end to end after a solve."""

import numpy as np
import pytest

import oracle
from paper_2510_10070_amd.inputs import lognormal_density

from .gpu_util import gpu_solve, oracle_solve, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _plan(shapes, precision):
    from paper_2510_10070_amd import Box, Plan

    return Plan([Box(*s) for s in shapes], precision=precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("ng", [1, 2, 3])
def test_ghosts_parity(precision, ng):
    import torch

    dt = torch.float64 if precision == "fp64" else torch.float32
    shapes = [(16, 8, 12, 1.0, 1.0, 1.0), (8, 12, 6, 2.0, 1.0, 0.5)]
    plan = _plan(shapes, precision)
    rng = np.random.default_rng(ng)
    phis = [torch.tensor(rng.standard_normal(s[:3]), dtype=dt, device="cuda:0") for s in shapes]
    outs = [torch.empty((s[0], s[1], s[2] + 2 * ng), dtype=dt, device="cuda:0") for s in shapes]
    plan.ghosts(phis, outs, ng)
    torch.cuda.synchronize()
    for p, o in zip(phis, outs):
        ref = oracle.fill_ghosts(p.double().cpu().numpy(), ng)
        assert rel_l2(o.double().cpu().numpy(), ref) <= TOL[precision]
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("t", [0.0, 0.37, 1.2])
def test_gravity_parity_on_same_potential(precision, t):
    import torch

    from paper_2510_10070_amd import Shear

    dt = torch.float64 if precision == "fp64" else torch.float32
    shape = (16, 24, 16, 1.0, 1.5, 1.0)
    plan = _plan([shape], precision)
    rng = np.random.default_rng(11)
    phi64 = rng.standard_normal(shape[:3])
    phi = torch.tensor(phi64, dtype=dt, device="cuda:0")
    g = [torch.empty_like(phi) for _ in range(3)]
    sh = (1.5, 1.0, t, 1.0)
    plan.gravity(phi, *g, Shear(*sh))
    torch.cuda.synchronize()
    box = oracle.Box(*shape)
    ref = oracle.gravity(oracle.fill_ghosts(phi.double().cpu().numpy(), 1), box, oracle.Shear(*sh), 1)
    for got, want in zip(g, ref):
        assert rel_l2(got.double().cpu().numpy(), want) <= TOL[precision]
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("remap", ["spectral", "linear"])
def test_solve_then_gravity_end_to_end(precision, remap):
    import torch

    from paper_2510_10070_amd import Box, Plan, Shear

    shape = (32, 32, 32, 1.0, 1.0, 1.0)
    sh = (1.5, 1.0, 0.61, 1.0)
    box = dict(nx=32, ny=32, nz=32, lx=1.0, ly=1.0, lz=1.0, pad=2, alpha=0.0, method="vgf", remap=remap)
    rho = lognormal_density(shape[:3], 1.0, 0.15, seed=23)
    dt = torch.float64 if precision == "fp64" else torch.float32
    plan = Plan(Box(**box), precision=precision)
    r = torch.tensor(rho, dtype=dt, device="cuda:0")
    phi = torch.empty_like(r)
    g = [torch.empty_like(r) for _ in range(3)]
    plan.solve(r, phi, Shear(*sh))
    plan.gravity(phi, *g, Shear(*sh))
    torch.cuda.synchronize()
    ob = oracle.Box(**box)
    ref_phi = oracle.solve(r.double().cpu().numpy(), ob, oracle.Shear(*sh))
    ref = oracle.gravity(oracle.fill_ghosts(ref_phi, 1), ob, oracle.Shear(*sh), 1)
    # the solve's tolerance carried through a centred difference: an error field of relative
    # size TOL in Phi can grow to TOL |Phi| / (h |g|) in g (h: the spacing of that direction)
    assert rel_l2(phi.double().cpu().numpy(), ref_phi) <= TOL[precision]
    for name, h, got, want in zip("xyz", (1.0 / 32, 1.0 / 32, 1.0 / 32), g, ref):
        amp = max(1.0, np.linalg.norm(ref_phi) / (h * np.linalg.norm(want)))
        err = rel_l2(got.double().cpu().numpy(), want)
        print(f"{precision} {remap} g{name}: rel-L2 {err:.3e} (bound {TOL[precision] * amp:.2e})")
        assert err <= TOL[precision] * amp, (name, err, amp)
    plan.close()
