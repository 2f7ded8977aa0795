"""sbp_solve_static, the entry point that allocates nothing, against sbp_solve.

Both run the same kernels; only the workspace differs (the library's fixed per-device array
instead of the plan's own), so their results must agree bit for bit, and both must match the
oracle.  Two calls in a row, the second on a smaller plan, so that the second reads an array the
first left dirty.  Also the size and state errors it documents."""

import numpy as np
import pytest

from paper_2510_10070_amd.inputs import lognormal_density

from .gpu_util import oracle_solve, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _run(box, precision, seed, method="vgf", graph=False):
    import torch

    from paper_2510_10070_amd import Box, Plan, Shear

    nx, ny, nz = box[:3]
    dt = torch.float32 if precision == "fp32" else torch.float64
    rho64 = lognormal_density((nx, ny, nz), box[5], 0.2 * box[5], seed=seed)
    rho = torch.tensor(rho64, dtype=dt, device="cuda:0")
    plan = Plan(Box(*box, method=method), precision=precision, graph=graph)
    shear = Shear(1.5, 1.0, 0.37, 1.0)
    ref_out = torch.empty_like(rho)
    if graph:
        plan.solve(rho, ref_out, shear)  # a graph plan captures its graph on its first sbp_solve
    out = torch.full_like(rho, float("nan"))
    plan.solve_static(rho, out, shear)
    plan.solve(rho, ref_out, shear)
    torch.cuda.synchronize()
    plan.close()
    return out, ref_out, rho.double().cpu().numpy(), (1.5, 1.0, 0.37, 1.0)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_static_matches_solve_then_smaller(precision):
    import torch

    cases = [((128, 128, 64, 1.0, 1.0, 1.0), "vgf", False), ((32, 16, 16, 1.0, 2.0, 1.0), "sasha", False),
             ((48, 24, 12, 1.0, 1.0, 0.5), "vgf", True)]  # fused, then smaller fused, then five-pass graph
    for i, (box, method, graph) in enumerate(cases):
        out, ref_out, used, shear = _run(box, precision, seed=700 + i, method=method, graph=graph)
        assert torch.equal(out, ref_out), (box, precision)
        b = dict(nx=box[0], ny=box[1], nz=box[2], lx=box[3], ly=box[4], lz=box[5], pad=2, alpha=0.0, method=method)
        err = rel_l2(out.double().cpu().numpy(), oracle_solve(b, used, shear))
        assert err <= TOL[precision], (box, err)


def test_static_errors():
    import torch

    from paper_2510_10070_amd import Box, Plan, SbpError, Shear
    from paper_2510_10070_amd._lib import SBP_STATIC_WORKSPACE_BYTES

    big = Plan(Box(512, 256, 512, 1.0, 1.0, 1.0), precision="fp32")  # 256 MiB of workspace
    assert big.workspace_size() > SBP_STATIC_WORKSPACE_BYTES
    rho = torch.zeros((512, 256, 512), dtype=torch.float32, device="cuda:0")
    with pytest.raises(SbpError) as e:
        big.solve_static(rho, torch.empty_like(rho), Shear())
    assert e.value.status == 2  # SBP_E_SIZE
    big.close()
    del rho
    g = Plan(Box(16, 16, 16, 1.0, 1.0, 1.0), precision="fp32", graph=True)
    r = torch.zeros((16, 16, 16), dtype=torch.float32, device="cuda:0")
    with pytest.raises(SbpError) as e:
        g.solve_static(r, torch.empty_like(r), Shear())
    assert e.value.status == 6  # SBP_E_STATE: graph not captured yet
    g.close()
