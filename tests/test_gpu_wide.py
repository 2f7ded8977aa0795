"""The wide fused schedule against the FP64 oracle and the five-pass schedule.

Float boxes with Nx in {512, 1024}, Ny in {512, 1024}, padding 2 and M <= 512 run fused on
request (schedule "fused"), with B = 64 pencils per pass-B item (A = Nx/64 planes per pass-A
block); by default they run five-pass, the faster on gfx950.  Every kernel shape the wide
schedule instantiates appears below: Ny = 512 and 1024, A = 8 and 16 (16-byte rows, and 8-byte
rows at Ny = 1024 with A = 16), M = 64 to 512, VGF and SASHA, spectral and linear remap, direct
launches and graph replay; then a plan that mixes a wide box with narrow fused and five-pass
boxes, and two full-size boxes (the 1024 x 1024 x 256 clumpy box among them) against the five-pass
solve."""

import numpy as np
import pytest

from paper_2510_10070_amd.inputs import lognormal_density, workload

from .gpu_util import gpu_solve, max_pointwise_error, oracle_solve, per_mode_error, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5

# (nx, ny, nz): the kernel shapes each covers
CASES = [
    (512, 512, 32),    # A 8, Ny 512, M 64
    (1024, 512, 64),   # A 16, Ny 512, M 128
    (512, 1024, 32),   # A 8, Ny 1024: two positions per lane pair, M 64
    (1024, 1024, 32),  # A 16, Ny 1024: 8-byte rows, M 64
    (512, 512, 128),   # M 256
    (512, 512, 256),   # M 512 (the 144 KB pass-B tile)
]


def _box(shape, method, remap, i):
    nx, ny, nz = shape
    return dict(nx=nx, ny=ny, nz=nz, lx=1.0 + 0.25 * i, ly=0.9 + 0.1 * i, lz=0.8 + 0.1 * i, pad=2, alpha=0.0,
                method=method, remap=remap)


def _ids(c):
    return "x".join(map(str, c))


@pytest.mark.parametrize("method", ["vgf", "sasha"])
@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_wide_against_oracle(case, method):
    from paper_2510_10070_amd import Box, Plan

    i = CASES.index(case)
    remap = "linear" if i % 2 else "spectral"
    box = _box(case, method, remap, i)
    plan = Plan([Box(**box)], precision="fp32", schedule="fused")
    d = plan.describe()
    plan.close()
    assert d["path"] == "fused-3pass", d
    assert all(g["variant"] == 4 for g in d["groups"]), d  # the wide kernels in all three passes
    plan = Plan([Box(**box)], precision="fp32")
    assert plan.describe()["path"] == "streaming-5pass"  # the default schedule for wide boxes
    plan.close()
    rho = lognormal_density(case, 1.0, 0.25, seed=300 + 7 * i + (method == "sasha"))
    shear = (1.5, 1.0, 0.37 + 0.1 * i, 1.0)
    graph = i % 3 == 2
    got, used = gpu_solve(box, rho, shear, "fp32", schedule="fused", graph=graph)
    ref = oracle_solve(box, used[0], shear)
    err, mp, pm = rel_l2(got[0], ref), max_pointwise_error(got[0], ref), per_mode_error(got[0], ref)
    five, _ = gpu_solve(box, used[0], shear, "fp32", schedule="five_pass")
    err5 = rel_l2(five[0], ref)
    print(f"{case} {method} {remap} graph={graph}: rel-L2 {err:.3e}, max pointwise {mp:.3e}, per-mode {pm:.3e}; "
          f"five-pass {err5:.3e}")
    assert np.isfinite(got[0]).all()
    assert err <= TOL and mp <= TOL and pm <= TOL, (err, mp, pm)
    assert rel_l2(got[0], five[0]) <= 2 * TOL


def test_wide_in_a_mixed_plan():
    # a wide box, a narrow fused box and a five-pass box (nx = 48) in one plan: the wide box's
    # passes run launches of their own, next to the narrow ones, in every phase
    from paper_2510_10070_amd import Box, Plan

    shapes = [(512, 1024, 64), (256, 64, 32), (48, 24, 12), (1024, 512, 32)]
    boxes = [dict(_box(s, "sasha" if k % 2 else "vgf", "linear" if k == 3 else "spectral", k)) for k, s in
             enumerate(shapes)]
    plan = Plan([Box(**b) for b in boxes], precision="fp32", schedule="fused")
    d = plan.describe()
    plan.close()
    assert d["path"] == "mixed", d
    wide = sorted((g["pass"], g["len"], g["boxes"]) for g in d["groups"] if g["variant"] == 4)
    assert wide == [("fused_a", 512, 1), ("fused_a", 1024, 1), ("fused_b", 64, 1), ("fused_b", 128, 1),
                    ("fused_c", 512, 1), ("fused_c", 1024, 1)], d
    # the autotuner times the narrow box's tile variants and leaves the wide box's kernels alone
    plan = Plan([Box(**b) for b in boxes], precision="fp32", schedule="fused", autotune=True)
    dt = plan.describe()
    plan.close()
    assert dt["tuning"] in ("measured", "cache"), dt
    assert sorted((g["pass"], g["len"], g["boxes"]) for g in dt["groups"] if g["variant"] == 4) == wide, dt
    rhos = [lognormal_density(s, 1.0, 0.2, seed=330 + k) for k, s in enumerate(shapes)]
    shears = [(1.5, 1.0, 0.2 + 0.15 * k, 1.0) for k in range(len(shapes))]
    for graph, tuned in ((False, False), (True, False), (False, True)):
        got, used = gpu_solve(boxes, rhos, shears, "fp32", schedule="fused", graph=graph, autotune=tuned)
        for b, g, u, s in zip(boxes, got, used, shears):
            ref = oracle_solve(b, u, s)
            err, pm = rel_l2(g, ref), per_mode_error(g, ref)
            print(f"{b['nx']}x{b['ny']}x{b['nz']} {b['method']} graph={graph} tuned={tuned}: {err:.2e} {pm:.2e}")
            assert err <= TOL and pm <= TOL, b


@pytest.mark.timeout(300)
@pytest.mark.parametrize("shape", [(1024, 1024, 256), (512, 1024, 256)], ids=["clumpy1024", "lognormal512x1024"])
def test_wide_full_size_against_five_pass(shape):
    # full-size boxes fused on request, element by element against the five-pass solve of the same
    # input: the 1024 x 1024 x 256 clumpy box (A = 16, Ny = 1024, 8-byte rows, M = 512; the
    # full-size tests hold its five-pass solve to the oracle cell by cell) and a 512 x 1024 x 256
    # log-normal box (A = 8, 16-byte rows)
    import torch

    from paper_2510_10070_amd import Box, Plan, Shear

    if shape == (1024, 1024, 256):
        w = workload("clumpy-1024")
        b, shear, rho = w["box"], w["shear"], w["make"]()
    else:
        b, shear = shape + (8.0, 16.0, 4.0), (1.5, 1.0, 2.5, 1.0)
        rho = lognormal_density(shape, 4.0, 1.0, seed=350)
    rho = torch.tensor(rho, dtype=torch.float32, device="cuda:0")
    out = {}
    for sched in ("fused", "five_pass"):
        plan = Plan(Box(*b), precision="fp32", schedule=sched)
        phi = torch.empty_like(rho)
        plan.solve(rho, phi, Shear(*shear))
        torch.cuda.synchronize()
        out[sched] = (plan.describe()["path"], phi.double().cpu().numpy())
        plan.close()
        del phi
    assert out["fused"][0] == "fused-3pass" and out["five_pass"][0] == "streaming-5pass"
    got, ref = out["fused"][1], out["five_pass"][1]
    err, mp, pm = rel_l2(got, ref), max_pointwise_error(got, ref), per_mode_error(got, ref, zchunk=32)
    print(f"{shape} fp32 fused vs five-pass: rel-L2 {err:.3e}, max pointwise {mp:.3e}, per-mode {pm:.3e}")
    assert np.isfinite(got).all()
    assert err <= 2 * TOL and mp <= 2 * TOL and pm <= 2 * TOL, (err, mp, pm)


@pytest.mark.parametrize("precision,shape,pad", [("fp64", (512, 512, 32), 2), ("fp32", (512, 512, 32), 4),
                                                 ("fp32", (512, 256, 32), 2), ("fp32", (1024, 512, 512), 2)],
                         ids=["fp64", "pad4", "ny256", "m1024"])
def test_wide_request_outside_its_domain_runs_five_pass(precision, shape, pad):
    # the fused request covers the wide boxes in FP32 with padding 2, Ny in {512, 1024} and
    # M <= 512 only; any other box of that width runs five-pass under the same flag
    from paper_2510_10070_amd import Box, Plan

    box = dict(_box(shape, "vgf", "spectral", 1), pad=pad)
    plan = Plan([Box(**box)], precision=precision, schedule="fused")
    d = plan.describe()
    plan.close()
    assert d["path"] == "streaming-5pass", d
    if shape[2] <= 32:  # small enough for the oracle here
        rho = lognormal_density(shape, 1.0, 0.25, seed=360 + pad)
        shear = (1.5, 1.0, 0.61, 1.0)
        got, used = gpu_solve(box, rho, shear, precision, schedule="fused")
        ref = oracle_solve(box, used[0], shear)
        tol = 1e-12 if precision == "fp64" else TOL
        assert rel_l2(got[0], ref) <= tol and max_pointwise_error(got[0], ref) <= tol
