"""Parity of the HIP solve (through the C ABI) with the FP64 CPU oracle, element by element
on identical seeded inputs.  Tolerances: relative L2 error <= 1e-12 for FP64 plans and
<= 1e-5 for FP32 plans (inputs rounded to FP32 first; the oracle sees the rounded values)."""

import numpy as np
import pytest

from paper_2510_10070_amd.inputs import gaussian_noise_density, lognormal_density

from .gpu_util import gpu_solve, oracle_solve, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}

# (nx, ny, nz, lx, ly, lz, pad, alpha): spans several tiles of every pass, ragged z chunks
# (nz not a multiple of the tile depth), ragged pencil groups, radix-3 lengths, non-cubic boxes
SHAPES = [
    (8, 8, 4, 1.0, 1.0, 1.0, 2, 0.0),
    (32, 32, 32, 1.0, 1.0, 1.0, 2, 0.0),
    (16, 24, 12, 1.3, 0.9, 0.7, 2, 0.0),
    (48, 64, 24, 2.0, 3.0, 1.5, 2, 0.0),
    (96, 32, 48, 1.0, 1.0, 1.0, 2, 0.0),
    (24, 12, 6, 1.0, 2.0, 1.0, 4, 1.1),
    (64, 128, 96, 1.0, 1.0, 1.0, 2, 0.0),
]


def _box(s, method):
    nx, ny, nz, lx, ly, lz, pad, alpha = s
    return dict(nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz, pad=pad, alpha=alpha, method=method)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("method", ["vgf", "sasha"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s[:3])) + f"_P{s[6]}")
def test_parity_noise(shape, method, precision):
    box = _box(shape, method)
    rho = gaussian_noise_density(shape[:3], shape[5], 0.2 * shape[5], seed=hash(shape) % 1000 + 17)
    shear = (1.5, 1.0, 0.37, 1.0)
    got, used = gpu_solve(box, rho, shear, precision)
    ref = oracle_solve(box, used[0], shear)
    err = rel_l2(got[0], ref)
    print(f"{shape} {method} {precision}: rel-L2 {err:.3e}")
    assert err <= TOL[precision], err


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_parity_config_stratified_32(precision):
    # 32^3, L = 1, H = 0.1, q = 1.5, Omega = 1, t = 0.3, G = 1, noise 0.1
    box = _box((32, 32, 32, 1.0, 1.0, 1.0, 2, 0.0), "vgf")
    rho = gaussian_noise_density((32, 32, 32), 1.0, 0.1, seed=251010071)
    shear = (1.5, 1.0, 0.3, 1.0)
    got, used = gpu_solve(box, rho, shear, precision)
    assert rel_l2(got[0], oracle_solve(box, used[0], shear)) <= TOL[precision]


@pytest.mark.parametrize("t", [0.0, 0.3, 1.9])
def test_parity_shear_times_and_G(t):
    box = _box((32, 16, 16, 1.0, 1.0, 1.0, 2, 0.0), "vgf")
    rho = lognormal_density((32, 16, 16), 1.0, 0.2, seed=5)
    shear = (2.0, 0.7, t, 0.37)
    got, used = gpu_solve(box, rho, shear, "fp64")
    assert rel_l2(got[0], oracle_solve(box, used[0], shear)) <= TOL["fp64"]


@pytest.mark.parametrize("method", ["vgf", "sasha"])
def test_plain_path_parity(method):
    box = _box((32, 24, 16, 1.0, 1.5, 1.0, 2, 0.0), method)
    rho = gaussian_noise_density((32, 24, 16), 1.0, 0.2, seed=9)
    shear = (1.5, 1.0, 0.61, 1.0)
    got, used = gpu_solve(box, rho, shear, "fp64", plain=True)
    assert rel_l2(got[0], oracle_solve(box, used[0], shear)) <= TOL["fp64"]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_multi_box_plan(precision):
    shapes = [(16, 16, 8, 1.0, 1.0, 1.0, 2, 0.0), (32, 8, 12, 2.0, 1.0, 0.5, 2, 0.0), (8, 24, 16, 1.0, 1.0, 1.0, 4, 0.0)]
    methods = ["vgf", "sasha", "vgf"]
    boxes = [_box(s, m) for s, m in zip(shapes, methods)]
    rhos = [lognormal_density(s[:3], s[5], 0.2 * s[5], seed=i + 3) for i, s in enumerate(shapes)]
    shears = [(1.5, 1.0, 0.2 * (i + 1), 1.0 + i) for i in range(3)]
    got, used = gpu_solve(boxes, rhos, shears, precision)
    for b, g, u, s in zip(boxes, got, used, shears):
        assert rel_l2(g, oracle_solve(b, u, s)) <= TOL[precision]


def test_graph_replay_matches_direct_launch():
    import torch

    from paper_2510_10070_amd import Box, Plan, Shear

    shape = (32, 32, 16)
    rho = torch.tensor(lognormal_density(shape, 1.0, 0.2, seed=11), dtype=torch.float32, device="cuda:0")
    direct = Plan(Box(*shape, 1.0, 1.0, 1.0), precision="fp32")
    graph = Plan(Box(*shape, 1.0, 1.0, 1.0), precision="fp32", graph=True)
    out_d = torch.empty_like(rho)
    out_g = torch.empty_like(rho)
    for t in (0.1, 0.5, 0.9, 0.5):  # per-solve parameters change between replays
        direct.solve(rho, out_d, Shear(t=t))
        torch.cuda.synchronize()
        graph.solve(rho, out_g, Shear(t=t))
        torch.cuda.synchronize()
        _ = (out_g * 2).sum().item()  # unrelated eager work between replays
        assert torch.equal(out_d, out_g)
    direct.close()
    graph.close()


def test_caller_workspace_and_determinism():
    import torch

    from paper_2510_10070_amd import Box, Plan, Shear

    shape = (64, 32, 32)
    rho = torch.tensor(lognormal_density(shape, 1.0, 0.2, seed=13), dtype=torch.float64, device="cuda:0")
    plan = Plan(Box(*shape, 1.0, 1.0, 1.0, method="sasha"), precision="fp64")
    ws = torch.empty(plan.workspace_size() // 8 + 64, dtype=torch.float64, device="cuda:0")
    plan.set_workspace(ws)
    a = torch.empty_like(rho)
    b = torch.empty_like(rho)
    plan.solve(rho, a, Shear(t=0.3))
    plan.solve(rho, b, Shear(t=0.3))
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    plan.close()


def test_argument_errors_on_device():
    import torch

    from paper_2510_10070_amd import Box, Plan, SbpError, Shear

    plan = Plan(Box(16, 16, 8, 1.0, 1.0, 1.0), precision="fp32")
    rho = torch.zeros((16, 16, 8), dtype=torch.float32, device="cuda:0")
    with pytest.raises(SbpError) as e:
        plan.solve(rho, rho, Shear())  # phi aliases rho
    assert e.value.status == 1
    small = torch.empty(16, dtype=torch.float32, device="cuda:0")
    with pytest.raises(SbpError) as e:
        plan.set_workspace(small)
    assert e.value.status == 4
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batched_groups_and_autotune(precision, tmp_path, monkeypatch):
    # several boxes share each kernel shape (one launch per group), uneven sizes, per-box shear
    monkeypatch.setenv("SBP_TUNE_CACHE", str(tmp_path / "tune.txt"))
    shapes = [(32, 32, 16), (16, 32, 32), (32, 32, 16), (16, 32, 32), (32, 16, 16), (32, 32, 16)]
    boxes = [_box(s + (1.0, 1.0 + 0.1 * i, 0.8, 2, 0.0), "vgf" if i % 3 else "sasha") for i, s in enumerate(shapes)]
    rhos = [lognormal_density(s, 0.8, 0.2, seed=40 + i) for i, s in enumerate(shapes)]
    shears = [(1.5 if i % 2 else 2.0, 1.0, 0.13 * i, 1.0) for i in range(len(shapes))]
    # the five-pass kernels come in several tile variants (the autotuner times them; the second
    # autotuned plan reads the cache); the fused schedule has one tile shape per length
    for autotune, five in ((False, False), (True, True), (True, True), (True, False)):
        got, used = gpu_solve(boxes, rhos, shears, precision, autotune=autotune,
                               schedule="five_pass" if five else "fused")
        for b, g, u, s in zip(boxes, got, used, shears):
            assert rel_l2(g, oracle_solve(b, u, s)) <= TOL[precision]
    assert (tmp_path / "tune.txt").exists()


def test_graph_replay_with_new_pointers():
    import torch

    from paper_2510_10070_amd import Box, Plan, Shear

    shape = (32, 16, 16)
    plan = Plan(Box(*shape, 1.0, 1.0, 1.0), precision="fp64", graph=True)
    ref_plan = Plan(Box(*shape, 1.0, 1.0, 1.0), precision="fp64")
    for i in range(3):
        rho = torch.tensor(lognormal_density(shape, 1.0, 0.2, seed=60 + i), dtype=torch.float64, device="cuda:0")
        out = torch.empty_like(rho)
        ref = torch.empty_like(rho)
        plan.solve(rho, out, Shear(t=0.2 * i))
        ref_plan.solve(rho, ref, Shear(t=0.2 * i))
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
    plan.close()
    ref_plan.close()


@pytest.mark.parametrize("nbox", [8, 9])
def test_record_delivery_direct(nbox):
    # direct launches: plans of up to 8 boxes pass each solve's records as kernel arguments,
    # larger plans stage them in a pinned ring of 64 slots.  70 solves wrap the ring; each
    # changes every box's shear time and alternates between two output sets, so the last two
    # solves (different records) are both checked against the oracle.
    import torch

    from paper_2510_10070_amd import Box, Plan, Shear

    shapes = [(16, 16, 16) if i % 2 else (32, 16, 16) for i in range(nbox)]
    boxes = [_box(s + (1.0, 1.0 + 0.05 * i, 1.0, 2, 0.0), "sasha" if i % 3 == 2 else "vgf")
             for i, s in enumerate(shapes)]
    rhos = [lognormal_density(s, 0.8, 0.2, seed=90 + i) for i, s in enumerate(shapes)]
    plan = Plan([Box(**b) for b in boxes], precision="fp64")
    r_t = [torch.tensor(r, dtype=torch.float64, device="cuda:0") for r in rhos]
    outs = [[torch.empty_like(r) for r in r_t] for _ in range(2)]
    shear = lambda k, i: (1.5, 1.0, 0.01 * k + 0.1 * i, 1.0 + 0.01 * i)
    nsolve = 70
    for k in range(nsolve):
        plan.solve(r_t, outs[k % 2], [Shear(*shear(k, i)) for i in range(nbox)])
    torch.cuda.synchronize()
    for k in (nsolve - 2, nsolve - 1):
        for i, b in enumerate(boxes):
            got = outs[k % 2][i].cpu().numpy()
            assert rel_l2(got, oracle_solve(b, rhos[i], shear(k, i))) <= TOL["fp64"], (k, i)
    plan.close()


@pytest.mark.parametrize("remap", ["spectral", "linear"])
def test_mixed_nx_launch_groups_fp32(remap):
    # FP32 passes A and C run boxes that differ only in Nx = 16 A (A <= 8) in one launch each,
    # every block taking its box's A and x twiddles from the record: one launch per pass, and
    # every box matches the oracle
    from paper_2510_10070_amd import Box, Plan

    shapes = [(16, 16, 16), (32, 16, 16), (64, 16, 16), (96, 16, 16), (128, 16, 16), (32, 16, 16)]
    boxes = [dict(_box(s + (1.0 + 0.1 * i, 1.0, 1.0, 2, 0.0), "sasha" if i % 2 else "vgf"), remap=remap)
             for i, s in enumerate(shapes)]
    plan = Plan([Box(**b) for b in boxes], precision="fp32", schedule="fused")
    assert plan.describe()["launches"] == 3  # pass A, pass B (one M), pass C
    plan.close()
    rhos = [lognormal_density(s, 1.0, 0.2, seed=120 + i) for i, s in enumerate(shapes)]
    shears = [(1.5, 1.0, 0.2 + 0.1 * i, 1.0) for i in range(len(shapes))]
    got, used = gpu_solve(boxes, rhos, shears, "fp32", schedule="fused")
    for b, g, u, s in zip(boxes, got, used, shears):
        assert rel_l2(g, oracle_solve(b, u, s)) <= TOL["fp32"], b


# shapes inside the fused three-pass domain: x split A = nx/16 in {1, 2, 4, 6, 8, 16}, y up to
# 512, padded z from 32 to 512 and 192, P in {2, 4}; float boxes with nx <= 128 and ny <= 256 take
# 64-byte rows (16 z cells), so nz = 8 leaves a ragged tile
FUSED_SHAPES = [
    (16, 16, 16, 1.0, 1.0, 1.0, 2, 0.0),
    (32, 64, 32, 1.2, 0.8, 1.0, 2, 0.0),
    (64, 32, 48, 1.0, 1.0, 1.0, 2, 0.0),
    (128, 16, 16, 2.0, 1.0, 1.0, 4, 1.5),
    (256, 16, 16, 1.0, 1.0, 1.0, 2, 0.0),
    (16, 512, 16, 1.0, 4.0, 1.0, 2, 0.0),
    (16, 16, 256, 1.0, 1.0, 2.0, 2, 0.0),
    (96, 96, 96, 1.0, 1.5, 1.0, 2, 0.0),  # A = 6, Ny = 96, M = 192
    (96, 16, 32, 1.0, 1.0, 1.0, 2, 0.0),
    (32, 32, 8, 1.0, 1.0, 0.5, 4, 0.0),  # fewer z cells than one 64-byte row: a ragged tile
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("method", ["vgf", "sasha"])
@pytest.mark.parametrize("shape", FUSED_SHAPES, ids=lambda s: "x".join(map(str, s[:3])) + f"_P{s[6]}")
def test_fused_schedule_parity(shape, method, precision):
    box = _box(shape, method)
    rho = lognormal_density(shape[:3], shape[5], 0.2 * shape[5], seed=sum(shape[:3]) + 101)
    shear = (1.5, 1.0, 0.83, 0.7)
    got, used = gpu_solve(box, rho, shear, precision, schedule="fused")
    ref = oracle_solve(box, used[0], shear)
    err = rel_l2(got[0], ref)
    five, _ = gpu_solve(box, used[0], shear, precision, schedule="five_pass")
    err5 = rel_l2(five[0], ref)
    print(f"{shape} {method} {precision}: fused {err:.3e} five-pass {err5:.3e}")
    assert err <= TOL[precision], err
    assert err5 <= TOL[precision], err5


def test_fused_is_selected_and_mixed_schedules():
    from paper_2510_10070_amd import Box, Plan

    for boxes, want in (([Box(32, 32, 32, 1.0, 1.0, 1.0)], "fused-3pass"),
                        ([Box(32, 32, 32, 1.0, 1.0, 1.0), Box(48, 32, 16, 1.0, 1.0, 1.0)], "mixed")):
        plan = Plan(boxes, precision="fp64", schedule="fused")
        d = plan.describe()
        plan.close()
        assert want in str(d), d
    # one plan holding a fused box, a five-pass box and a SASHA fused box
    shapes = [(32, 32, 32), (48, 32, 16), (64, 16, 16)]
    boxes = [_box(s + (1.0, 1.0, 1.0, 2, 0.0), m) for s, m in zip(shapes, ["vgf", "vgf", "sasha"])]
    rhos = [lognormal_density(s, 1.0, 0.2, seed=70 + i) for i, s in enumerate(shapes)]
    shears = [(1.5, 1.0, 0.1 + 0.4 * i, 1.0) for i in range(3)]
    for prec in ("fp64", "fp32"):
        got, used = gpu_solve(boxes, rhos, shears, prec, graph=True, schedule="fused")
        for b, g, u, s in zip(boxes, got, used, shears):
            assert rel_l2(g, oracle_solve(b, u, s)) <= TOL[prec]


# linear-interpolation remap (the real-space variant of Sect. 2.1) in both schedules; the
# shears give fractional and whole-cell row shifts
LINEAR_CASES = [
    ((32, 32, 16, 1.0, 1.0, 1.0, 2, 0.0), (1.5, 1.0, 0.37, 1.0)),
    ((16, 64, 32, 1.0, 4.0, 1.0, 2, 0.0), (2.0, 1.0, 1.0, 0.7)),    # s = 2: whole-cell shifts
    ((48, 24, 12, 2.0, 1.0, 0.8, 2, 0.0), (1.5, 1.0, 0.81, 1.0)),   # five-pass only (nx = 48)
    ((64, 16, 16, 1.0, 2.0, 1.0, 4, 1.5), (1.5, 1.0, 1.3, 1.0)),
]


@pytest.mark.parametrize("schedule", ["fused", "five_pass"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("method", ["vgf", "sasha"])
@pytest.mark.parametrize("case", LINEAR_CASES, ids=lambda c: "x".join(map(str, c[0][:3])) + f"_t{c[1][2]}")
def test_linear_remap_parity(case, method, precision, schedule):
    shape, shear = case
    box = dict(_box(shape, method), remap="linear")
    rho = lognormal_density(shape[:3], shape[5], 0.2 * shape[5], seed=sum(shape[:3]) + 7)
    got, used = gpu_solve(box, rho, shear, precision, schedule=schedule)
    err = rel_l2(got[0], oracle_solve(box, used[0], shear))
    print(f"{shape} linear {method} {precision} {schedule}: rel-L2 {err:.3e}")
    assert err <= TOL[precision], err
