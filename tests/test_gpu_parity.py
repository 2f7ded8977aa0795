"""Parity of the HIP solve (through the C ABI) with the FP64 CPU oracle, element by element
on identical seeded inputs.  Tolerances: relative L2 error <= 1e-12 for FP64 plans and
<= 1e-5 for FP32 plans (inputs rounded to FP32 first; the oracle sees the rounded values)."""

import numpy as np
import pytest

from paper_2510_10070_amd.inputs import gaussian_noise_density, lognormal_density

from .gpu_util import condition_tolerance, gpu_solve, max_pointwise_error, oracle_solve, per_mode_error, rel_l2

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
    pm, mp = per_mode_error(got[0], ref), max_pointwise_error(got[0], ref)
    print(f"{shape} {method} {precision}: rel-L2 {err:.3e}, per-mode {pm:.3e}, max pointwise {mp:.3e}")
    assert err <= TOL[precision], err
    assert pm <= TOL[precision], pm
    assert mp <= TOL[precision], mp


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


@pytest.mark.parametrize("remap", ["spectral", "linear"])
def test_mixed_ny_launch_groups_fp32(remap):
    # FP32 passes A and C also run boxes of different Ny <= 128 (and A <= 8) in one launch, every
    # block taking its box's Ny, A and twiddles from the record; boxes of Ny = 256 keep their own
    shapes = [(16, 16, 16), (32, 32, 16), (64, 64, 16), (96, 96, 16), (128, 128, 16), (32, 96, 16), (64, 16, 16),
              (128, 32, 16)]
    boxes = [dict(_box(s + (1.0 + 0.1 * i, 1.0 + 0.05 * i, 1.0, 2, 0.0), "sasha" if i % 3 == 1 else "vgf"), remap=remap)
             for i, s in enumerate(shapes)]
    from paper_2510_10070_amd import Box, Plan

    plan = Plan([Box(**b) for b in boxes], precision="fp32", schedule="fused")
    d = plan.describe()
    plan.close()
    assert d["launches"] == 3, d  # pass A, pass B (one M), pass C
    rhos = [lognormal_density(s, 1.0, 0.2, seed=140 + i) for i, s in enumerate(shapes)]
    shears = [(1.5, 1.0, 0.15 + 0.1 * i, 1.0) for i in range(len(shapes))]
    for graph in (False, True):
        got, used = gpu_solve(boxes, rhos, shears, "fp32", schedule="fused", graph=graph)
        for b, g, u, s in zip(boxes, got, used, shears):
            ref = oracle_solve(b, u, s)
            assert rel_l2(g, ref) <= TOL["fp32"], b
            assert per_mode_error(g, ref) <= TOL["fp32"], b


@pytest.mark.parametrize("remap", ["spectral", "linear"])
def test_mixed_ny_wide_rows_fp32(remap):
    # in a launch that mixes Ny, boxes of Ny <= 64 or A <= 4 take 128-byte rows (32 z cells per
    # tile), the others 64-byte rows: z lengths that fill one tile, several tiles, and ragged last
    # tiles (nz = 8, 48, 96), with the SASHA partial sums of the wider tiles and P = 4 boxes
    shapes = [(64, 64, 48, 4), (32, 32, 8, 4), (128, 16, 96, 2), (16, 64, 128, 2), (96, 128, 32, 2),
              (64, 96, 64, 2), (32, 32, 32, 2), (128, 64, 16, 2), (64, 128, 48, 4), (32, 96, 96, 2),
              (128, 128, 64, 2)]
    boxes = [dict(_box((nx, ny, nz, 1.0 + 0.1 * i, 0.9 + 0.05 * i, 1.0, pad, 0.0),
                       "sasha" if i % 2 else "vgf"), remap=remap)
             for i, (nx, ny, nz, pad) in enumerate(shapes)]
    from paper_2510_10070_amd import Box, Plan

    plan = Plan([Box(**b) for b in boxes], precision="fp32", schedule="fused")
    d = plan.describe()
    plan.close()
    assert d["path"] == "fused-3pass", d
    assert sorted((g["pass"], g["len"]) for g in d["groups"] if g["pass"] != "fused_b") == \
        [("fused_a", 0), ("fused_c", 0)], d  # passes A and C: one launch each
    rhos = [lognormal_density(s[:3], 1.0, 0.2, seed=180 + i) for i, s in enumerate(shapes)]
    shears = [(1.5, 1.0, 0.35 + 0.1 * i, 1.0) for i in range(len(shapes))]
    for graph in (False, True):
        got, used = gpu_solve(boxes, rhos, shears, "fp32", schedule="fused", graph=graph)
        for b, g, u, s in zip(boxes, got, used, shears):
            ref = oracle_solve(b, u, s)
            err, pm = rel_l2(g, ref), per_mode_error(g, ref)
            print(f"{b['nx']}x{b['ny']}x{b['nz']} P{b['pad']} {b['method']} graph={graph}: {err:.2e} {pm:.2e}")
            assert err <= TOL["fp32"], b
            assert pm <= TOL["fp32"], b


@pytest.mark.parametrize("remap", ["spectral", "linear"])
def test_mixed_m_launch_groups_fp32(remap):
    # FP32 pass B runs boxes of different padded length M <= 256 (padding 2) in one launch, every
    # block taking its box's M and z twiddles from the record; where an item needs fewer than four
    # wavefronts (M <= 128) a block holds several items of its box, the k = 0 item among them in
    # the box's first block.  A box with padding 4 keeps a launch of its own.
    shapes = [(16, 16, 16, 2), (32, 32, 32, 2), (64, 16, 64, 2), (32, 96, 96, 2), (16, 32, 128, 2),
              (128, 128, 64, 2), (256, 16, 16, 2), (32, 16, 32, 4), (96, 32, 32, 2)]
    boxes = [dict(_box((nx, ny, nz, 1.0 + 0.1 * i, 1.0 + 0.05 * i, 0.8 + 0.1 * i, pad, 0.0),
                       "sasha" if i % 3 == 1 else "vgf"), remap=remap)
             for i, (nx, ny, nz, pad) in enumerate(shapes)]
    from paper_2510_10070_amd import Box, Plan

    plan = Plan([Box(**b) for b in boxes], precision="fp32", schedule="fused")
    d = plan.describe()
    plan.close()
    assert d["path"] == "fused-3pass", d
    fb = sorted((g["len"], g["boxes"]) for g in d["groups"] if g["pass"] == "fused_b")
    assert fb == [(0, 8), (128, 1)], d  # one launch for every M of padding 2, one for the P = 4 box
    rhos = [lognormal_density(s[:3], 1.0, 0.2, seed=160 + i) for i, s in enumerate(shapes)]
    shears = [(1.5, 1.0, 0.25 + 0.1 * i, 1.0) for i in range(len(shapes))]
    for graph in (False, True):
        got, used = gpu_solve(boxes, rhos, shears, "fp32", schedule="fused", graph=graph)
        for b, g, u, s in zip(boxes, got, used, shears):
            ref = oracle_solve(b, u, s)
            err, pm = rel_l2(g, ref), per_mode_error(g, ref)
            print(f"{b['nx']}x{b['ny']}x{b['nz']} P{b['pad']} {b['method']} graph={graph}: {err:.2e} {pm:.2e}")
            assert err <= TOL["fp32"], b
            assert pm <= TOL["fp32"], b


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
    # 4x padding in pass B: M = 128, 192, 256, 512 (tile layouts and k = 0 staging of Q = 4)
    (16, 16, 32, 1.0, 1.0, 1.0, 4, 0.0),
    (32, 16, 48, 1.0, 1.0, 1.0, 4, 1.3),
    (16, 32, 64, 1.0, 1.0, 1.0, 4, 0.0),
    (16, 16, 128, 1.0, 1.0, 1.0, 4, 0.0),
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
    pm, pm5 = per_mode_error(got[0], ref), per_mode_error(five[0], ref)
    print(f"{shape} {method} {precision}: fused {err:.3e} (per-mode {pm:.3e}) five-pass {err5:.3e} "
          f"(per-mode {pm5:.3e})")
    assert err <= TOL[precision], err
    assert err5 <= TOL[precision], err5
    assert pm <= TOL[precision], pm
    assert pm5 <= TOL[precision], pm5
    assert max_pointwise_error(got[0], ref) <= TOL[precision]
    assert max_pointwise_error(five[0], ref) <= TOL[precision]


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


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_ring_wraps_with_changing_shear(precision):
    # a graph plan reads each solve's records from a pinned ring of 64 slots through a device-side
    # counter that the replayed fetch kernel advances.  70 replays without synchronisation wrap the
    # ring; the shear time changes every replay and the outputs alternate, so the last two replays
    # (different records, different slots) are both checked against the oracle.
    import torch

    from paper_2510_10070_amd import Box, Plan, Shear

    shape = (32, 16, 16)
    box = _box(shape + (1.0, 1.0, 1.0, 2, 0.0), "sasha")
    rho = lognormal_density(shape, 1.0, 0.2, seed=301)
    dt = torch.float64 if precision == "fp64" else torch.float32
    r = torch.tensor(rho, dtype=dt, device="cuda:0")
    outs = [torch.empty_like(r) for _ in range(2)]
    plan = Plan(Box(**box), precision=precision, graph=True)
    shear = lambda k: (1.5, 1.0, 0.013 * k, 1.0 + 0.002 * k)
    nsolve = 70
    for k in range(nsolve):
        plan.solve(r, outs[k % 2], Shear(*shear(k)))
    torch.cuda.synchronize()
    used = r.double().cpu().numpy()
    for k in (nsolve - 2, nsolve - 1):
        err = rel_l2(outs[k % 2].double().cpu().numpy(), oracle_solve(box, used, shear(k)))
        assert err <= TOL[precision], (k, err)
    # and again, past a second wrap, after synchronising in between
    for k in range(nsolve, 2 * nsolve):
        plan.solve(r, outs[k % 2], Shear(*shear(k)))
    torch.cuda.synchronize()
    k = 2 * nsolve - 1
    assert rel_l2(outs[k % 2].double().cpu().numpy(), oracle_solve(box, used, shear(k))) <= TOL[precision]
    plan.close()


@pytest.mark.parametrize("schedule", ["fused", "five_pass", "plain"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sasha_zero_total_mass(schedule, precision):
    # SASHA takes z0 = sum(z rho)/sum(rho); with sum(rho) = 0 the analytic part is dropped
    # (Phi_0 = 0).  rho = 0 must give Phi = 0 exactly; a zero-mean density must match the oracle,
    # which takes the same branch.
    if schedule == "plain" and precision == "fp32":
        pytest.skip("the plain path is FP64 only")
    shape = (32, 16, 16)
    box = _box(shape + (1.0, 1.0, 1.0, 2, 0.0), "sasha")
    kw = dict(plain=True) if schedule == "plain" else dict(schedule=schedule)
    shear = (1.5, 1.0, 0.4, 1.0)
    zero = np.zeros(shape)
    got, _ = gpu_solve(box, zero, shear, precision, **kw)
    assert np.all(got[0] == 0.0)
    # a zero-mean density of small integers: every partial sum is exact in any order and
    # precision, so both sides see sum(rho) = 0 exactly
    sign = np.where(np.arange(32) % 2 == 0, 1.0, -1.0)[:, None, None]
    rho = sign * (1.0 + (np.arange(16) % 3)[None, :, None] + (np.arange(16) % 2)[None, None, :])
    assert rho.sum() == 0.0
    got, used = gpu_solve(box, rho, shear, precision, **kw)
    ref = oracle_solve(box, used[0], shear)
    assert rel_l2(got[0], ref) <= TOL[precision]


# FP32 checks that an error confined to a few high-|k| modes cannot hide under rel-L2: per-mode
# comparison on a random field, and densities that excite only the top horizontal modes
@pytest.mark.parametrize("schedule", ["fused", "five_pass"])
def test_fp32_per_mode_and_pointwise(schedule):
    from paper_2510_10070_amd.inputs import grf_density

    shape = (64, 64, 32)
    box = _box(shape + (2.0, 2.0, 3.0, 2, 0.0), "vgf")
    rho = grf_density(shape, (2.0, 2.0, 3.0), 0.5, seed=401)
    shear = (1.5, 1.0, 0.3, 1.0)
    got, used = gpu_solve(box, rho, shear, "fp32", schedule=schedule)
    ref = oracle_solve(box, used[0], shear)
    pm, mp = per_mode_error(got[0], ref), max_pointwise_error(got[0], ref)
    print(f"grf 64x64x32 fp32 {schedule}: per-mode {pm:.3e}, max pointwise {mp:.3e}, rel-L2 {rel_l2(got[0], ref):.3e}")
    assert pm <= TOL["fp32"], pm
    assert mp <= TOL["fp32"], mp


def _top_mode_wave(shape, lengths, s, mx, my):
    """cos(Kx x) cos(Ky (y + s x)) exp(-z^2/2 H^2) at mode numbers (mx, my): shear-periodic."""
    nx, ny, nz = shape
    lx, ly, lz = lengths
    x = (np.arange(nx) + 0.5) * lx / nx
    y = (np.arange(ny) + 0.5) * ly / ny
    z = -0.5 * lz + (np.arange(nz) + 0.5) * lz / nz
    X, Y = np.meshgrid(x, y, indexing="ij")
    h = np.cos(2 * np.pi * mx * X / lx) * np.cos(2 * np.pi * my * (Y + s * X) / ly)
    return h[:, :, None] * np.exp(-0.5 * (z / (0.2 * lz)) ** 2)[None, None, :]


@pytest.mark.parametrize("schedule", ["fused", "five_pass"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("shape", [(64, 64, 32), (256, 32, 16), (96, 96, 24)], ids=lambda s: "x".join(map(str, s)))
def test_top_horizontal_modes(shape, precision, schedule):
    # waves at the largest mode numbers in x and y (and their mix), so the whole result lives in the
    # high-|k| pencils that a wrong twiddle, tile row or padding slot there would corrupt.  Such an
    # input is ill-conditioned for any solve in float (rounding in the other modes is weighed by
    # their far larger Green's function): the bound is the FP32 tolerance or 20 eps kappa, whichever
    # is larger (condition_tolerance), at most 5e-4 here, far below the O(1) error of such a bug.
    lengths = (1.0, 1.0, 1.0)
    q, om, t, G = 1.5, 1.0, 0.5, 1.0  # s = 0.75
    s = (q * om * lengths[0] * t) % lengths[1] / lengths[0]
    nx, ny, _ = shape
    box = _box(shape + lengths + (2, 0.0), "vgf")
    for mx, my in ((nx // 2 - 1, 1), (1, ny // 2 - 1), (nx // 2 - 1, ny // 2 - 1), (nx // 3, ny // 2 - 2)):
        rho = _top_mode_wave(shape, lengths, s, mx, my)
        got, used = gpu_solve(box, rho, (q, om, t, G), precision, schedule=schedule)
        ref = oracle_solve(box, used[0], (q, om, t, G))
        tol = condition_tolerance(used[0], box, (q, om, t, G), precision)
        assert tol <= (5e-4 if precision == "fp32" else 1e-11)
        err, mp = rel_l2(got[0], ref), max_pointwise_error(got[0], ref)
        print(f"{shape} mode ({mx},{my}) {precision} {schedule}: rel-L2 {err:.3e}, max pointwise {mp:.3e}, "
              f"bound {tol:.2e}")
        assert err <= tol, (mx, my, err)
        assert mp <= 2 * tol, (mx, my, mp)


def test_max_box_count():
    # the largest plan the ABI accepts: 4096 boxes (tiny, of three shapes, both methods, per-box
    # shear), one FP32 solve, each box against the oracle
    shapes = [(8, 8, 4), (16, 8, 4), (8, 16, 8)]
    boxes, rhos, shears = [], [], []
    for i in range(4096):
        s = shapes[i % 3]
        boxes.append(_box(s + (1.0, 1.0 + 0.01 * (i % 7), 1.0, 2, 0.0), "sasha" if i % 5 == 0 else "vgf"))
        rhos.append(lognormal_density(s, 1.0, 0.2, seed=1000 + i))
        shears.append((1.5, 1.0, 0.001 * i, 1.0))
    got, used = gpu_solve(boxes, rhos, shears, "fp32")
    worst = 0.0
    for b, g, u, s in zip(boxes, got, used, shears):
        worst = max(worst, rel_l2(g, oracle_solve(b, u, s)))
    print(f"4096 boxes fp32: worst rel-L2 {worst:.3e}")
    assert worst <= TOL["fp32"], worst


@pytest.mark.parametrize("shape,pad", [((128, 16, 16), 4), ((128, 32, 32), 2), ((128, 64, 64), 2)],
                         ids=["128x16x16_P4", "128x32x32_P2", "128x64x64_P2"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_repeated_solves_are_bitwise_identical(shape, pad, precision):
    # the same solve repeated gives the same bits: boxes whose pass-A y transforms are each owned by
    # one wavefront (A = 8 planes side by side: 64-byte rows in float, the split kernel in double;
    # with Ny = 16 the y twiddle table of a block comes from its first wavefront alone), launched
    # directly and back to back
    import torch

    from paper_2510_10070_amd import Box, Plan, Shear

    dt = torch.float32 if precision == "fp32" else torch.float64
    rho = torch.tensor(lognormal_density(shape, 1.0, 0.3, seed=sum(shape) + pad), dtype=dt, device="cuda:0")
    plan = Plan(Box(*shape, 1.2, 0.9, 1.0, pad=pad), precision=precision, schedule="fused")
    outs = [torch.empty_like(rho) for _ in range(48)]
    for o in outs:
        plan.solve(rho, o, Shear(t=0.41))
    torch.cuda.synchronize()
    for k, o in enumerate(outs[1:], 1):
        assert torch.equal(o, outs[0]), k
    plan.close()
