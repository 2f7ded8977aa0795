"""A seeded sweep over the plan space against the FP64 oracle.

Each case draws a box (every axis from the lengths the ABI accepts, kept small enough for the
oracle), the padding and truncation, the method, the remap, the precision, the shear parameters
and the launch mode (direct or graph-replayed, fused or five-pass by default); a few cases hold
several boxes at once, a second draw holds only plans of 2 to 8 boxes, and a third wide FP32 boxes
(Nx, Ny in {512, 1024}) fused on request, alone or beside a box of the first draw.  The draws are fixed
(seeds below), so a failure names a reproducible case."""

import numpy as np
import pytest

from paper_2510_10070_amd.inputs import lognormal_density

from .gpu_util import gpu_solve, max_pointwise_error, oracle_solve, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}
LENS = [8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256]
SEED = 20260


def _draw_box(rng):
    while True:
        nx, ny = int(rng.choice(LENS)), int(rng.choice(LENS))
        pad = int(rng.choice([2, 2, 4]))
        m = int(rng.choice([l for l in LENS + [384, 512] if l % pad == 0 and l // pad >= 4 and (l // pad) % 2 == 0]))
        nz = m // pad
        if nx * ny * nz <= 1 << 19:
            break
    alpha = 0.0 if pad == 2 or rng.random() < 0.5 else float(rng.uniform(1.0, 2.0))
    return dict(nx=nx, ny=ny, nz=nz, lx=float(rng.uniform(0.5, 3.0)), ly=float(rng.uniform(0.5, 3.0)),
                lz=float(rng.uniform(0.5, 2.0)), pad=pad, alpha=alpha, method=str(rng.choice(["vgf", "sasha"])),
                remap=str(rng.choice(["spectral", "spectral", "linear"])))


def _cases():
    rng = np.random.default_rng(SEED)
    out = []
    for i in range(150):
        nbox = 1 if i < 120 else int(rng.integers(2, 6))
        boxes = [_draw_box(rng) for _ in range(nbox)]
        shears = [(float(rng.choice([1.5, 2.0])), float(rng.uniform(0.5, 1.5)), float(rng.uniform(0.0, 3.0)),
                   float(rng.uniform(0.2, 2.0))) for _ in range(nbox)]
        out.append(dict(boxes=boxes, shears=shears, precision=str(rng.choice(["fp32", "fp64"])),
                        graph=bool(rng.random() < 0.3), schedule=str(rng.choice(["auto", "auto", "five_pass"])),
                        seed=int(rng.integers(0, 2**31))))
    return out


CASES = _cases()


@pytest.mark.parametrize("case", CASES, ids=[f"case{i}" for i in range(len(CASES))])
def test_random_plan(case):
    boxes, shears = case["boxes"], case["shears"]
    rhos = [lognormal_density((b["nx"], b["ny"], b["nz"]), b["lz"], 0.25 * b["lz"], seed=case["seed"] + k)
            for k, b in enumerate(boxes)]
    got, used = gpu_solve(boxes, rhos, shears, case["precision"], graph=case["graph"], schedule=case["schedule"])
    for b, g, u, s in zip(boxes, got, used, shears):
        ref = oracle_solve(b, u, s)
        err, mp = rel_l2(g, ref), max_pointwise_error(g, ref)
        assert err <= TOL[case["precision"]], (b, s, case["precision"], err)
        assert mp <= TOL[case["precision"]], (b, s, case["precision"], mp)


def _batch_cases():
    # plans of 2 to 8 boxes, mostly float, so that launches mix Nx, Ny and M (the multi-box
    # kernels, their wide rows and their items per block) across many shapes
    rng = np.random.default_rng(SEED + 1)
    out = []
    for _ in range(60):
        nbox = int(rng.integers(2, 9))
        boxes = [_draw_box(rng) for _ in range(nbox)]
        shears = [(float(rng.choice([1.5, 2.0])), float(rng.uniform(0.5, 1.5)), float(rng.uniform(0.0, 3.0)),
                   float(rng.uniform(0.2, 2.0))) for _ in range(nbox)]
        out.append(dict(boxes=boxes, shears=shears, precision=str(rng.choice(["fp32", "fp32", "fp64"])),
                        graph=bool(rng.random() < 0.3), schedule="auto", seed=int(rng.integers(0, 2**31))))
    return out


BATCH_CASES = _batch_cases()


@pytest.mark.parametrize("case", BATCH_CASES, ids=[f"batch{i}" for i in range(len(BATCH_CASES))])
def test_random_batch_plan(case):
    test_random_plan(case)


def _wide_cases():
    # wide FP32 boxes fused on request (B = 64), each with a random partner box of the main draw
    # in the same plan half of the time: Nx, Ny in {512, 1024}, M = 64 or 128
    rng = np.random.default_rng(SEED + 2)
    out = []
    for _ in range(12):
        nx, ny = int(rng.choice([512, 1024])), int(rng.choice([512, 1024]))
        nz = 32 if nx * ny > 512 * 512 else int(rng.choice([32, 64]))
        wide = dict(nx=nx, ny=ny, nz=nz, lx=float(rng.uniform(0.5, 3.0)), ly=float(rng.uniform(0.5, 3.0)),
                    lz=float(rng.uniform(0.5, 2.0)), pad=2, alpha=0.0, method=str(rng.choice(["vgf", "sasha"])),
                    remap=str(rng.choice(["spectral", "spectral", "linear"])))
        boxes = [wide] + ([_draw_box(rng)] if rng.random() < 0.5 else [])
        shears = [(float(rng.choice([1.5, 2.0])), float(rng.uniform(0.5, 1.5)), float(rng.uniform(0.0, 3.0)),
                   float(rng.uniform(0.2, 2.0))) for _ in boxes]
        out.append(dict(boxes=boxes, shears=shears, precision="fp32", graph=bool(rng.random() < 0.3),
                        schedule="fused", seed=int(rng.integers(0, 2**31))))
    return out


WIDE_CASES = _wide_cases()


@pytest.mark.parametrize("case", WIDE_CASES, ids=[f"wide{i}" for i in range(len(WIDE_CASES))])
def test_random_wide_plan(case):
    test_random_plan(case)
