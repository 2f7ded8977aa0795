"""Every tile variant of the fused passes A and C against the FP64 oracle.

Passes A and C of the fused schedule exist in several tile shapes (variant 0: 32-byte rows;
1: 64-byte rows, float with Nx <= 128 and Ny <= 256; 2: pass C in 256-thread blocks over 16-byte
rows, Ny <= 256; 3: the split kernels holding one z column per lane, Ny <= 256).  The autotuner
picks among them per (pass, Ny, Nx); here a seeded tune cache makes a plan take a chosen pair,
which describe() must confirm, and the result must match the oracle."""

import itertools

import pytest

from paper_2510_10070_amd.inputs import lognormal_density

from .gpu_util import gpu_solve, oracle_solve, per_mode_error, rel_l2, seed_tune_cache

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}
KIND_A, KIND_C = 5, 7

# (nx, ny, nz, pad), all inside the fused domain (M = pad nz in {32, 64, 128, 192, 256, 512}):
# A = nx/16 in {4, 6, 16, 8}; nz = 8 is narrower than the 64-byte rows of variant 1, so its
# only tile per plane is ragged
SHAPES = [(64, 32, 8, 4), (96, 96, 48, 4), (256, 64, 16, 2), (128, 256, 32, 2)]


def variant_ok(precision, kind, shape, v):
    nx, ny = shape[:2]
    if v == 0:
        return True
    if v == 1:
        return precision == "fp32" and nx // 16 <= 8 and ny <= 256
    if v == 2:
        return kind == KIND_C and ny <= 256
    return ny <= 256


PAIRS = [(p, va, vc) for p in ("fp32", "fp64") for va, vc in itertools.product((0, 1, 3), (0, 1, 2, 3))
         if not (p == "fp64" and 1 in (va, vc))]


@pytest.mark.parametrize("precision,va,vc", PAIRS, ids=lambda x: str(x))
def test_fused_variant_pair(precision, va, vc, tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("SBP_TUNE_CACHE", str(cache))
    ran = 0
    for shape in SHAPES:
        if not (variant_ok(precision, KIND_A, shape, va) and variant_ok(precision, KIND_C, shape, vc)):
            continue
        nx, ny, nz, pad = shape
        seed_tune_cache(cache, precision, [(KIND_A, ny, nx, va), (KIND_C, ny, nx, vc)])
        for method, remap in (("vgf", "spectral"), ("sasha", "linear"), ("sasha", "spectral")):
            box = dict(nx=nx, ny=ny, nz=nz, lx=1.0, ly=1.2, lz=0.9, pad=pad, alpha=0.0, method=method, remap=remap)
            rho = lognormal_density((nx, ny, nz), 0.9, 0.2, seed=nx + ny + nz + va * 10 + vc)
            shear = (1.5, 1.0, 0.29, 1.0)
            from paper_2510_10070_amd import Box, Plan

            plan = Plan(Box(**box), precision=precision, autotune=True, schedule="fused")
            d = plan.describe()
            plan.close()
            assert d["path"] == "fused-3pass", d
            groups = {g["pass"]: g for g in d["groups"]}
            assert groups["fused_a"]["variant"] == va and groups["fused_a"]["tuned"] == "cache", d
            assert groups["fused_c"]["variant"] == vc and groups["fused_c"]["tuned"] == "cache", d
            got, used = gpu_solve(box, rho, shear, precision, autotune=True, schedule="fused")
            ref = oracle_solve(box, used[0], shear)
            err, pm = rel_l2(got[0], ref), per_mode_error(got[0], ref)
            print(f"{shape} A{va} C{vc} {method} {remap} {precision}: rel-L2 {err:.3e}, per-mode {pm:.3e}")
            assert err <= TOL[precision], (shape, method, remap, err)
            assert pm <= TOL[precision], (shape, method, remap, pm)
            ran += 1
    assert ran > 0


def test_autotuner_measures_fused_variants(tmp_path, monkeypatch):
    # an empty cache: the tuner times the variants of passes A and C and records its choice
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("SBP_TUNE_CACHE", str(cache))
    from paper_2510_10070_amd import Box, Plan

    for precision in ("fp32", "fp64"):
        plan = Plan(Box(64, 64, 32, 1.0, 1.0, 1.0), precision=precision, autotune=True, schedule="fused")
        d = plan.describe()
        plan.close()
        assert d["tuning"] == "measured", d
        for g in d["groups"]:
            assert g["tuned"] == ("default" if g["pass"] == "fused_b" else "measured"), d
        plan = Plan(Box(64, 64, 32, 1.0, 1.0, 1.0), precision=precision, autotune=True, schedule="fused")
        d2 = plan.describe()
        plan.close()
        assert d2["tuning"] == "cache", d2
        assert [g["variant"] for g in d2["groups"]] == [g["variant"] for g in d["groups"]]
    lines = cache.read_text().split("\n")
    assert sum(1 for ln in lines if ln.strip()) == 4  # (A, C) x (fp32, fp64)
