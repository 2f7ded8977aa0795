"""Parity at the full sizes of the measured workloads, in the launch configurations the
benchmark uses.

* 256^3 random-field workload: the benchmark's FP32 and FP64 plans (fused, autotuned), launched
  directly and graph-replayed, element by element against the full FP64 oracle.
* 128^3 log-normal workload (FP32) and the 64-box batch (FP32, autotuned, direct and
  graph-replayed, boxes of uneven size and shear), against the oracle box by box.
* 1024 x 1024 x 256 clumpy box (FP32), in the launch configuration of its workload: element by
  element against the full FP64 oracle (about a minute and 26 GiB of host memory), with the
  per-mode and max-pointwise bounds; also
    - a sheared plane wave at full size, checked at sampled points against the z profiles the
      oracle computes on a small horizontal grid of the same box (the operator is diagonal in the
      sheared horizontal modes, so these profiles do not depend on Nx, Ny);
    - on the clumpy density itself, properties that hold at any size: y-translation
      equivariance and linearity.
* 1024 x 1024 x 512 (the largest box the ABI accepts, M = 1024), FP32 and FP64: the sheared-wave
  check at sampled points.
"""

import math

import numpy as np
import pytest

import oracle
from paper_2510_10070_amd.inputs import batch_workload, workload

from .gpu_util import gpu_solve, max_pointwise_error, oracle_solve, per_mode_error, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _box(b, method="vgf"):
    nx, ny, nz, lx, ly, lz = b
    return dict(nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz, pad=2, alpha=0.0, method=method)


@pytest.mark.parametrize("graph", [False, True], ids=["direct", "graph"])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_benchmark_workload_256(precision, graph):
    w = workload("grf-256")
    box = _box(w["box"])
    rho = w["make"]()
    got, used = gpu_solve(box, rho, w["shear"], precision, graph=graph, autotune=True)
    ref = oracle_solve(box, used[0], w["shear"])
    err = rel_l2(got[0], ref)
    mp, pm = max_pointwise_error(got[0], ref), per_mode_error(got[0], ref)
    print(f"grf-256 {precision} {'graph' if graph else 'direct'}: rel-L2 {err:.3e}, max pointwise {mp:.3e}, "
          f"per-mode {pm:.3e}")
    assert err <= TOL[precision], err
    assert mp <= TOL[precision], mp
    assert pm <= TOL[precision], pm


def test_lognormal_128_fp32():
    w = workload("lognormal-128")
    box = _box(w["box"])
    got, used = gpu_solve(box, w["make"](), w["shear"], "fp32")
    err = rel_l2(got[0], oracle_solve(box, used[0], w["shear"]))
    print(f"lognormal-128 fp32: rel-L2 {err:.3e}")
    assert err <= TOL["fp32"], err


@pytest.mark.parametrize("graph", [False, True], ids=["direct", "graph"])
def test_batch_of_64_uneven_boxes_fp32(graph):
    ws = batch_workload()
    boxes = [_box(w["box"]) for w in ws]
    rhos = [w["make"]() for w in ws]
    shears = [w["shear"] for w in ws]
    got, used = gpu_solve(boxes, rhos, shears, "fp32", graph=graph, autotune=True)
    worst = 0.0
    for b, g, u, s in zip(boxes, got, used, shears):
        worst = max(worst, rel_l2(g, oracle_solve(b, u, s)))
    print(f"64-box batch fp32: worst rel-L2 {worst:.3e}")
    assert worst <= TOL["fp32"], worst


# ------------------------------------------------------------------------------------------
# 1024 x 1024 x 256


@pytest.mark.timeout(900)
def test_clumpy_1024_elementwise_against_oracle():
    import gc

    import torch

    from paper_2510_10070_amd import Box, Plan, Shear

    w = workload("clumpy-1024")
    b = w["box"]
    box = _box(b)
    rho = torch.tensor(w["make"](), dtype=torch.float32, device="cuda:0")
    plan = Plan(Box(*b), precision="fp32")
    phi = torch.empty_like(rho)
    plan.solve(rho, phi, Shear(*w["shear"]))
    torch.cuda.synchronize()
    print(f"clumpy-1024 fp32 schedule: {plan.describe()['path']}", flush=True)
    plan.close()
    used = rho.double().cpu().numpy()
    got = phi.cpu().numpy()
    del rho, phi
    torch.cuda.empty_cache()
    ref = oracle_solve(box, used, w["shear"])
    del used
    gc.collect()
    err = rel_l2(got, ref)
    mp = max_pointwise_error(got, ref)
    pm = per_mode_error(got, ref, zchunk=32)
    print(f"clumpy-1024 fp32 vs oracle: rel-L2 {err:.3e}, max pointwise {mp:.3e}, per-mode {pm:.3e}")
    assert err <= TOL["fp32"], err
    assert mp <= TOL["fp32"], mp
    assert pm <= TOL["fp32"], pm


def _sheared_wave(nx, ny, box, shear, mx=1, my=2):
    """cos(Kx x) cos(Ky (y + s x)) exp(-z^2/2): shear-periodic for integer mode numbers."""
    _, _, nz, lx, ly, lz = box
    q, om, t, _ = shear
    s = math.fmod(q * om * lx * t, ly) / lx
    x = (np.arange(nx) + 0.5) * lx / nx
    y = (np.arange(ny) + 0.5) * ly / ny
    z = -0.5 * lz + (np.arange(nz) + 0.5) * lz / nz
    Kx, Ky = 2 * math.pi * mx / lx, 2 * math.pi * my / ly
    X, Y = np.meshgrid(x, y, indexing="ij")
    horiz = np.cos(Kx * X) * np.cos(Ky * (Y + s * X))
    rho = horiz[:, :, None] * np.exp(-0.5 * z * z)[None, None, :]
    th1 = (Kx + s * Ky) * X + Ky * Y
    th2 = (Kx - s * Ky) * X - Ky * Y
    return rho, th1, th2


def test_clumpy_1024_sampled_against_oracle_profiles():
    import torch

    from paper_2510_10070_amd import Box, Plan, Shear

    w = workload("clumpy-1024")
    b = w["box"]
    nx, ny, nz = b[:3]
    # oracle on a small horizontal grid of the same box: Phi = cos(th1) P1(z) + cos(th2) P2(z)
    small = 16
    rho_s, th1_s, th2_s = _sheared_wave(small, small, b, w["shear"])
    ob = oracle.Box(small, small, nz, *b[3:])
    phi_s = oracle.solve(rho_s, ob, oracle.Shear(*w["shear"]))
    basis = np.stack([np.cos(th1_s).ravel(), np.cos(th2_s).ravel()], axis=1)
    prof, res, *_ = np.linalg.lstsq(basis, phi_s.reshape(small * small, nz), rcond=None)
    fit = basis @ prof
    assert np.abs(fit - phi_s.reshape(small * small, nz)).max() <= 1e-12 * np.abs(phi_s).max()

    # the same wave at full size on the GPU, in float
    rho_f, th1, th2 = _sheared_wave(nx, ny, b, w["shear"])
    plan = Plan(Box(*b), precision="fp32")
    r = torch.tensor(rho_f, dtype=torch.float32, device="cuda:0")
    del rho_f
    phi = torch.empty_like(r)
    plan.solve(r, phi, Shear(*w["shear"]))
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    ix, iy, iz = rng.integers(0, nx, 400000), rng.integers(0, ny, 400000), rng.integers(0, nz, 400000)
    got = phi[torch.as_tensor(ix), torch.as_tensor(iy), torch.as_tensor(iz)].double().cpu().numpy()
    want = np.cos(th1[ix, iy]) * prof[0, iz] + np.cos(th2[ix, iy]) * prof[1, iz]
    err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    print(f"clumpy-1024 box, sheared wave fp32: sampled rel-L2 {err:.3e}")
    # the input itself is rounded to float: allow for that on top of the float solve
    assert err <= TOL["fp32"], err
    plan.close()


def test_clumpy_1024_translation_and_linearity():
    import torch

    from paper_2510_10070_amd import Box, Plan, Shear

    w = workload("clumpy-1024")
    b = w["box"]
    rho = torch.tensor(w["make"](), dtype=torch.float32, device="cuda:0")
    plan = Plan(Box(*b), precision="fp32")
    sh = Shear(*w["shear"])
    phi = torch.empty_like(rho)
    plan.solve(rho, phi, sh)
    # y translation by 37 cells: the operator commutes with it (periodic y, x-independent shift)
    rolled = torch.roll(rho, 37, dims=1).contiguous()
    phi_r = torch.empty_like(rho)
    plan.solve(rolled, phi_r, sh)
    torch.cuda.synchronize()
    e_roll = (torch.linalg.vector_norm((torch.roll(phi, 37, dims=1) - phi_r).double())
              / torch.linalg.vector_norm(phi.double())).item()
    # linearity: Phi(rho + 0.5 rolled) = Phi(rho) + 0.5 Phi(rolled)
    mix = (rho + 0.5 * rolled).contiguous()
    phi_m = torch.empty_like(rho)
    plan.solve(mix, phi_m, sh)
    torch.cuda.synchronize()
    e_lin = (torch.linalg.vector_norm((phi_m.double() - phi.double() - 0.5 * phi_r.double()))
             / torch.linalg.vector_norm(phi_m.double())).item()
    assert torch.isfinite(phi).all().item()
    print(f"clumpy-1024 fp32: translation {e_roll:.3e}, linearity {e_lin:.3e}")
    assert e_roll <= TOL["fp32"], e_roll
    assert e_lin <= TOL["fp32"], e_lin
    plan.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_largest_box_sampled_against_oracle_profiles(precision):
    # the largest box the ABI accepts, 1024 x 1024 x 512 (M = 1024, five-pass): a sheared wave of
    # mode numbers (5, 7) at full size, sampled against the z profiles the oracle computes on a
    # 16 x 16 horizontal grid of the same box (the operator is diagonal in the sheared modes)
    import torch

    from paper_2510_10070_amd import Box, Plan, Shear

    b = (1024, 1024, 512, 16.0, 16.0, 4.0)
    shear = (1.5, 1.0, 5.0, 1.0)
    nx, ny, nz = b[:3]
    small = 16
    rho_s, th1_s, th2_s = _sheared_wave(small, small, b, shear, mx=5, my=7)
    phi_s = oracle.solve(rho_s, oracle.Box(small, small, nz, *b[3:]), oracle.Shear(*shear))
    basis = np.stack([np.cos(th1_s).ravel(), np.cos(th2_s).ravel()], axis=1)
    prof, *_ = np.linalg.lstsq(basis, phi_s.reshape(small * small, nz), rcond=None)
    assert np.abs(basis @ prof - phi_s.reshape(small * small, nz)).max() <= 1e-12 * np.abs(phi_s).max()

    rho_f, th1, th2 = _sheared_wave(nx, ny, b, shear, mx=5, my=7)
    dt = torch.float32 if precision == "fp32" else torch.float64
    plan = Plan(Box(*b), precision=precision)
    assert plan.describe()["path"] == "streaming-5pass"
    r = torch.tensor(rho_f, dtype=dt, device="cuda:0")
    del rho_f
    phi = torch.empty_like(r)
    plan.solve(r, phi, Shear(*shear))
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    ix, iy, iz = rng.integers(0, nx, 400000), rng.integers(0, ny, 400000), rng.integers(0, nz, 400000)
    got = phi[torch.as_tensor(ix), torch.as_tensor(iy), torch.as_tensor(iz)].double().cpu().numpy()
    want = np.cos(th1[ix, iy]) * prof[0, iz] + np.cos(th2[ix, iy]) * prof[1, iz]
    err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    print(f"1024x1024x512 sheared wave {precision}: sampled rel-L2 {err:.3e}")
    assert err <= TOL[precision], err
    plan.close()
