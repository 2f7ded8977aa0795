"""Every transform length the C ABI accepts, in every role, against the FP64 oracle.

sbp_box admits nx, ny and pad*nz in {8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512,
768, 1024}.  Each length appears below at least once as the x length, the y length and the
padded z length (P = 2 and P = 4), in FP64 and FP32, VGF and SASHA, with the other two axes
kept small so that the oracle finishes quickly.  Boxes outside the fused domain run the
five-pass schedule; the rest run fused by default and five-pass on request, so both schedules
see them."""

import numpy as np
import pytest

from paper_2510_10070_amd.inputs import lognormal_density

from .gpu_util import gpu_solve, max_pointwise_error, oracle_solve, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}

# (nx, ny, nz, pad): the length under test first, then the axis it sits on
CASES = [
    (8, 12, 4, 2),       # x 8, y 12, M 8
    (12, 8, 6, 2),       # x 12, M 12
    (24, 16, 12, 2),     # x 24, M 24
    (48, 24, 16, 2),     # x 48, y 24, M 32
    (192, 12, 8, 2),     # x 192, M 16
    (384, 8, 6, 2),      # x 384
    (512, 16, 4, 2),     # x 512
    (768, 8, 4, 2),      # x 768
    (1024, 8, 4, 2),     # x 1024
    (8, 48, 24, 2),      # y 48, M 48
    (8, 192, 6, 2),      # y 192
    (12, 384, 4, 2),     # y 384
    (8, 768, 4, 2),      # y 768
    (8, 1024, 4, 2),     # y 1024
    (8, 8, 48, 2),       # M 96
    (8, 8, 96, 2),       # M 192
    (8, 12, 192, 2),     # M 384
    (12, 8, 384, 2),     # M 768
    (8, 8, 512, 2),      # M 1024
    (8, 8, 256, 4),      # M 1024 with 4x padding
    (16, 16, 96, 4),     # M 384 with 4x padding
    (16, 8, 6, 4),       # M 24 with 4x padding
    (1024, 1024, 4, 2),  # x and y 1024 together
    (768, 384, 6, 2),
]


def _id(c):
    return "x".join(map(str, c[:3])) + f"_P{c[3]}"


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("method", ["vgf", "sasha"])
@pytest.mark.parametrize("case", CASES, ids=_id)
def test_every_length(case, method, precision):
    nx, ny, nz, pad = case
    box = dict(nx=nx, ny=ny, nz=nz, lx=1.0 + 0.001 * nx, ly=0.9 + 0.001 * ny, lz=1.0, pad=pad, alpha=0.0,
               method=method)
    rho = lognormal_density((nx, ny, nz), 1.0, 0.25, seed=nx * 7 + ny * 3 + nz)
    shear = (1.5, 1.0, 0.41, 1.0)
    for schedule in ("auto", "five_pass"):
        got, used = gpu_solve(box, rho, shear, precision, schedule=schedule)
        ref = oracle_solve(box, used[0], shear)
        err = rel_l2(got[0], ref)
        mp = max_pointwise_error(got[0], ref)
        print(f"{case} {method} {precision} {schedule}: rel-L2 {err:.3e}, max pointwise {mp:.3e}")
        assert err <= TOL[precision], (schedule, err)
        assert mp <= TOL[precision], (schedule, mp)
        assert np.isfinite(got[0]).all()
