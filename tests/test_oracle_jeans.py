"""Jeans instability (Sect. 3.4) with the oracle as the Poisson solver: the oscillation period
and the collapse time of a one-dimensional isothermal gas must follow the linear theory, an
analytic dispersion relation independent of the solver."""

import pytest

import oracle

from . import jeans

OSC_RATIOS = (0.25, 0.5, 0.75)
COLL_RATIOS = (1.5, 2.0, 4.0)


def oracle_accel_factory(dx):
    s = jeans.SLAB
    box = oracle.Box(jeans.NX, s["ny"], s["nz"], jeans.LAM, s["ly"], s["lz"], method="vgf")
    sh = oracle.Shear(q=0.0, omega=1.0, t=0.0, G=jeans.G)
    mid = s["nz"] // 2

    def accel(rho_x):
        phi = oracle.solve(jeans.slab_density(rho_x, s["ny"], s["nz"]), box, sh)
        gx, _, _ = oracle.gravity(oracle.fill_ghosts(phi, 1), box, sh, 1)
        return 0.5 * (gx[:, 0, mid - 1] + gx[:, 0, mid])  # midplane

    return accel


@pytest.mark.parametrize("ratio", OSC_RATIOS)
def test_jeans_oscillation_period(ratio):
    ts, a = jeans.run(ratio, oracle_accel_factory, 1.4 * jeans.t_osc(ratio))
    got = jeans.measured_period(ts, a)
    err = abs(got / jeans.t_osc(ratio) - 1.0)
    print(f"lam/lam_J = {ratio}: T_osc {got:.5f} vs {jeans.t_osc(ratio):.5f}, error {err:.2e}")
    assert err < jeans.OSC_TOL


@pytest.mark.parametrize("ratio", COLL_RATIOS)
def test_jeans_collapse_time(ratio):
    ts, a = jeans.run(ratio, oracle_accel_factory, 1.5 * jeans.t_coll(ratio))
    got = jeans.measured_collapse(ts, a)
    err = abs(got / jeans.t_coll(ratio) - 1.0)
    print(f"lam/lam_J = {ratio}: T_coll {got:.5f} vs {jeans.t_coll(ratio):.5f}, error {err:.2e}")
    assert err < jeans.COLL_TOL
