"""The pins must catch plausible oracle mistakes: each case plants one in the oracle (on the
CPU, by monkeypatching a module-level function) and checks that a pin then fails."""

import math

import numpy as np
import pytest

import oracle.shearing_poisson as sp

from . import test_oracle_bruteforce as tb
from . import test_oracle_green as tg
from . import test_oracle_physics as tp
from . import test_oracle_gravity as tgr
from . import test_oracle_remap_linear as tl


ORIG_GREEN = sp.green_vgf
ORIG_MODES = sp.mode_numbers
ORIG_OFFSET = sp.shear_offset
ORIG_WAVENUMBERS = sp.sheared_wavenumbers
ORIG_PHI0 = sp.sasha_phi0
ORIG_SHIFT = sp.shift_y_linear


def green_wrong_sign_sin(k, kz, L):
    # flips the sign of the kz/k sin term in the k != 0 branch
    k, kz = np.broadcast_arrays(np.asarray(k, float), np.asarray(kz, float))
    out = ORIG_GREEN(k, kz, L)
    c = k != 0
    kk, q = k[c], kz[c]
    out[c] = -(np.exp(-kk * L) * (-(q / kk) * np.sin(q * L) - np.cos(q * L)) + 1.0) / (kk * kk + q * q)
    return out


def green_truncation_2L(k, kz, L):
    # uses the full width 2L where the paper's rect has half-width L
    return ORIG_GREEN(k, kz, 2.0 * L)


def modes_no_negative(n):
    return np.arange(n, dtype=np.int64)


def wavenumbers_lx_ly_swapped(box, s):
    b2 = sp.Box(box.nx, box.ny, box.nz, box.ly, box.lx, box.lz, box.pad, box.alpha, box.method)
    return ORIG_WAVENUMBERS(b2, s)


def offset_negated(q, omega, lx, ly, t):
    return -ORIG_OFFSET(q, omega, lx, ly, t)


def phi0_box_mean(rho, box, G):
    return ORIG_PHI0(rho, box, G) * box.pad


def shift_wrong_direction(f, d):
    # interpolates at j - d instead of j + d
    return ORIG_SHIFT(f, -np.asarray(d))


def shift_nearest_cell(f, d):
    # rounds to the nearest cell instead of interpolating
    return ORIG_SHIFT(f, np.round(np.asarray(d)))


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


@pytest.mark.parametrize(
    "attr,mutant,pin",
    [
        ("green_vgf", green_wrong_sign_sin, lambda: tg.test_green_vgf_matches_quadrature(2.5, 1.0, 1.0)),
        ("green_vgf", green_truncation_2L, lambda: tp.test_1d_vgf_fixes_the_constant()),
        ("green_vgf", green_truncation_2L, lambda: tg.test_green_vgf_matches_quadrature(1.0, 0.3, 1.0)),
        ("mode_numbers", modes_no_negative, lambda: tp.test_sheared_closed_form(0.3)),
        ("mode_numbers", modes_no_negative, lambda: tb.test_oracle_equals_brute_force(tb.CASES[1])),
        ("sheared_wavenumbers", wavenumbers_lx_ly_swapped, lambda: tp.test_sheared_closed_form_non_cubic()),
        ("shear_offset", offset_negated, lambda: tp.test_sheared_closed_form(0.3)),
        ("shear_offset", offset_negated, lambda: tp.test_shear_offset_wraps_into_box()),
        ("sasha_phi0", phi0_box_mean, lambda: tp.test_sasha_phi0_solves_its_equation()),
        ("sasha_phi0", phi0_box_mean, lambda: tb.test_oracle_equals_brute_force(tb.CASES[3])),
        ("shift_y_linear", shift_wrong_direction,
         lambda: tl.test_linear_equals_spectral_for_whole_cell_shifts((8, 32, 4, 1.0, 4.0, 1.0, 2.0, 1.0, 1.0), "vgf")),
        ("shift_y_linear", shift_nearest_cell, lambda: tl.test_linear_remap_converges_at_second_order()),
        ("shift_y_linear", shift_wrong_direction, lambda: tgr.test_gravity_second_order(0.41)),
    ],
)
def test_pin_catches_mutation(monkeypatch, attr, mutant, pin):
    pin()  # passes on the real oracle
    monkeypatch.setattr(sp, attr, mutant)
    # the test modules imported names from the oracle package; patch those too
    import oracle

    if hasattr(oracle, attr):
        monkeypatch.setattr(oracle, attr, mutant)
    for mod in (tb, tg, tp, tl, tgr):
        if hasattr(mod, attr):
            monkeypatch.setattr(mod, attr, mutant)
    assert _fails(pin), f"pin did not catch mutated {attr}"


def test_mutation_of_normalisation_caught(monkeypatch):
    monkeypatch.setattr(sp, "FOUR_PI", 2.0 * math.pi)
    assert _fails(tp.test_sheared_closed_form, 0.3)
