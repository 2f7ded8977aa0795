"""FP64 CPU oracle (test infrastructure only; never imported by the product path)."""

from .shearing_poisson import (  # noqa: F401
    Box,
    Shear,
    FOUR_PI,
    cell_centres,
    fill_ghosts,
    gravity,
    green_sasha,
    green_vgf,
    mode_numbers,
    sasha_phi0,
    shear_offset,
    shift_y_linear,
    sheared_wavenumbers,
    solve,
)
