"""MI355X-native hot path of gradient-decomposed multislice ptychography.

The work is done by the HIP library ``libptycho.so`` (include/ptycho.h);
this package is its Python binding plus the host-side tile scheduler.
"""
from ._binding import (  # noqa: F401
    Context,
    PtychoError,
    bin_positions,
    gd_step_size,
    lib,
    ptycho_forward,
    ptycho_shift_probes,
    split_positions,
    ptycho_loss,
    ptycho_loss_grad,
    ptycho_loss_grad_static,
    ptycho_tile_accumulate,
    ptycho_tile_grad,
    ptycho_tiles_grad,
    ptycho_zero_gradient,
    ptycho_box_exchange,
    ptycho_box_axpy,
    ptycho_potential_gradient,
    ptycho_potential_transmission,
    tile_box,
    validate_positions,
    version,
)
