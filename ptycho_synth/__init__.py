"""Seeded synthetic inputs for the multislice ptychography path.

This module only draws and shapes inputs: phase objects made of Gaussian
"atoms" on a jittered lattice, a defocused probe behind a circular aperture,
raster scan positions and Poisson counts.  It holds none of the method's
arithmetic (no multislice propagation, no loss, no gradient), so both the
FP64 oracle tests and the GPU path can consume the very same arrays.

The stand-in workloads mirror the paper's experimental setup (Section VI-A):
electron ptychography of a crystalline sample (atomic columns rendered as
Gaussian blobs), a probe formed by a ~30 mrad aperture with defocus, and a
raster scan with strong overlap between neighbouring windows (Section II-A).
"""
from .generators import (  # noqa: F401
    PHYSICS,
    WorkloadSpec,
    atom_phase,
    make_object,
    make_probe,
    raster_positions,
    raster_offset,
    poisson_counts,
    eval_object,
    workload,
    WORKLOAD_NAMES,
    build_inputs,
    batch_specs,
    seed_streams,
    with_overrides,
    reduced,
)
