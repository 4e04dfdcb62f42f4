"""Seeded synthetic inputs for the VANSE Carreau-Yasuda lattice Boltzmann step.

This package only builds geometry, porosity and boundary-condition inputs
(voxel masks, porosity fields, inlet shapes, parameter sets).  It holds none of
the method's arithmetic and is imported by both the FP64 oracle's tests and the
GPU path's tests and benchmark.
"""

from .cases import (  # noqa: F401
    Case,
    channel_case,
    aneurysm_case,
    coarsen2,
    coil_cases,
    periodic_box_case,
    tiny_case,
    tiny_random,
    fd_voxels,
    sampled_waveform,
    aniso_shape,
    as_d3q27,
    slab_of,
    with_anisotropic_drag,
    CONFIGS,
    make_config,
)
