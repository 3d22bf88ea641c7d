"""Seeded synthetic inputs shared by the GPU path and the CPU oracle.

This package draws the initial particle phase space and evaluates the initial
laser field of a workload.  It holds no arithmetic of the PIC step itself
(gather, push, spin rotation, deposit, field update or the polarization sum):
both the HIP library and the oracle receive its output as plain arrays.
"""

from .workloads import (  # noqa: F401
    LAMBDA, ME_C2_MEV, MP_OVER_ME, A_E, A_P,
    electron, proton, courant_dt, preset, PRESETS,
    make_particles, make_laser_fields, make_state, grid_shape, make_static_fields,
    MICRON, tracking_preset, make_beam, batch_specs,
)
