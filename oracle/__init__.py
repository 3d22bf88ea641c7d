"""FP64 CPU oracle of the spin-resolved PIC step.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``, never by the library or its Python
binding.  It shares no code with the HIP path.
"""

from .pic import (  # noqa: F401
    Grid, Sim, interpolate, gather, cross_matrix, midpoint_rotate, boris,
    tbmt_omega, spin_precess, move, wrap, shape_pair, deposit,
    charge_density, curl_E, curl_B, div_E, yee_step, kinetic_energy_mev,
    polarization, E_STAGGER, B_STAGGER, kinetic_energy_binned, bin_index,
    spectrum, phase_space,
)
from .tracking import (  # noqa: F401
    wake_fields, tracking_step, tracking_forward, objective, gradient_complex_step,
    per_particle_complex_step,
)
