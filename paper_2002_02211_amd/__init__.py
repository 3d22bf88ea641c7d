"""MI355X-native spin-resolved particle-in-cell step (arXiv:2002.02211).

The computation lives in ``libspinpic.so`` (HIP kernels for gfx950 behind the
C ABI of ``include/spinpic.h``); ``spinpic`` is its ctypes binding.
"""

from . import spinpic  # noqa: F401
from .spinpic import (  # noqa: F401
    Simulation, PicError, make_config, config_from_spec, load_library,
    pic_init, pic_step, pic_polarization, pic_fields, pic_particles, pic_energy,
    pic_stats, pic_timing, pic_timing_read, pic_free,
    PIC_FP64, PIC_FP32_MIXED, PIC_ACC_FP32, PIC_ACC_FP64,
)
