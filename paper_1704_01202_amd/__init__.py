"""MI355X-native per-cell Monte-Carlo collision / ionization step for
XFEL-heated solid-density Al (collisional PIC method of Royle et al.).

The computation runs in libxpic.so (HIP kernels for gfx950, C ABI in
include/xpic.h).  This package holds the ctypes binding (`binding`), the
device-resident run driver (`runtime`) and the seeded input generators
(`workloads`).
"""

from . import binding, workloads  # noqa: F401
from .binding import (XP_ALL, XP_DECAY, XP_EE, XP_EI, XP_ION, XP_PHOTO, XP_REC,  # noqa: F401
                      bin_particles, collide_ionize_step, diagnostics, init_species,
                      photo_auger_step)

__all__ = ["binding", "workloads", "init_species", "bin_particles", "collide_ionize_step",
           "photo_auger_step", "diagnostics"]
