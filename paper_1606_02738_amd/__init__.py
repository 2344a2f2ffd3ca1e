"""MI355X-native cell-based SPH neighbour interactions (density with smoothing-
length iteration, ghost, symmetric force, kick-drift-kick step) behind the
C-ABI of include/sph.h; see :mod:`paper_1606_02738_amd.sph` for the binding."""
from .sph import SPH, SPHError, lib, to_device, to_host  # noqa: F401
