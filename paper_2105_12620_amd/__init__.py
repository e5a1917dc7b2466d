"""MI355X-native screen-space lattice-offset optimiser (Belcour & Heitz,
SIGGRAPH 2021 Talks): hand-written gfx950 kernels behind the C ABI in
include/bnlat.h, with a thin ctypes binding in :mod:`.bnlat`."""
from .bnlat import (BnlatError, Problem, create_problem, draw_heavisides, heaviside_area,  # noqa: F401
                    heaviside_array, lib, make_config, validate_config, window_classes)
