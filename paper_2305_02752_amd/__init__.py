"""MI355X-native coupled fluid-cell time step (HemoCell model, arXiv 2305.02752).

The compute path is libhemo.so (hand-written HIP for gfx950 behind the C ABI
in include/hemo.h); `hemo` is its Python binding.
"""
from .hemo import (  # noqa: F401
    HC_PERIODIC, HC_WALL, HC_PHI2, HC_PHI4, HemoError, Simulation, Batch, Packer, load_library, LIB_PATH,
)
