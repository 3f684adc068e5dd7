"""MI355X-native maintenance of exact nearest-neighbour certificates for moving points.

The compute path is libnncert.so (hand-written HIP kernels for gfx950 behind a C
ABI declared in include/nncert.h); ``binding`` is its thin ctypes layer.
"""
from .binding import (NNCert, NNCError, allpairs_top2, load, NNC_FAILED, NNC_CANDIDATES,  # noqa: F401
                      EXPORTS)
