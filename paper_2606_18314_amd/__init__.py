"""MI355X-native maintenance of exact nearest-neighbour certificates for moving points.

The compute path is libnncert.so (hand-written HIP kernels for gfx950 behind a C
ABI declared in include/nncert.h); ``binding`` is its thin ctypes layer.
"""
from .binding import (NNCert, NNCBatch, NNCError, allpairs_top2, load, NNC_FAILED,  # noqa: F401
                      NNC_CANDIDATES, EXPORTS, POLICY_REPAIR, POLICY_REBUILD, POLICY_THRESHOLD,
                      POLICY_LEARNED)
