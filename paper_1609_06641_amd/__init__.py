"""libchw: the Cascading Haar Wavelet (CHW) Walsh-Hadamard transform on
AMD Instinct MI355X (gfx950).

The transform itself lives in libchw.so (HIP kernels behind the C ABI of
include/chw.h); this package holds its sources (csrc/), the build step
(_build.py) and the ctypes binding (chw.py).
"""

from .chw import (  # noqa: F401
    CHWError,
    Plan,
    chw_function,
    load,
    transform,
    version,
)
