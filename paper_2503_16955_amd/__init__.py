"""MI355X-native per-ray Monte Carlo transport of mosaic-crystal
spectrometers (after HEART, arXiv 2503.16955).

The transport runs in hand-written HIP kernels for gfx950 behind the C-ABI
library ``libmosaicrt.so`` (declared in ``include/mosaicrt.h``).  The
``mosaicrt`` module is the thin Python binding: it marshals workload
descriptions into the library's structs and hands it torch device buffers
and the current stream.  Importing the package loads nothing; the library is
loaded on the first call and a missing library is an error.
"""
from . import workloads  # noqa: F401  (input descriptions only)
