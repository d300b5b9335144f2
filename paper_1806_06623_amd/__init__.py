"""MI355X-native exact discrete Poisson solver on spherical polar grids.

Python binding of ``libsphpoisson.so`` (declared in ``include/sphpoisson.h``;
the streaming-copy reference in ``include/spp_reference.h``).
The binding only marshals arguments: every step of a solve runs in the HIP
kernels of the library.  PyTorch provides device memory and streams.
Importing this package fails loudly if the library has not been built
(``python paper_1806_06623_amd/build.py``).
"""
from ._binding import (  # noqa: F401
    LIB_PATH,
    Batch,
    Plan,
    Server,
    SphPoissonError,
    lib,
    precision_codes,
    stream_copy,
)

__all__ = ["Batch", "Plan", "Server", "SphPoissonError", "lib", "LIB_PATH", "precision_codes", "stream_copy"]
