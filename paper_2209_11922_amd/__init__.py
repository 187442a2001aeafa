"""MI355X-native exponential-integrator Q1 finite element (EIFE) library.

The compute path is the HIP library libeife.so (C ABI in include/eife.h);
this package is a thin ctypes binding that marshals arguments and uses
PyTorch only for device memory and streams.  There is no fallback: without
the built library every entry point raises.
"""
from .binding import (  # noqa: F401
    BC_DIRICHLET,
    BC_PERIODIC,
    Batch,
    Corrector,
    EIFEError,
    Grid,
    LOAD_LUMPED,
    LOAD_NODAL,
    F_AFFINE_T,
    F_ALLEN_CAHN,
    F_CONST,
    F_EX51,
    F_FLORY_HUGGINS,
    F_TRAVELING_WAVE,
    F_MMS_U2,
    F_ZERO,
    library_path,
    load_library,
)
