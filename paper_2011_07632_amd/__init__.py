"""MI355X-native SPD HSS preconditioner for H^2 kernel matrices.

A thin Python binding over the C-ABI library ``libspdhss.so`` (see
include/spdhss.h).  PyTorch supplies device memory and the HIP stream; every
step of the computation runs in the library's HIP kernels.  There is no CPU
fallback: importing this package without the built library raises.
"""
from .binding import (  # noqa: F401
    KERNELS,
    SpdError,
    H2Matrix,
    HSSMatrix,
    ULVFactor,
    h2_build,
    spdhss_build,
    ulv_factor,
    ulv_apply,
    h2_matvec,
    pcg_solve,
    lib,
)
