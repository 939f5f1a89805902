"""MI355X (gfx950) implementation of the S-ADI time step of Sun & Sun (arXiv 2312.06206).

The work runs in libsadi.so (hand-written HIP kernels behind the C ABI of
include/sadi.h); this package only marshals arguments.  Importing the package does
not load the library: `Solver` and the host helpers load it on first use and raise
if it has not been built (`python -m paper_2312_06206_amd.build`).
"""
from .binding import (  # noqa: F401
    LIB_PATH,
    Batch,
    SadiError,
    Solver,
    host_laplacian_coeffs,
    host_line_generator,
    host_line_tables,
    host_quadrature_rows,
    host_riesz_coeffs,
    load_library,
)
