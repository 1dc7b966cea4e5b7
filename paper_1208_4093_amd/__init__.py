"""MI355X-native hierarchical lattice solver (gfx950 HIP kernels behind a C ABI).

The compute path is libtl.so; this package only binds it.  Importing the
package does not load the library; the first call does, and raises when the
library has not been built.
"""
from .tl import (TL_E_BUDGET, TL_E_DEVICE, TL_E_INVAL, TL_E_NOCONV, TL_E_NOMEM,  # noqa: F401
                 TL_E_NONFINITE, TL_FP64, TL_MIXED, TL_OK, TL_PENDING, Lattice, Server, TLError,
                 load, make_trace, tl_lattice_create, tl_poll, tl_residual, tl_server_create,
                 tl_solve, tl_solve_batch, tl_solve_noalloc, tl_strerror, tl_submit)
