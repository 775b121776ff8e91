"""MI355X (gfx950) supernodal sparse Cholesky and sparse triangular solve.

A thin ctypes binding over the C ABI in ``include/sym.h`` (library
``libsym.so`` built in-tree by ``build.py``).  Argument marshalling only:
the symbolic analysis runs in the library's host code and every numeric
step runs in its HIP kernels on the device and stream torch supplies.
"""
from .binding import (Analysis, Batch, RhsPlan, SymError, load_library, opts_default,  # noqa: F401
                      SYM_ORDER_ND, SYM_ORDER_NATURAL, SYM_ORDER_USER, SYM_F64, SYM_F32,
                      SYM_BF16, SYM_F16)
