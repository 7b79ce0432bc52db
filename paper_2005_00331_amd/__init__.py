"""Matrix-free phase-field fracture linear solver for AMD MI355X (gfx950).

The compute path lives in libmfpff.so (HIP kernels behind the C ABI of
include/mfpff.h); this package is its ctypes binding and the autograd
wrapper of the residual.
"""
from .binding import (F32, F64, OP_ACCUMULATE, OP_BLOCKDIAG, OP_G, OP_GT, Context, MfpffError, Problem,  # noqa: F401
                      load_library, make_problem, problem_from)
