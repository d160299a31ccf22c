"""MI355X-native discrete-ordinates source iteration (HIP kernels for gfx950
behind the C ABI of include/dsn.h).  The Python layer only marshals
arguments; see dsn.py."""
from .dsn import (CONVERGED, DSN_FP32, DSN_FP64, DsnError, Problem, quadrature, solve_batch,  # noqa: F401
                  BATCH_FUSED, BATCH_STREAMS, LIB_PATH, lib, last_error)
from .autograd import fluence  # noqa: F401
