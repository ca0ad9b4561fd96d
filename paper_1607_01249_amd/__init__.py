"""ttx: out-of-place N-D tensor transposition with scaling and update on MI355X.

B_{Pi(i)} <- alpha * A_i + beta * B_{Pi(i)} (Springer et al., TTC, Eqn. 1)
computed by hand-written HIP kernels for gfx950 behind the C ABI declared in
``include/ttx.h``.  This package is a thin ctypes binding of that library.
"""
from ._ttx import *  # noqa: F401,F403
from ._ttx import lib, transpose, TTXError, Config  # noqa: F401
