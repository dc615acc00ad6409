"""MI355X (gfx950) twisted-mass solves and disconnected quark loops.

The compute path is the HIP library libtm.so (C-ABI in include/tm.h); this
package holds its sources (csrc/), the build script and a ctypes binding
with the same entry-point names.
"""
from .binding import *  # noqa: F401,F403
from .binding import Batch, Context, TMError, solve_params  # noqa: F401
from .storage import Base2Store  # noqa: F401
