"""MI355X (gfx950) sequential posterior simulator: hand-written HIP kernels
behind the C ABI of include/smc.h, with a thin ctypes binding (``_lib``).

The package holds no numerical fallback: every step of the path runs in
libsmc.so, and calls raise if the library is missing.
"""
from . import _lib  # noqa: F401
from ._lib import *  # noqa: F401,F403
