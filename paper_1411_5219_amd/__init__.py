"""MI355X (gfx950) Wilson / twisted-mass Wilson Dslash and Krylov solvers.

The compute path is the HIP library lib/liblqcd.so behind the C ABI of
include/lqcd.h; ``lqcd`` is its ctypes binding and ``fields`` holds torch
helpers that allocate device buffers and call the library's pack kernels.
"""

from . import lqcd  # noqa: F401  (fails loudly when the library is missing)

__all__ = ["lqcd"]
