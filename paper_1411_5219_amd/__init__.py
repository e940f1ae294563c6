"""MI355X (gfx950) Wilson / twisted-mass Wilson Dslash and Krylov solvers.

The compute path is the HIP library lib/liblqcd.so behind the C ABI of
include/lqcd.h; ``lqcd`` is its ctypes binding (importing it fails loudly
when the library has not been built) and ``fields`` holds torch helpers that
allocate device buffers and call the library's pack kernels.  The package
itself imports nothing eagerly so that ``paper_1411_5219_amd.build`` can run
before the library exists.
"""

__all__ = ["lqcd", "fields", "build"]
