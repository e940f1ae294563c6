"""FP64 CPU oracle of the Wilson / twisted-mass fermion matrix and solvers.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import it; the product library never
does, and this package never imports the product library.
"""

from . import accounting, solvers, wilson  # noqa: F401
