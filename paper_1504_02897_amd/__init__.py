"""MI355X-native NUFFT dipole-dipole interaction (DDI) solver.

The compute path is the HIP library ``libddi.so`` (built from ``csrc/``) behind
the C ABI declared in ``include/ddi.h``; ``ddi`` holds the ctypes binding and
the autograd functions.  ``inputs`` holds the seeded synthetic workloads.

The binding is imported lazily so that ``inputs`` can be used without the
library.
"""

__all__ = ["inputs"]
