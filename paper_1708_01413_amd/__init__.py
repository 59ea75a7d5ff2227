"""MI355X-native Accelerated Projection-based Consensus (APC) solver.

The solver is a C-ABI shared library of hand-written HIP kernels for gfx950
(``libapc.so``, declared in ``include/apc.h``); ``paper_1708_01413_amd.apc``
is its thin Python binding.  Importing this package does not load the
library; importing the binding does, and fails loudly if it is missing.
"""

__all__ = ["apc", "synth"]
