"""Plain FP64 CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library: the arithmetic lives in ``oracle.c`` (own radix-2 FFT, tensor-index
operator, textbook PCG, Green-matrix and projected routes, dense solve,
Newmark, direct convolution); this module only marshals numpy arrays.
"""
from .oracle import *  # noqa: F401,F403
