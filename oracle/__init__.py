"""Oracle: a plain, slow, FP64 CPU implementation of the GLS map-making
problem of Szydlarski, Grigori & Stompor (A&A 2014, arXiv 1408.3048).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
call it.  It shares no code with the HIP path (no kernels, headers, helpers,
table generators or pre/post-processing).

Parity status of each function is listed in ``mapmaking.__doc__``.
"""

from .mapmaking import *  # noqa: F401,F403
