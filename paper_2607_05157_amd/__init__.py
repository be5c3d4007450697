"""MI355X (gfx950) stochastic trace estimation for the Wilson-Dirac operator.

The computation runs in libwdt.so (hand-written HIP kernels behind the C
interface in include/wdt.h); this package is its Python binding plus the
host-side estimator bookkeeping.
"""
from . import wdt  # noqa: F401
from .wdt import (FP16, FP32, FP64, Gauge, Lattice, apply_D, colouring_check,  # noqa: F401
                  colouring_search, contract, force, init, solve, source_descs, sources)
