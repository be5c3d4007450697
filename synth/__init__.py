"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This package holds input generators only: random SU(3) gauge fields and the
seeded parameter streams of the workloads.  It contains none of the trace
estimator's arithmetic (no Dirac operator, no noise, no solver, no contraction),
so the oracle and the HIP path can both consume its output without sharing code.
"""
from .gauge import gauge_field, gell_mann, reunitarise  # noqa: F401
from .workloads import WORKLOADS, workload, batched_instances  # noqa: F401
