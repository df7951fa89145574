"""Seeded synthetic workloads shared by the tests, the benchmark and the CPU checker.

This package only describes problems (mesh size, decomposition, material and
boundary data) and draws seeded random numbers.  It contains none of the
preconditioner's arithmetic, so both the HIP path and the CPU checker can take
their inputs from it without sharing any of the method.
"""
from .workloads import (  # noqa: F401
    Workload,
    WORKLOADS,
    workload,
    random_vector,
    c3_inflow_amplitudes,
    c5_batch_draws,
    paper_variant_cases,
    small_parity_cases,
    voronoi_partition,
)
