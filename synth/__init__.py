"""Seeded synthetic visibility workloads.

This package only draws inputs: baseline coordinates (u, v, w) in wavelengths,
complex visibilities, weights and grid geometry.  It holds none of the
imaging arithmetic (no kernel, no gridding, no transform, no phase screen), so
both the HIP path and the oracle can take their inputs from here without
sharing any code of the method.
"""
from .workloads import (  # noqa: F401
    Workload,
    config1,
    config2,
    config3,
    config4,
    config5,
    random_case,
    hermitian_pairs,
    edge_case,
    rows_case,
    RowsWorkload,
    CONFIGS,
)
