"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package only draws pixels and job lists. It holds none of the resampling
arithmetic: coordinates, taps, weights and rounding live in the HIP library and,
independently, in the oracle.
"""

from .fields import (  # noqa: F401
    BatchJob,
    batch_jobs,
    field_u8,
    field_u8_torch,
    field_unit,
    normal_f32,
    smooth_field,
    smooth_field_torch,
    uniform_u8,
)
