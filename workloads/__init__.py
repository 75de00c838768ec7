"""Seeded synthetic sparse-tensor workloads.

This package only draws random inputs: coordinates, values, factor matrices
and job streams.  It holds none of the MTTKRP or CP-ALS arithmetic, so both
the CPU oracle (through the tests) and the GPU path can consume its output
without sharing any code of the method.
"""

from .gen import (  # noqa: F401
    SparseTensor,
    named_tensor,
    batch_tensors,
    job_stream,
    random_factors,
    random_tensor,
    zipf_cdf,
    WORKLOADS,
)
