"""Seeded synthetic compaction workloads.

This package draws the *logical* content of input tables (user keys, sequence
numbers, value types and value bytes) and nothing else: it holds no part of the
table format or of the compaction arithmetic.  Both the CPU oracle and the GPU
library consume what it draws; each encodes or decodes tables on its own.
"""
from .generate import (  # noqa: F401
    Run, Job, TYPE_DELETION, TYPE_VALUE,
    plain_small, plain_large, plain_variable, batch_job, batch_job_sizes, tiny_job, job_input_bytes_estimate,
    compressible,
)
