"""FP64 CPU oracle for the MASK hot path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.
"""
from . import compare, mask_oracle  # noqa: F401
