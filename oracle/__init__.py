"""FP64 CPU oracle of the reactive-mixture LBM step.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the benchmark's
CPU-baseline leg.  The product path (paper_2101_01702_amd) never imports it.
"""
from .oracle import OracleSim, load  # noqa: F401
