"""Seeded synthetic snapshot generator shared by the oracle tests, the HIP-path
tests and the benchmark.

This package holds no arithmetic of the FOA method itself: it only draws the
flow-shaped synthetic snapshot sequences x_j = Re(sum_m b_m phi_m lambda_m^(j-1))
+ noise (the snapshot model of Section 2 of the paper, with a linear map whose
eigenvalues are the lambda_m) and the workload descriptions they follow.
"""

from .workloads import WORKLOADS, Workload, BatchedWorkload, get_workload
from .snapshots import (
    mode_parameters,
    snapshots_numpy,
    snapshots_torch,
    batched_streams,
    expected_rms,
)

__all__ = [
    "WORKLOADS",
    "Workload",
    "BatchedWorkload",
    "get_workload",
    "mode_parameters",
    "snapshots_numpy",
    "snapshots_torch",
    "batched_streams",
    "expected_rms",
]
