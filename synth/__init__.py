"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package only draws random numbers and fixes the model constants of the
synthetic carbon clusters.  It computes nothing of the method itself (no
Hamiltonian, no integrals, no density matrices): both sides of every parity
test take their inputs from here and do all of the arithmetic themselves.
"""

from .clusters import (  # noqa: F401
    ModelParams,
    OverlapModel,
    System,
    carbon_cluster,
    ensemble_sizes,
    WORKLOADS,
    workload,
)
