"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package generates *inputs only*: U(1) gauge fields for the 2D Schwinger
model, gauge rotations of them, and seeded right-hand sides.  It holds none of
the trace-estimation arithmetic (no Dirac operator, no multigrid, no noise of
the estimator); the oracle and the HIP path each implement that on their own.
"""
from .gauge import (
    metropolis_u1,
    plaquette_mean,
    links_from_theta,
    random_gauge_transform,
    constant_phase_theta,
    free_theta,
)
from .workloads import WORKLOADS, gauge_for, rhs_vectors
from .cnn import cnn_init_params, cnn_param_count

__all__ = [
    "metropolis_u1",
    "plaquette_mean",
    "links_from_theta",
    "random_gauge_transform",
    "constant_phase_theta",
    "free_theta",
    "WORKLOADS",
    "gauge_for",
    "rhs_vectors",
    "cnn_init_params",
    "cnn_param_count",
]
