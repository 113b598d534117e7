"""The synthetic workloads: lattice sizes, gauge-field recipes and solver settings.

Each workload stands in for the paper's single 128^2 Schwinger configuration
(Sec. 4, Table 1), which is not available: the gauge fields are seeded
quenched U(1) Metropolis fields (see ``gauge.py``), paired with a negative
Wilson mass so that the operator is ill-conditioned but not singular.
"""
from __future__ import annotations

import numpy as np

from .gauge import metropolis_u1

# Multigrid hierarchy is given as a list of aggregate block shapes (bx, bt)
# per coarsening step and the number of test vectors per step.
WORKLOADS = {
    # Plain method, small: 16x16, 2-level MG, Hutch++ with 8 vectors,
    # Rademacher noise, eps 1e-2.
    "schwinger16": dict(
        Lx=16, Lt=16, beta=3.0, sweeps=200, gauge_seed=1000, m0=-0.05,
        blocks=[(4, 4)], ntv=[4], noise="rademacher", d=[8], k_power=2,
        eps=1e-2, trace_seed=1,
    ),
    # Plain method at scale: 128x128, 3-level MG (4x4 then 2x2, 8 test
    # vectors), Hutch++ with 32 vectors, Z2xZ2 noise, eps 1e-3.
    "schwinger128": dict(
        Lx=128, Lt=128, beta=3.0, sweeps=200, gauge_seed=2000, m0=-0.10,
        blocks=[(4, 4), (2, 2)], ntv=[8, 8], noise="z2z2", d=[32, 32], k_power=2,
        eps=1e-3, trace_seed=2,
    ),
    # Small lattices used by parity tests that span several tiles and a
    # ragged RHS count.
    "schwinger32": dict(
        Lx=32, Lt=32, beta=3.0, sweeps=200, gauge_seed=3100, m0=-0.08,
        blocks=[(4, 4), (2, 2)], ntv=[8, 8], noise="z2z2", d=[8, 8], k_power=2,
        eps=1e-2, trace_seed=3,
    ),
    "schwinger64": dict(
        Lx=64, Lt=64, beta=3.0, sweeps=200, gauge_seed=3200, m0=-0.10,
        blocks=[(4, 4), (2, 2)], ntv=[8, 8], noise="z2z2", d=[16, 16], k_power=2,
        eps=1e-2, trace_seed=4,
    ),
    # Mixed-precision workload: 512x512, 3-level MG, 256 RHS.
    "schwinger512": dict(
        Lx=512, Lt=512, beta=4.0, sweeps=200, gauge_seed=4000, m0=-0.08,
        blocks=[(4, 4), (4, 4)], ntv=[8, 8], noise="z2z2", d=[32, 32], k_power=2,
        eps=1e-3, trace_seed=5,
    ),
}


# Batching workload: 8 independent fields on mixed lattices, (beta, m0, L, nRHS)
# per field, gauge seeds 3000 + i; each field's mass is kept clear of the
# critical mass of its coupling.
BATCH8 = [
    (2.0, -0.12, 256, 64), (2.0, -0.11, 64, 256), (3.0, -0.10, 128, 128), (3.0, -0.09, 256, 256),
    (4.0, -0.07, 64, 128), (4.0, -0.06, 128, 64), (5.0, -0.05, 256, 128), (5.0, -0.05, 64, 256),
]


def batch8_fields(sweeps: int = 200):
    """[(theta, m0, nrhs)] for the batching workload."""
    return [(metropolis_u1(L, L, beta, sweeps, 3000 + i), m0, nrhs)
            for i, (beta, m0, L, nrhs) in enumerate(BATCH8)]


def gauge_for(name_or_cfg) -> np.ndarray:
    cfg = WORKLOADS[name_or_cfg] if isinstance(name_or_cfg, str) else name_or_cfg
    return metropolis_u1(cfg["Lx"], cfg["Lt"], cfg["beta"], cfg["sweeps"], cfg["gauge_seed"])


def rhs_vectors(n: int, nrhs: int, seed: int) -> np.ndarray:
    """Seeded Z2xZ2 right-hand sides, complex128 of shape (nrhs, n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = np.sqrt(0.5)
    re = np.where(rng.random((nrhs, n)) < 0.5, -h, h)
    im = np.where(rng.random((nrhs, n)) < 0.5, -h, h)
    return (re + 1j * im).astype(np.complex128)
