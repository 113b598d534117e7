"""Seeded inputs for the learned initial-guess network: its initial weights
and the gauge fields it is trained and evaluated on.

Network shape (interface only): 3x3 convolutions 4 -> 32 -> 32 -> 32 -> 4
channels, parameters packed as W1 b1 W2 b2 W3 b3 W4 b4 with W[co][ci][dt][dx].
"""
from __future__ import annotations

import numpy as np

from .gauge import metropolis_u1

WIDTHS = (4, 32, 32, 32, 4)

# training: 20 fields at 128^2, beta 3.0, m0 -0.10, seeds 5000..5019;
# evaluation: unseen fields, seeds 5100.., at 256^2 and 512^2
TRAIN_FIELDS = [dict(L=128, beta=3.0, m0=-0.10, seed=5000 + i) for i in range(20)]
EVAL_FIELDS = [dict(L=L, beta=3.0, m0=-0.10, seed=5100 + i)
               for i, L in enumerate([256] * 8 + [512] * 8)]


def cnn_param_count(widths=WIDTHS) -> int:
    return int(sum(co * ci * 9 + co for ci, co in zip(widths[:-1], widths[1:])))


def cnn_init_params(seed: int, widths=WIDTHS, scale: float = 1.0) -> np.ndarray:
    """He-style normal weights (std sqrt(2 / (9 cin))) and zero biases, float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for ci, co in zip(widths[:-1], widths[1:]):
        out.append((scale * np.sqrt(2.0 / (9 * ci)) * rng.standard_normal((co, ci, 3, 3))).ravel())
        out.append(np.zeros(co))
    return np.concatenate(out)


def field(spec, sweeps: int = 200) -> np.ndarray:
    return metropolis_u1(spec["L"], spec["L"], spec["beta"], sweeps, spec["seed"])
