"""Seeded quenched U(1) gauge fields on a periodic Lx x Lt lattice.

Layout of every field returned here: ``theta[mu][t][x]`` (float64), the phase
of the link U_mu(x, t) = exp(i theta) that joins site (x, t) to its neighbour
in direction mu (mu = 0: x, mu = 1: t).  The gauge field itself is periodic in
both directions; the fermion boundary condition is applied by the operator, not
here.

The generator is a Metropolis chain for the Wilson plaquette action
S = beta * sum_p (1 - cos theta_p), started cold (all theta = 0).  Links are
updated in four checkerboard classes -- x-links on even t, x-links on odd t,
t-links on even x, t-links on odd x -- so that no two links of one class share
a plaquette and a whole class can be proposed and accepted at once.  One hit
per link per sweep, proposal theta + delta * u with u ~ U(-1, 1), numpy PCG64
seeded with ``seed``.
"""
from __future__ import annotations

import numpy as np


def _plaquettes(theta: np.ndarray) -> np.ndarray:
    """theta_p(x,t) = th0(x,t) + th1(x+1,t) - th0(x,t+1) - th1(x,t)."""
    th0, th1 = theta[0], theta[1]
    return th0 + np.roll(th1, -1, axis=1) - np.roll(th0, -1, axis=0) - th1


def plaquette_mean(theta: np.ndarray) -> float:
    """Average of cos(theta_p) over all plaquettes."""
    return float(np.mean(np.cos(_plaquettes(theta))))


def metropolis_u1(Lx: int, Lt: int, beta: float, sweeps: int, seed: int,
                  delta: float = 1.0) -> np.ndarray:
    """Return theta[2][Lt][Lx] after ``sweeps`` checkerboard Metropolis sweeps."""
    if Lx % 2 or Lt % 2:
        raise ValueError("checkerboard Metropolis needs even Lx and Lt")
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = np.zeros((2, Lt, Lx), dtype=np.float64)
    for _ in range(sweeps):
        # x-links, classes by parity of t: the link enters p(x,t) with +1 and
        # p(x,t-1) with -1.
        for par in (0, 1):
            p = _plaquettes(theta)
            pm = np.roll(p, 1, axis=0)  # p(x, t-1)
            d = delta * rng.uniform(-1.0, 1.0, size=(Lt // 2, Lx))
            u = rng.random(size=(Lt // 2, Lx))
            pc, pmc = p[par::2], pm[par::2]
            dS = beta * (np.cos(pc) - np.cos(pc + d) + np.cos(pmc) - np.cos(pmc - d))
            acc = u < np.exp(-dS)
            theta[0, par::2] += np.where(acc, d, 0.0)
        # t-links, classes by parity of x: the link enters p(x,t) with -1 and
        # p(x-1,t) with +1.
        for par in (0, 1):
            p = _plaquettes(theta)
            pm = np.roll(p, 1, axis=1)  # p(x-1, t)
            d = delta * rng.uniform(-1.0, 1.0, size=(Lt, Lx // 2))
            u = rng.random(size=(Lt, Lx // 2))
            pc, pmc = p[:, par::2], pm[:, par::2]
            dS = beta * (np.cos(pc) - np.cos(pc - d) + np.cos(pmc) - np.cos(pmc + d))
            acc = u < np.exp(-dS)
            theta[1, :, par::2] += np.where(acc, d, 0.0)
    return np.mod(theta + np.pi, 2.0 * np.pi) - np.pi


def links_from_theta(theta: np.ndarray) -> np.ndarray:
    """complex128 links[mu][t][x] = exp(i theta[mu][t][x])."""
    return np.exp(1j * theta).astype(np.complex128)


def random_gauge_transform(theta: np.ndarray, seed: int) -> np.ndarray:
    """theta_mu(x) -> theta_mu(x) + alpha(x) - alpha(x + mu) for random alpha.

    This is U_mu(x) -> g(x) U_mu(x) g(x+mu)^*, g(x) = exp(i alpha(x)).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    Lt, Lx = theta.shape[1:]
    alpha = rng.uniform(-np.pi, np.pi, size=(Lt, Lx))
    out = np.empty_like(theta)
    out[0] = theta[0] + alpha - np.roll(alpha, -1, axis=1)
    out[1] = theta[1] + alpha - np.roll(alpha, -1, axis=0)
    return out


def constant_phase_theta(Lx: int, Lt: int, phi_x: float, phi_t: float) -> np.ndarray:
    theta = np.empty((2, Lt, Lx), dtype=np.float64)
    theta[0] = phi_x
    theta[1] = phi_t
    return theta


def free_theta(Lx: int, Lt: int) -> np.ndarray:
    return np.zeros((2, Lt, Lx), dtype=np.float64)
