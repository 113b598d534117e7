"""Deflated Hutchinson, the paper's reference method (Sec. 2.1-2.3, Sec. 4).

Exact deflation (Sec. 2.2): with the singular triplets (u_i, v_i, sigma_i) of
D, D v_i = sigma_i u_i, sigma ascending, the orthogonal projector
Pi = V_k V_k^H splits tr(D^{-1}) = tr((I - Pi) D^{-1}) + tr(Pi D^{-1}); the
second term is sum_{i<=k} u_i^H v_i / sigma_i and the first is estimated by
Hutchinson (Alg. 1) on (I - Pi) D^{-1}.  Deflating the k smallest singular
triplets removes exactly sum_{i<=k} sigma_i^{-2} from ||D^{-1}||_F^2
(Sec. 2.1: the Frobenius norm is the 2-norm of the singular values).

The right singular vectors of D for the smallest sigma span the dominant
invariant subspace of D^{-1} D^{-H}; for the gamma5-hermitian Schwinger
operator D^{-H} = gamma5 D^{-1} gamma5, so the subspace needs solves with D
only.  ``subspace_basis`` runs block subspace iteration
X <- qr(D^{-1} gamma5 D^{-1} gamma5 X) from a seeded noise block (the
library runs the same steps on the GPU); with an approximate basis Q the
split tr(D^{-1}) = tr((I - QQ^H) D^{-1}) + tr(Q^H D^{-1} Q) still holds
exactly (Sec. 2.3, the second form), so the estimator stays unbiased.  The
Ritz triplets of D on span(Q) give the exact-deflation formula's value for
comparison (``ritz_triplet_trace``).

Test infrastructure: imported only by the tests and the benchmark's CPU
baseline.
"""
from __future__ import annotations

import numpy as np

from . import rng


def exact_triplets(D: np.ndarray, k: int):
    """The k smallest singular triplets of dense D: (U_k, sigma_k, V_k)."""
    U, s, Vh = np.linalg.svd(D)
    idx = np.argsort(s)[:k]
    return U[:, idx], s[idx], Vh.conj().T[:, idx]


def exact_deflated_trace(D: np.ndarray, k: int) -> complex:
    """tr(Pi D^{-1}) = sum_{i<=k} u_i^H v_i / sigma_i (Sec. 2.2)."""
    U, s, V = exact_triplets(D, k)
    return complex(np.sum(np.einsum("ij,ij->j", U.conj(), V) / s))


def subspace_basis(solve, g5, n: int, k: int, sweeps: int, noise: str, seed: int):
    """Orthonormal n x k basis from ``sweeps`` steps of block subspace
    iteration on D^{-1} D^{-H} = D^{-1} g5 D^{-1} g5, started from the noise
    block of purpose DEFLATE.  ``solve(X)`` = D^{-1} X, ``g5`` the gamma5
    sign vector (length n)."""
    X = rng.noise_block(noise, seed, rng.PURPOSE_DEFLATE, 0, 0, k, n)
    for _ in range(sweeps):
        Y = solve(g5[:, None] * X)
        Y = solve(g5[:, None] * Y)
        X, _ = np.linalg.qr(Y, mode="reduced")
    return X


def ritz_triplet_trace(Dop, Q: np.ndarray):
    """Ritz singular triplets of D on span(Q): W = D Q, W^H W = Y diag(s^2)
    Y^H, v_i = Q y_i, u_i = W y_i / s_i; returns (sum u_i^H v_i / s_i,
    s ascending)."""
    W = Dop @ Q
    lam, Y = np.linalg.eigh(W.conj().T @ W)
    s = np.sqrt(lam)
    C = W.conj().T @ Q
    tr = complex(np.sum(np.einsum("ij,ik,kj->j", Y.conj(), C, Y) / lam))
    return tr, s
