"""The 2D Schwinger (U(1) Wilson-Dirac) operator used in the paper's numerics
(Sec. 4, Table 1): two spin components per site, nearest-neighbour hops,
shifted by a (negative) multiple of the identity.

Readings of the paper (it only names "the Schwinger discretization"):

* Wilson term r = 1, gamma matrices sigma_1 (x) and sigma_2 (t), gamma5 =
  sigma_3.  Every row then holds 1 diagonal entry and 4 full 2x2 hop blocks,
  i.e. 9 non-zeros per row: nnz(D_1) = 9 * 2 * 128^2 = 2.94e5, as Table 1
  prints.
* D = (m0 + 2) I - 1/2 sum_mu [ (1 - sigma_mu) U_mu(x) delta_{x+mu,y}
                              + (1 + sigma_mu) U_mu(x-mu)^* delta_{x-mu,y} ],
  i.e. the massless operator (diagonal 2) shifted by m0 I (Sec. 4).
* periodic boundary in x, antiperiodic in t: a hop that crosses the t
  boundary picks up a factor -1.

Index convention (the library's "logical index"): dof (t * Lx + x) * 2 + s.

Parity: pinned by tests (nnz per row, gamma5-hermiticity D^H = s3 D s3, gauge
covariance, the free-field and constant-phase Fourier closed forms of tr D^-1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

SIGMA = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),      # sigma_1, direction x
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),   # sigma_2, direction t
)
SIGMA3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
I2 = np.eye(2, dtype=np.complex128)


def wilson_dirac(theta: np.ndarray, m0: float, bc_t_anti: bool = True) -> sp.csr_matrix:
    """Sparse D for the link phases theta[mu][t][x] (complex128, n = 2 Lx Lt)."""
    _, Lt, Lx = theta.shape
    V = Lx * Lt
    U = np.exp(1j * theta)
    t, x = np.meshgrid(np.arange(Lt), np.arange(Lx), indexing="ij")
    site = (t * Lx + x).ravel()
    rows, cols, vals = [], [], []

    # diagonal: (m0 + 2) on both spins
    for s in range(2):
        rows.append(2 * site + s)
        cols.append(2 * site + s)
        vals.append(np.full(V, m0 + 2.0, dtype=np.complex128))

    for mu in range(2):
        if mu == 0:
            xf, tf = (x + 1) % Lx, t
            xb, tb = (x - 1) % Lx, t
            sign_f = np.ones_like(x, dtype=np.float64)
            sign_b = np.ones_like(x, dtype=np.float64)
        else:
            xf, tf = x, (t + 1) % Lt
            xb, tb = x, (t - 1) % Lt
            sign_f = np.where((t == Lt - 1) & bc_t_anti, -1.0, 1.0)
            sign_b = np.where((t == 0) & bc_t_anti, -1.0, 1.0)
        fwd = (tf * Lx + xf).ravel()
        bwd = (tb * Lx + xb).ravel()
        u_f = (U[mu] * sign_f).ravel()                 # U_mu(x)
        u_b = (np.conj(U[mu][tb, xb]) * sign_b).ravel()  # U_mu(x - mu)^*
        proj_f = -0.5 * (I2 - SIGMA[mu])
        proj_b = -0.5 * (I2 + SIGMA[mu])
        for a in range(2):
            for b in range(2):
                if proj_f[a, b] != 0:
                    rows.append(2 * site + a)
                    cols.append(2 * fwd + b)
                    vals.append(proj_f[a, b] * u_f)
                if proj_b[a, b] != 0:
                    rows.append(2 * site + a)
                    cols.append(2 * bwd + b)
                    vals.append(proj_b[a, b] * u_b)

    n = 2 * V
    D = sp.coo_matrix(
        (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)
    ).tocsr()
    D.sum_duplicates()
    return D


def gamma5(n_sites: int) -> sp.csr_matrix:
    """sigma_3 on every site: diag(+1, -1, +1, -1, ...)."""
    return sp.diags(np.tile(np.array([1.0, -1.0]), n_sites)).astype(np.complex128).tocsr()
