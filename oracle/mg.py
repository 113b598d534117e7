"""Aggregation multigrid hierarchy for the Schwinger operator (Sec. 3.1, Sec. 4).

The paper builds the hierarchy "with a bootstrap setup and aggregation based
prolongations as in DD-alpha-AMG" and relies on R_l = P_l^H with orthonormal
columns, P_l^H P_l = I (Sec. 3.1, eq. mlmc_dec_trace_reduced), and on Galerkin
coarse operators D_{l+1} = R_l D_l P_l (Sec. 3.1).  It gives no further
details; the setup below is our own deterministic reading, chosen so that P is
unique (the reduced-form coarse noise depends on the exact coarse basis):

1. V <- Z2xZ2 noise (purpose SETUP, level l), n_l x ntv.
2. Three times: V <- qr+(D_l^{-1} V)          (block inverse iteration)
   where qr+ is the thin QR with real positive diag(R) (unique).
3. For every aggregate A and chirality c, the rows of V belonging to (A, c)
   -- sites of A in t-major order, then the dofs of chirality c of each
   site -- are replaced by qr+ of that row block: these are the columns
   (A, c, k), k < ntv, of P_l.  Aggregates split the chirality (spin on the
   fine level), so the coarse sigma_3 stays diagonal.
4. D_{l+1} = P_l^H D_l P_l.

Coarse logical index: ((A * 2 + c) * ntv + k), A = At * NAx + Ax.

Also here: the reference preconditioner (SAP smoother with exact block solves,
red/black; K-cycle with fixed-length inner FGMRES) that pins the HIP solver's
preconditioner.  It is a solver choice, not part of the method: the paper
leaves the solver open, so this part is "parity unpinned" with respect to the
paper and pinned only by the mathematical special cases in the tests.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import rng
from .dirac import wilson_dirac


@dataclass
class Level:
    Nx: int
    Nt: int
    M: int                      # dof per site
    D: sp.csr_matrix
    _lu: object = field(default=None, repr=False)

    @property
    def n(self) -> int:
        return self.Nx * self.Nt * self.M

    def solve(self, B: np.ndarray) -> np.ndarray:
        """Exact D^{-1} B by sparse LU (SuperLU)."""
        if self._lu is None:
            self._lu = spla.splu(self.D.tocsc())
        return self._lu.solve(np.ascontiguousarray(B))

    def chirality(self) -> np.ndarray:
        """+1 / -1 per dof: sigma_3 on the fine level, P^H sigma_3 P on coarse."""
        half = self.M // 2
        per_site = np.concatenate([np.ones(half), -np.ones(half)])
        return np.tile(per_site, self.Nx * self.Nt)


def qr_plus(A: np.ndarray) -> np.ndarray:
    """Thin QR of A (m >= n) with the real-positive-diagonal normalisation of R."""
    Q, R = np.linalg.qr(A, mode="reduced")
    d = np.diag(R)
    ph = d / np.abs(d)
    return Q * ph[None, :]


def aggregate_rows(Nx: int, Nt: int, M: int, bx: int, bt: int, A: int, c: int) -> np.ndarray:
    """Row indices of aggregate A, chirality c (sites t-major, then dofs)."""
    NAx = Nx // bx
    Ax, At = A % NAx, A // NAx
    half = M // 2
    rows = []
    for dt in range(bt):
        for dx in range(bx):
            site = (At * bt + dt) * Nx + (Ax * bx + dx)
            for kk in range(half):
                rows.append(site * M + c * half + kk)
    return np.array(rows, dtype=np.int64)


def build_prolongation(lev: Level, bx: int, bt: int, V: np.ndarray):
    """P (sparse, n x nc) and its dense blocks Pb[A][c][row][k]."""
    if lev.Nx % bx or lev.Nt % bt:
        raise ValueError("lattice not divisible by the aggregate block")
    ntv = V.shape[1]
    nagg = (lev.Nx // bx) * (lev.Nt // bt)
    nrow = bx * bt * (lev.M // 2)
    if nrow < ntv:
        raise ValueError("aggregate has fewer rows than test vectors")
    Pb = np.empty((nagg, 2, nrow, ntv), dtype=np.complex128)
    ri, ci, vv = [], [], []
    for A in range(nagg):
        for c in range(2):
            rows = aggregate_rows(lev.Nx, lev.Nt, lev.M, bx, bt, A, c)
            Qloc = qr_plus(V[rows, :])
            Pb[A, c] = Qloc
            for k in range(ntv):
                ri.append(rows)
                ci.append(np.full(nrow, (A * 2 + c) * ntv + k))
                vv.append(Qloc[:, k])
    nc = nagg * 2 * ntv
    P = sp.coo_matrix((np.concatenate(vv), (np.concatenate(ri), np.concatenate(ci))),
                      shape=(lev.n, nc)).tocsr()
    return P, Pb


@dataclass
class Hierarchy:
    levels: list
    P: list          # sparse prolongations, P[l]: level l+1 -> level l
    Pb: list         # dense aggregate blocks of P[l]
    V: list          # final test vectors per coarsening step (after inverse iteration)

    @property
    def L(self) -> int:
        return len(self.levels)


def setup_hierarchy(theta: np.ndarray, m0: float, blocks, ntv, seed: int,
                    setup_iters: int = 3, bc_t_anti: bool = True) -> Hierarchy:
    """Build levels 0..len(blocks) following the setup reading in the module doc."""
    _, Lt, Lx = theta.shape
    levels = [Level(Lx, Lt, 2, wilson_dirac(theta, m0, bc_t_anti))]
    Ps, Pbs, Vs = [], [], []
    for l, ((bx, bt), nt) in enumerate(zip(blocks, ntv)):
        lev = levels[l]
        V = rng.noise_block(rng.Z2Z2, seed, rng.PURPOSE_SETUP, l, 0, nt, lev.n)
        for _ in range(setup_iters):
            V = qr_plus(lev.solve(V))
        P, Pb = build_prolongation(lev, bx, bt, V)
        Dc = (P.conj().T @ lev.D @ P).tocsr()
        Dc.eliminate_zeros()
        levels.append(Level(lev.Nx // bx, lev.Nt // bt, 2 * nt, Dc))
        Ps.append(P)
        Pbs.append(Pb)
        Vs.append(V)
    return Hierarchy(levels, Ps, Pbs, Vs)


def coarsest_trace(lev: Level, dense_max: int = 8192, blk: int = 512) -> complex:
    """tr(D_L^{-1}) computed directly (Sec. 3.1; Alg. 2, coarsest level).

    Up to ``dense_max`` rows by a dense inverse; above, by sparse-LU solves
    against blocks of ``blk`` identity columns, summing the diagonal entries
    of D^{-1} they produce."""
    if lev.n <= dense_max:
        return complex(np.trace(np.linalg.inv(lev.D.toarray())))
    total = 0.0 + 0.0j
    for j0 in range(0, lev.n, blk):
        j1 = min(lev.n, j0 + blk)
        E = np.zeros((lev.n, j1 - j0), dtype=np.complex128)
        E[np.arange(j0, j1), np.arange(j1 - j0)] = 1.0
        X = lev.solve(E)
        total += np.sum(X[np.arange(j0, j1), np.arange(j1 - j0)])
    return complex(total)


# --------------------------------------------------------------------------
# Reference preconditioner (solver choice; parity unpinned w.r.t. the paper)
# --------------------------------------------------------------------------

def sap_blocks(lev: Level, sbx: int, sbt: int):
    """Dof index lists, colours and exact block inverses of D restricted to
    each sbx x sbt block of sites (sites t-major, then dofs)."""
    NBx, NBt = lev.Nx // sbx, lev.Nt // sbt
    idx, color, inv = [], [], []
    Dcsr = lev.D.tocsr()
    for ibt in range(NBt):
        for ibx in range(NBx):
            rows = []
            for dt in range(sbt):
                for dx in range(sbx):
                    site = (ibt * sbt + dt) * lev.Nx + ibx * sbx + dx
                    rows.extend(range(site * lev.M, (site + 1) * lev.M))
            rows = np.array(rows)
            DB = Dcsr[rows][:, rows].toarray()
            idx.append(rows)
            color.append((ibx + ibt) % 2)
            inv.append(np.linalg.inv(DB))
    return idx, np.array(color), inv


def sap_smooth(lev: Level, blocks, r: np.ndarray, x: np.ndarray, ncycles: int) -> np.ndarray:
    """Multiplicative Schwarz, red then black blocks, exact block solves.

    Each colour phase: res = r - D x (with the x of the start of the phase),
    then x_B += D_B^{-1} res_B for every block B of that colour.
    r, x: (n, nrhs)."""
    idx, color, inv = blocks
    x = x.copy()
    for _ in range(ncycles):
        for col in (0, 1):
            res = r - lev.D @ x
            for B in np.nonzero(color == col)[0]:
                x[idx[B]] += inv[B] @ res[idx[B]]
    return x


def fgmres_fixed(D, b: np.ndarray, m: int, precond) -> np.ndarray:
    """m steps of right-preconditioned FGMRES from x0 = 0, per column of b,
    no restart, least-squares solution at step m (classical Gram-Schmidt,
    applied twice)."""
    n, nrhs = b.shape
    x = np.zeros_like(b)
    for r in range(nrhs):
        beta = np.linalg.norm(b[:, r])
        if beta == 0:
            continue
        Vb = np.zeros((n, m + 1), dtype=np.complex128)
        Z = np.zeros((n, m), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        Vb[:, 0] = b[:, r] / beta
        steps = m
        for j in range(m):
            Z[:, j] = precond(Vb[:, j:j + 1])[:, 0]
            w = D @ Z[:, j]
            h1 = Vb[:, :j + 1].conj().T @ w
            w = w - Vb[:, :j + 1] @ h1
            h2 = Vb[:, :j + 1].conj().T @ w
            w = w - Vb[:, :j + 1] @ h2
            H[:j + 1, j] = h1 + h2
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] == 0:
                steps = j + 1
                break
            Vb[:, j + 1] = w / H[j + 1, j]
        g = np.zeros(steps + 1, dtype=np.complex128)
        g[0] = beta
        y = np.linalg.lstsq(H[:steps + 1, :steps], g, rcond=None)[0]
        x[:, r] = Z[:, :steps] @ y
    return x


@dataclass
class CycleParams:
    """Per-level solver choices of the reference K-cycle."""
    sap_block: list        # (sbx, sbt) per level < L-1
    sap_cycles: list       # SAP cycles per level < L-1
    inner_iters: list      # fixed FGMRES steps for the coarse solve on levels 1..L-2


class KCycle:
    """Preconditioner M_l ~ D_l^{-1}: coarse correction then SAP post-smoothing.

    M_l(r):  x  = P_l C_{l+1}(P_l^H r)
             x  = SAP_l(r, x)                      (sap_cycles[l] red/black cycles)
    C_{L-1}  = D_{L-1}^{-1} (dense, exact)
    C_j      = inner_iters[j] steps of FGMRES on D_j preconditioned by M_j (0 < j < L-1),
               or, when inner_iters[j] == 0, one application of M_j (a V-cycle level)
    """

    def __init__(self, hier: Hierarchy, prm: CycleParams):
        self.h = hier
        self.prm = prm
        L = hier.L
        self.blocks = [sap_blocks(hier.levels[l], *prm.sap_block[l]) for l in range(L - 1)]
        self.coarse_inv = np.linalg.inv(hier.levels[L - 1].D.toarray())

    def coarse(self, l: int, rc: np.ndarray) -> np.ndarray:
        L = self.h.L
        if l == L - 1:
            return self.coarse_inv @ rc
        if self.prm.inner_iters[l] == 0:
            return self.apply(l, rc)
        return fgmres_fixed(self.h.levels[l].D, rc, self.prm.inner_iters[l],
                            lambda v: self.apply(l, v))

    def apply(self, l: int, r: np.ndarray) -> np.ndarray:
        L = self.h.L
        if l == L - 1:
            return self.coarse_inv @ r
        P = self.h.P[l]
        x = P @ self.coarse(l + 1, P.conj().T @ r)
        return sap_smooth(self.h.levels[l], self.blocks[l], r, x, self.prm.sap_cycles[l])
