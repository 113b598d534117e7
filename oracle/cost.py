"""The arithmetic cost model of Sec. 4 (test infrastructure).

The paper measures cost by counting the arithmetic in every matrix-vector
product the method performs -- the projections, the restrictions and
prolongations, and the smoothing iterations inside the multigrid solves --
and notes that this count is proportional to the number of non-zeros of the
matrices involved.  Alg. 2 averages the cost C_{s,l} of each stochastic sample
(the work of its projection and its level-difference application) into C_l,
which weighs the optimal target variances (eq. optimal_variance).

This module writes that count out, in complex multiply-adds, for the solver
structure the library runs (its solver choices are not in the paper; they
are described by ``SolverShape``):

* D_j y: nnz(D_j), counted structurally: 9 per fine-level row (the diagonal
  and four 2x2 hop blocks; Table 1 prints nnz(D_1) = 2.94e5 = 9 * 2 * 128^2)
  and 5 M_j^2 per coarse site (its own block and four neighbour blocks of
  M_j x M_j).  This equals the true non-zero count whenever every lattice
  extent is at least 3 (on smaller grids neighbour blocks coincide).
* R_j y = P_j^H y and P_j y: nnz(P_j) = n_j * ntv_j (each fine dof row of
  the aggregation prolongation holds the ntv_j test-vector entries of its
  aggregate and chirality).
* One red/black SAP cycle on level j: per colour, the residual of that
  colour's blocks (the rows of the blocks: half of nnz(D_j)) and one
  block-inverse product per block (K_j^2 entries, K_j dofs per block), so
  nnz(D_j) + nblk_j K_j^2 per cycle.
* A dense inverse applied to a vector: n^2 (the solver's coarsest level in
  the preconditioner; the level that closes the MLMC sum, whose solves are
  one dense product plus the residual check D_j x).
* One multigrid preconditioner application M_j on a level with a coarser
  one: R_j, the coarse correction (the dense coarsest inverse; or M_{j+1}
  for a V-cycle level; or ``inner_iters`` FGMRES steps on level j+1, each
  one M_{j+1} and one D_{j+1} product), P_j, then ``sap_cycles`` SAP cycles.
* An FGMRES(m) solve of one right-hand side to its tolerance in ``its``
  iterations: per iteration one M_j and one D_j product; per restart cycle
  the initial and the true residual (two D_j products); the number of
  cycles is ceil(its / m) (at least one).  Gram-Schmidt and the Hessenberg
  least squares are vector work, not matrix-vector products, and are not
  counted.
* The projection z = zeta - Q (Q^H zeta) of Alg. 2: 2 n_l d_l.

Reading: the paper states what the model counts but not its constants; the
constants above follow from the operators' sparsity.  The oracle solves
exactly and so has no iteration counts of its own: a parity test passes the
GPU's per-sample iteration counts through this function and replays the
resulting costs in the oracle's Alg. 2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field


@dataclass
class LevelShape:
    Nx: int
    Nt: int
    M: int                    # dofs per site
    ntv: int = 0              # test vectors per chirality to the next level (0: none)
    sap_block: tuple = (1, 1)
    sap_cycles: int = 0
    inner_iters: int = 0      # FGMRES steps of the coarse solve on this level (0: V-cycle)

    @property
    def sites(self) -> int:
        return self.Nx * self.Nt

    @property
    def n(self) -> int:
        return self.sites * self.M


@dataclass
class SolverShape:
    levels: list = field(default_factory=list)   # LevelShape per solver level
    mlmc_levels: int = 0                          # levels of the telescoping sum (0: all)
    restart: int = 16                             # outer FGMRES restart length

    @property
    def L(self) -> int:
        return len(self.levels)

    @property
    def closing(self) -> int:
        """Level whose solves use its dense inverse (closes the MLMC sum)."""
        return (self.mlmc_levels or self.L) - 1


def shape_from_blocks(Lx: int, Lt: int, blocks, ntv, sap_block, sap_cycles, inner_iters=None,
                      mlmc_levels: int = 0, restart: int = 16) -> SolverShape:
    """Solver shape of the hierarchy with aggregates ``blocks`` (one per
    coarsening step) and ``ntv`` test vectors per chirality."""
    Nx, Nt, M = Lx, Lt, 2
    levels = []
    L = len(blocks) + 1
    inner_iters = inner_iters or [0] * L
    for j in range(L):
        levels.append(LevelShape(Nx, Nt, M, ntv[j] if j < L - 1 else 0,
                                 tuple(sap_block[j]) if j < L - 1 else (1, 1),
                                 sap_cycles[j] if j < L - 1 else 0,
                                 inner_iters[j] if j < L - 1 else 0))
        if j < L - 1:
            Nx, Nt, M = Nx // blocks[j][0], Nt // blocks[j][1], 2 * ntv[j]
    return SolverShape(levels, mlmc_levels, restart)


def nnz_D(lev: LevelShape, fine: bool) -> int:
    return 9 * lev.n if fine else 5 * lev.M * lev.M * lev.sites


def nnz_P(lev: LevelShape) -> int:
    return lev.n * lev.ntv


def sap_cycle(sh: SolverShape, j: int) -> int:
    lev = sh.levels[j]
    sbx, sbt = lev.sap_block
    K = sbx * sbt * lev.M
    nblk = lev.sites // (sbx * sbt)
    return nnz_D(lev, j == 0) + nblk * K * K


def precond(sh: SolverShape, j: int) -> int:
    """One application of the multigrid preconditioner M_j."""
    lev = sh.levels[j]
    if j == sh.L - 1:
        return lev.n * lev.n
    c = j + 1
    crs = sh.levels[c]
    if c == sh.L - 1:
        coarse = crs.n * crs.n
    elif crs.inner_iters == 0:
        coarse = precond(sh, c)
    else:
        coarse = crs.inner_iters * (precond(sh, c) + nnz_D(crs, False))
    return 2 * nnz_P(lev) + coarse + lev.sap_cycles * sap_cycle(sh, j)


def solve(sh: SolverShape, j: int, its: int) -> int:
    """One right-hand side solved on level j in ``its`` FGMRES iterations."""
    lev = sh.levels[j]
    if j == sh.closing or j == sh.L - 1:
        return lev.n * lev.n + nnz_D(lev, j == 0)
    cycles = max(1, math.ceil(its / sh.restart))
    return its * (nnz_D(lev, j == 0) + precond(sh, j)) + 2 * cycles * nnz_D(lev, j == 0)


def sample(sh: SolverShape, l: int, its_fine: int, its_coarse: int, d: int, form: str = "reduced",
           variant: str = "mlmcpp") -> int:
    """C_{s,l}: the projection and the level-difference application of one
    stochastic sample (Alg. 2, the projected vector and the sample value)."""
    if variant in ("hutchinson", "hutchpp", "deflated"):
        return solve(sh, 0, its_fine) + 2 * sh.levels[0].n * d
    if form == "reduced":
        lev = sh.levels[l]
        return 2 * nnz_P(lev) + solve(sh, l, its_fine) + solve(sh, l + 1, its_coarse) + 2 * lev.n * d
    # full form: vectors live on the fine level; level j is reached through
    # j restrictions and left through j prolongations
    walk = lambda j: 2 * sum(nnz_P(sh.levels[q]) for q in range(j))
    return (walk(l) + solve(sh, l, its_fine) + walk(l + 1) + solve(sh, l + 1, its_coarse)
            + 2 * sh.levels[0].n * d)
