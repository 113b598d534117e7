"""Stochastic trace estimators for tr(D^{-1}), run step by step.

* ``hutchinson``  Alg. 1 (plain Hutchinson) on D^{-1}.
* ``hutchpp``     Hutch++ (Sec. 2.4): a block-power deflation subspace Q from
                  D^{-1} S, the low-rank part tr(Q^H D^{-1} Q) computed from
                  d solves, Hutchinson on the projected remainder.
* ``mlmc``        MG-MLMC (Sec. 3.1): Alg. 2 with d_l = 0.
* ``mlmcpp``      MG-MLMC++ (Alg. 2).
* ``deflated``    deflated Hutchinson (Sec. 2.2, the reference method of
                  Sec. 4): the deflation basis from subspace iteration on
                  D^{-1} D^{-H} (``oracle.deflation``), tr(Q^H D^{-1} Q) from
                  d solves, Hutchinson on the projected remainder.

All four share one control loop, which is Alg. 2's stochastic part; with a
single stochastic level its stopping rule reduces to Alg. 1's
V/s <= (eps tau)^2, so Alg. 1 and the Hutch++ remainder use it too.

Readings of the paper taken here:

* Level operators.  Reduced form (Sec. 3.1, eq. mlmc_dec_trace_reduced, which
  Alg. 2's remarks allow): A_l = D_l^{-1} - P_l D_{l+1}^{-1} P_l^H on vectors
  of size n_l, l = 0..L-2 (0-based).  Full form (eq. mlmc_decomp_trace, as
  Alg. 2 is printed): A_l = Ph_l D_l^{-1} Ph_l^H - Ph_{l+1} D_{l+1}^{-1}
  Ph_{l+1}^H on fine vectors, Ph_l = P_0 ... P_{l-1}, R-hat = P-hat^H.
* Coarsest level: tau_L = tr(D_{L-1}^{-1}) exactly (Sec. 3.1; with R-hat
  P-hat = I the printed sum reduces to this).
* Block power iteration: k sweeps of  Y = A_l S, Q = qr(Y), S = Q  (Alg. 2
  remarks), then tau_lr = sum_i q_i^H A_l q_i on the final Q: 2 d_l (k+1)
  solves per level.
* Eq. hutchpp_decomp is read as D^{-1} = (I - QQ^H) D^{-1} + QQ^H D^{-1}.
* Samples are one-sided as printed: z = zeta - Q (Q^H zeta),
  tau_s = z^H (A_l zeta); the two-sided z^H (A_l z) is an option (same mean,
  different variance).
* tau is complex; the accuracy tests use |tau|, the variance uses
  |tau_i - mean|^2 (Alg. 1 / Alg. 2 as printed).  No stop test before
  ``min_samples`` (>= 2) samples, since V has a 1/(s-1) factor.
* Total: tau = sum_{l<L-1} (tau_l + tau_lr_l) + tau_L (Alg. 2 Ensure + line
  summing the level means).
* Optimal targets: rho_l^2 = sqrt(C_l V_l) / sum_j sqrt(C_j V_j) * (eps |tau|)^2
  with the sum over all L-1 difference levels (inactive ones frozen);
  uniform targets: rho_l^2 = (eps |tau|)^2 / (L-1)  (Sec. 3, eqs.
  accuracy_opt / optimal_variance).  If every sqrt(C_j V_j) is 0 the weights
  fall back to uniform.
* Cost per sample C_{s,l} (Alg. 2; the cost model of Sec. 4), three modes:
  ``flops`` -- the paper's model: the arithmetic of every matrix-vector
  product of the sample (``oracle.cost``), which depends on the iteration
  counts of its two solves; the oracle solves exactly, so these per-sample
  costs are given (``sample_costs``) and C_l is their running mean, as in
  Alg. 2.  ``static`` -- one deterministic number per level, nnz(D_l) +
  nnz(D_{l+1}) + 2 n_l d_l (structural non-zeros as in ``oracle.cost``),
  i.e. one matrix-vector product per solve.  ``fixed`` -- given per-level
  constants.

Parity: pinned by tests (unbiasedness, the Rademacher / Z4 single-sample
variance formulas of Sec. 2, the 1/N vs 1/N^2 slopes, telescoping, the
d >= rank and square-P special cases).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from . import cost as cmodel
from . import deflation
from . import rng
from .mg import Hierarchy, coarsest_trace


@dataclass
class TraceParams:
    variant: str = "mlmcpp"            # hutchinson | hutchpp | mlmc | mlmcpp
    form: str = "reduced"              # reduced | full
    eps: float = 1e-2
    d: list = field(default_factory=list)   # Hutch++ vectors per stochastic level
    k_power: int = 2
    noise: str = rng.Z2Z2
    targets: str = "optimal"           # optimal | uniform
    cost: str = "static"               # static | fixed | flops
    fixed_cost: Optional[list] = None  # per stochastic level (implies cost="fixed")
    sample_costs: Optional[list] = None  # flops mode: C_{s,l} per level, per sample index
    min_samples: int = 2
    max_samples: int = 1_000_000
    fixed_samples: Optional[list] = None   # replay mode: exact sample counts
    seed: int = 1
    levels: int = 0                    # hierarchy levels used by the MLMC variants (0 = all)
    projection: str = "one-sided"      # one-sided (Alg. 2 as printed) | two-sided
    d_max: int = 0                     # > 0: adaptive d_l, candidates d[l] * 2^j <= d_max
    pilot: int = 16                    # pilot samples per candidate (adaptive d_l)


@dataclass
class StochLevel:
    apply: Callable[[np.ndarray], np.ndarray]
    n: int
    d: int
    cost: float
    Q: Optional[np.ndarray] = None
    tau_lr: complex = 0.0
    samples: list = field(default_factory=list)
    active: bool = True
    sample_costs: Optional[list] = None   # given C_{s,l} (flops mode)
    cost_sum: float = 0.0

    @property
    def s(self) -> int:
        return len(self.samples)

    def mean(self) -> complex:
        return complex(np.mean(self.samples)) if self.samples else 0.0

    def var(self) -> float:
        if len(self.samples) < 2:
            return float("nan")
        t = np.asarray(self.samples)
        return float(np.sum(np.abs(t - t.mean()) ** 2) / (len(t) - 1))


def static_cost(hier: Hierarchy, l: int, n: int, d: int, L: int) -> float:
    """nnz(D_l) + nnz(D_{l+1}) + 2 n d: one product with each operator of
    the difference and the projection (structural non-zeros)."""
    def nnz(j):
        lev = hier.levels[j]
        return cmodel.nnz_D(cmodel.LevelShape(lev.Nx, lev.Nt, lev.M), j == 0)
    c = nnz(l) + 2 * n * d
    if l + 1 < L:
        c += nnz(l + 1)
    return float(c)


def level_ops(hier: Hierarchy, variant: str, form: str, levels: int = 0):
    """List of (apply_A, n) for the stochastic levels and the exact part.

    ``levels`` < hier.L closes the telescoping sum at level ``levels - 1``:
    the coarser levels of the hierarchy then only serve the solver."""
    L = levels if levels else hier.L
    if variant in ("hutchinson", "hutchpp", "deflated"):
        lev0 = hier.levels[0]
        return [(lev0.solve, lev0.n)], 0.0
    if L < 2:
        raise ValueError("MLMC needs at least two levels")
    ops = []
    if form == "reduced":
        for l in range(L - 1):
            fine, P = hier.levels[l], hier.P[l]
            coarse = hier.levels[l + 1]

            def A(X, fine=fine, coarse=coarse, P=P):
                return fine.solve(X) - P @ coarse.solve(P.conj().T @ X)
            ops.append((A, fine.n))
    elif form == "full":
        Phat = [None]
        acc = None
        for l in range(L - 1):
            acc = hier.P[l] if acc is None else acc @ hier.P[l]
            Phat.append(acc.tocsr())

        def lift(l, X):
            return X if l == 0 else Phat[l] @ hier.levels[l].solve(Phat[l].conj().T @ X)
        for l in range(L - 1):
            def A(X, l=l):
                X0 = hier.levels[0].solve(X) if l == 0 else lift(l, X)
                return X0 - lift(l + 1, X)
            ops.append((A, hier.levels[0].n))
    else:
        raise ValueError(form)
    return ops, coarsest_trace(hier.levels[L - 1])


def low_rank(A, n: int, d: int, k: int, noise: str, seed: int, level: int):
    """Block power iteration (k sweeps) and tau_lr = tr(Q^H A Q)."""
    S = rng.noise_block(noise, seed, rng.PURPOSE_SKETCH, level, 0, d, n)
    Q = None
    for _ in range(k):
        Y = A(S)
        Q, _ = np.linalg.qr(Y, mode="reduced")
        S = Q
    tau_lr = complex(np.trace(Q.conj().T @ A(Q)))
    return Q, tau_lr


def sample(lvl: StochLevel, noise: str, seed: int, level: int, index: int, two_sided: bool = False) -> complex:
    """tau_{s,l} = z^H (A_l zeta), z = zeta - Q (Q^H zeta): Alg. 2's projected
    vector and sample value, one-sided as printed.  ``two_sided``:
    tau_{s,l} = z^H (A_l z), Hutchinson on (I - QQ^H) A_l (I - QQ^H), which
    has the same mean tr((I - QQ^H) A_l) and another variance."""
    zeta = rng.noise_vector(noise, seed, rng.PURPOSE_SAMPLE, level, index, lvl.n)
    z = zeta if lvl.Q is None else zeta - lvl.Q @ (lvl.Q.conj().T @ zeta)
    x = lvl.apply((z if two_sided else zeta)[:, None])[:, 0]
    return complex(np.vdot(z, x))


def estimate(hier: Hierarchy, prm: TraceParams) -> dict:
    ops, tau_exact = level_ops(hier, prm.variant, prm.form, prm.levels)
    nl = len(ops)
    use_lr = prm.variant in ("hutchpp", "mlmcpp", "deflated")
    mode = "fixed" if prm.fixed_cost is not None else prm.cost
    if mode not in ("static", "fixed", "flops"):
        raise ValueError(prm.cost)
    if mode == "flops" and prm.sample_costs is None:
        raise ValueError("cost='flops' needs the per-sample costs (sample_costs)")
    levels = []
    for l, (A, n) in enumerate(ops):
        d = prm.d[l] if use_lr else 0
        if mode == "fixed":
            cost = float(prm.fixed_cost[l])
        elif mode == "static":
            cost = static_cost(hier, l, n, d, prm.levels or hier.L)
        else:
            cost = float("nan")   # C_l: the mean of the costs of the samples taken
        levels.append(StochLevel(A, n, d, cost,
                                 sample_costs=prm.sample_costs[l] if mode == "flops" else None))

    # deflation vectors and low-rank parts (Alg. 2, first loop)
    chosen = None
    if use_lr and prm.d_max > 0 and prm.variant in ("hutchpp", "mlmcpp"):
        chosen = _adaptive_d(hier, levels, prm, tau_exact, mode)
    for l, lv in enumerate(levels):
        if chosen is not None:
            pass  # Q and tau_lr set by the adaptive choice
        elif lv.d > 0 and prm.variant == "deflated":
            g5 = hier.levels[0].chirality().astype(np.complex128)
            lv.Q = deflation.subspace_basis(lv.apply, g5, lv.n, lv.d, max(1, prm.k_power), prm.noise, prm.seed)
            lv.tau_lr = complex(np.trace(lv.Q.conj().T @ lv.apply(lv.Q)))
        elif lv.d > 0:
            lv.Q, lv.tau_lr = low_rank(lv.apply, lv.n, lv.d, prm.k_power, prm.noise, prm.seed, l)

    # stochastic part (Alg. 2, second loop)
    s = 0
    tau = 0.0
    while any(lv.active for lv in levels):
        s += 1
        for l, lv in enumerate(levels):
            if lv.active:
                lv.samples.append(sample(lv, prm.noise, prm.seed, l, s - 1,
                                         two_sided=prm.projection == "two-sided"))
                if lv.sample_costs is not None:
                    if s - 1 >= len(lv.sample_costs):
                        raise IndexError(f"no cost given for sample {s - 1} of level {l}")
                    lv.cost_sum += lv.sample_costs[s - 1]
                    lv.cost = lv.cost_sum / lv.s
        tau = sum(lv.mean() + lv.tau_lr for lv in levels) + tau_exact
        if prm.fixed_samples is not None:
            for l, lv in enumerate(levels):
                if lv.s >= prm.fixed_samples[l]:
                    lv.active = False
            continue
        weights = _target_weights(levels, prm.targets)
        for l, lv in enumerate(levels):
            if not lv.active:
                continue
            if lv.s >= prm.max_samples:
                lv.active = False
                continue
            if lv.s < max(2, prm.min_samples):
                continue
            rho2 = weights[l] * (prm.eps * abs(tau)) ** 2
            if lv.var() / lv.s <= rho2:
                lv.active = False

    return dict(
        tau=complex(tau),
        tau_exact=complex(tau_exact),
        level_d=[lv.d for lv in levels],
        level_mean=[lv.mean() for lv in levels],
        level_lr=[lv.tau_lr for lv in levels],
        level_var=[lv.var() for lv in levels],
        level_cost=[lv.cost for lv in levels],
        level_samples=[lv.s for lv in levels],
        samples=[list(lv.samples) for lv in levels],
        Q=[lv.Q for lv in levels],
    )


def _adaptive_d(hier: Hierarchy, levels: list, prm: TraceParams, tau_exact, mode: str) -> list:
    """Adaptive number of deflation vectors per level difference (the choice
    of d_l is left open by the paper, Sec. 5; adaptive Hutch++ is cited in
    Sec. 2.4).  Candidates d = d_l, 2 d_l, 4 d_l, ... <= d_max.  For each,
    the block power iteration gives Q_d and tau_lr(d); ``pilot`` samples of
    the projected remainder (noise purpose PILOT, the same vectors for every
    candidate, discarded afterwards) give its variance V(d); the predicted
    cost of the level is T(d) = W_lr(d) + V(d) C(d) / rho^2 with the
    per-sample cost C(d), the low-rank work W_lr(d) = (k+1) d C_A (C_A: one
    application of A_l) and rho^2 = (eps |tau0|)^2 / (number of differences),
    tau0 the estimate from the first candidates' pilot means.  The doubling
    stops at the first candidate that does not lower T; the best Q and
    tau_lr are kept.  Costs: the static or fixed model (the flops model needs
    the GPU's iteration counts).  Parity unpinned with respect to the paper:
    this rule is a reading of "how to choose d" left open there; it is
    pinned only by its own definition and the d = n special case."""
    if mode == "flops":
        raise ValueError("adaptive d_l in the oracle needs cost='static' or 'fixed'")
    L = prm.levels or hier.L
    nl = len(levels)
    kp = max(1, prm.k_power)

    def cost_apply(l, lv):
        return float(prm.fixed_cost[l]) if mode == "fixed" else static_cost(hier, l, lv.n, 0, L)

    def candidate(l, lv, d):
        Q, tau_lr = low_rank(lv.apply, lv.n, d, prm.k_power, prm.noise, prm.seed, l)
        Z = rng.noise_block(prm.noise, prm.seed, rng.PURPOSE_PILOT, l, 0, prm.pilot, lv.n)
        two = prm.projection == "two-sided"
        Zp = Z - Q @ (Q.conj().T @ Z)
        X = lv.apply(Zp if two else Z)
        t = np.einsum("ij,ij->j", Zp.conj(), X)
        V = float(np.sum(np.abs(t - t.mean()) ** 2) / (len(t) - 1))
        ca = cost_apply(l, lv)
        return dict(d=d, Q=Q, tau_lr=tau_lr, V=V, mean=complex(t.mean()),
                    C=ca + (0.0 if mode == "fixed" else 2.0 * lv.n * d), W=(kp + 1) * d * ca)

    cur = [candidate(l, lv, lv.d) for l, lv in enumerate(levels)]
    tau0 = tau_exact + sum(c["mean"] + c["tau_lr"] for c in cur)
    rho2 = (prm.eps * abs(tau0)) ** 2 / nl
    T = lambda c: c["W"] + c["V"] * c["C"] / rho2
    chosen = []
    for l, lv in enumerate(levels):
        best = cur[l]
        d = best["d"]
        while 2 * d <= prm.d_max:
            d *= 2
            trial = candidate(l, lv, d)
            if T(trial) < T(best):
                best = trial
            else:
                break
        lv.d, lv.Q, lv.tau_lr = best["d"], best["Q"], best["tau_lr"]
        if mode != "fixed":
            lv.cost = static_cost(hier, l, lv.n, lv.d, L)
        chosen.append(best["d"])
    return chosen


def _target_weights(levels, targets: str) -> list:
    nl = len(levels)
    if targets == "uniform":
        return [1.0 / nl] * nl
    if targets != "optimal":
        raise ValueError(targets)
    cv = [np.sqrt(lv.cost * lv.var()) if lv.s >= 2 else 0.0 for lv in levels]
    tot = float(np.sum(cv))
    if not np.isfinite(tot) or tot == 0.0:
        return [1.0 / nl] * nl
    return [c / tot for c in cv]
