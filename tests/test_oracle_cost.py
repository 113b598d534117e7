"""Pins for the oracle's cost model (Sec. 4: arithmetic of every
matrix-vector product) and for two further parts of the oracle: the blocked
branch of the coarsest exact trace and the telescoping sum closed on a level
above the hierarchy's coarsest."""
import numpy as np
import pytest

from lattice_inputs import free_theta, metropolis_u1
from oracle import cost, mg, rng
from oracle import trace as tr
from test_oracle_dirac import free_trace_closed_form


# ---------------------------------------------------------------- hand counts

def test_hand_count_two_level():
    # 8x8 fine lattice (n0 = 128), 2x2 aggregates with 2 vectors -> 4x4
    # coarse sites with 4 dofs (n1 = 64, solved by its dense inverse);
    # fine SAP on 2x2-site blocks (K = 8, 16 blocks), 3 cycles; FGMRES(16).
    sh = cost.shape_from_blocks(8, 8, [(2, 2)], [2], [(2, 2)], [3], restart=16)
    # nnz(D0) = 9 * 128 = 1152; nnz(P0) = 128 * 2 = 256; dense n1^2 = 4096
    # SAP cycle = 1152 + 16 * 8^2 = 2176
    assert cost.sap_cycle(sh, 0) == 2176
    # M_0 = R + dense + P + 3 cycles = 256 + 4096 + 256 + 6528 = 11136
    assert cost.precond(sh, 0) == 11136
    # 5 iterations: 5 * (1152 + 11136) + 2 residuals * 1152 = 63744
    assert cost.solve(sh, 0, 5) == 63744
    # level 1 closes the sum: one dense product (4096) plus the residual
    # check with D1 (5 blocks of 4x4 per coarse site: 5 * 16 * 16 = 1280)
    assert cost.solve(sh, 1, 0) == 5376
    # a sample: R + solve(0) + solve(1) + P + projection 2 * 128 * 3
    assert cost.sample(sh, 0, 5, 0, 3) == 512 + 63744 + 5376 + 768


def test_hand_count_three_level_kcycle():
    # 16x16 fine (n0 = 512) -> 4x4 sites, 4 dofs (n1 = 64) -> 2x2 sites,
    # 4 dofs (n2 = 16, dense).  Fine SAP 4x4 blocks (K = 32, 16 blocks) x 2
    # cycles; level-1 SAP on single sites (K = 4, 16 blocks) x 3 cycles;
    # level 1's coarse solve is 4 inner FGMRES steps.
    sh = cost.shape_from_blocks(16, 16, [(4, 4), (2, 2)], [2, 2], [(4, 4), (1, 1)], [2, 3],
                                inner_iters=[0, 4], restart=16)
    # level 1: nnz(D1) = 1280, nnz(P1) = 64 * 2 = 128, SAP cycle 1280 + 256
    # M_1 = 128 + 16^2 + 128 + 3 * 1536 = 5120
    assert cost.precond(sh, 1) == 5120
    # M_0 = 2 * 1024 + 4 * (5120 + 1280) + 2 * (4608 + 16 * 1024) = 69632
    assert cost.precond(sh, 0) == 69632
    assert cost.solve(sh, 0, 7) == 7 * (4608 + 69632) + 2 * 4608
    # 20 iterations with restart 16 = two cycles, four residuals
    assert cost.solve(sh, 1, 20) == 20 * (1280 + 5120) + 4 * 1280
    # the coarsest level: n2^2 + nnz(D2) = 256 + 5 * 16 * 4
    assert cost.solve(sh, 2, 3) == 576
    assert cost.sample(sh, 1, 20, 1, 5) == 256 + 133120 + 576 + 640
    assert cost.sample(sh, 0, 7, 20, 5) == 2048 + 528896 + 133120 + 5120
    # full form: difference 1 walks one restriction down and back up for
    # its fine part and two for its coarse part
    assert cost.sample(sh, 1, 20, 1, 5, form="full") == (2 * 1024 + 133120 + 2 * (1024 + 128)
                                                          + 576 + 2 * 512 * 5)
    assert cost.sample(sh, 0, 7, 0, 5, variant="hutchpp") == 528896 + 5120


# ------------------------------------------- structural counts vs the matrices

@pytest.fixture(scope="module")
def hier8():
    # every lattice extent >= 3 on both levels, so neighbour blocks are distinct
    th = metropolis_u1(12, 12, 3.0, 30, 77)
    return mg.setup_hierarchy(th, 0.05, blocks=[(3, 3)], ntv=[2], seed=6)


def test_structural_nnz_matches_sparse_matrices(hier8):
    sh = cost.shape_from_blocks(12, 12, [(3, 3)], [2], [(3, 3)], [1])
    for j, lev in enumerate(hier8.levels):
        assert lev.D.nnz == cost.nnz_D(sh.levels[j], j == 0)
    assert hier8.P[0].nnz == cost.nnz_P(sh.levels[0])
    # the SAP blocks: inverse entries and the rows each colour touches
    idx, color, inv = mg.sap_blocks(hier8.levels[0], 3, 3)
    sbx, sbt = sh.levels[0].sap_block
    assert sum(b.size for b in inv) == cost.sap_cycle(sh, 0) - cost.nnz_D(sh.levels[0], True)
    rownnz = np.diff(hier8.levels[0].D.indptr)
    for col in (0, 1):
        rows = np.concatenate([idx[b] for b in np.nonzero(color == col)[0]])
        assert rownnz[rows].sum() * 2 == hier8.levels[0].D.nnz


def test_static_cost_counts_both_operators_and_projection(hier8):
    c = tr.static_cost(hier8, 0, hier8.levels[0].n, 5, 2)
    assert c == hier8.levels[0].D.nnz + hier8.levels[1].D.nnz + 2 * hier8.levels[0].n * 5
    # the last difference of a truncated sum has no coarser operator term
    assert tr.static_cost(hier8, 1, hier8.levels[1].n, 0, 2) == hier8.levels[1].D.nnz


# ---------------------------------------------------------- flops-mode replay

@pytest.fixture(scope="module")
def small3():
    th = metropolis_u1(8, 8, 3.0, 40, 55)
    return mg.setup_hierarchy(th, 0.02, blocks=[(2, 2), (2, 2)], ntv=[2, 2], seed=9)


def _run(h, **kw):
    base = dict(variant="mlmc", eps=3e-2, noise=rng.Z2Z2, seed=17)
    base.update(kw)
    return tr.estimate(h, tr.TraceParams(**base))


def test_flops_mode_with_constant_costs_equals_fixed(small3):
    costs = [[7.0] * 5000, [3.0] * 5000]
    a = _run(small3, cost="flops", sample_costs=costs)
    b = _run(small3, fixed_cost=[7.0, 3.0])
    assert a["level_samples"] == b["level_samples"]
    assert a["tau"] == b["tau"]
    assert a["level_cost"] == [7.0, 3.0]


def test_flops_mode_uses_running_mean_of_sample_costs(small3):
    rs = np.random.default_rng(3)
    costs = [list(rs.uniform(5, 9, 5000)), list(rs.uniform(1, 2, 5000))]
    a = _run(small3, cost="flops", sample_costs=costs)
    for l, s in enumerate(a["level_samples"]):
        assert a["level_cost"][l] == pytest.approx(np.mean(costs[l][:s]), rel=1e-14)
    # the optimal weights are scale-free: all costs times 1000 change nothing
    b = _run(small3, cost="flops", sample_costs=[[1000 * c for c in v] for v in costs])
    assert a["level_samples"] == b["level_samples"] and a["tau"] == b["tau"]
    # a dearer level gets relatively fewer samples (eq. accuracy_opt:
    # N_l ~ sqrt(V_l / C_l))
    c = _run(small3, cost="flops", sample_costs=[[100 * x for x in costs[0]], costs[1]])
    assert c["level_samples"][0] / c["level_samples"][1] < a["level_samples"][0] / a["level_samples"][1]


def test_flops_mode_needs_costs(small3):
    with pytest.raises(ValueError):
        _run(small3, cost="flops")
    with pytest.raises(IndexError):
        _run(small3, cost="flops", sample_costs=[[1.0], [1.0]])


# ------------------------------------------------------- coarsest exact trace

def test_coarsest_trace_blocked_branch_matches_dense_and_closed_form():
    # n = 2 * 16^2 = 512: the dense branch and the blocked sparse-LU branch
    # (ragged last block of 512 % 100 = 12 columns) agree, and on the free
    # field both give the Fourier closed form
    th = free_theta(16, 16)
    h = mg.setup_hierarchy(th, 0.3, blocks=[], ntv=[], seed=1)
    lev = h.levels[0]
    dense = mg.coarsest_trace(lev)
    blocked = mg.coarsest_trace(lev, dense_max=0, blk=100)
    ref = free_trace_closed_form(16, 16, 0.3)
    assert abs(dense - ref) < 1e-11 * abs(ref)
    assert abs(blocked - ref) < 1e-11 * abs(ref)
    # on an interacting field the two branches still agree
    th = metropolis_u1(16, 16, 3.0, 30, 61)
    lev = mg.setup_hierarchy(th, 0.05, blocks=[], ntv=[], seed=1).levels[0]
    a, b = mg.coarsest_trace(lev), mg.coarsest_trace(lev, dense_max=0, blk=64)
    assert abs(a - b) < 1e-11 * abs(a)


# ---------------------------------------------- truncated telescoping sums

@pytest.mark.parametrize("form", ["reduced", "full"])
def test_telescoping_closed_on_every_level(small3, form):
    # sum over the first T-1 differences of tr(A_l) plus tr(D_{T-1}^{-1})
    # equals tr(D^{-1}) for every closing level T (levels=T), in both forms
    exact = np.trace(np.linalg.inv(small3.levels[0].D.toarray()))
    for T in (2, 3):
        ops, tau_T = tr.level_ops(small3, "mlmc", form, levels=T)
        assert len(ops) == T - 1
        total = tau_T
        for A, n in ops:
            total += np.trace(A(np.eye(n, dtype=complex)))
        assert abs(total - exact) < 1e-11 * abs(exact), T
    # the closing trace is the exact trace of that level's operator
    _, t2 = tr.level_ops(small3, "mlmc", form, levels=2)
    assert abs(t2 - np.trace(np.linalg.inv(small3.levels[1].D.toarray()))) < 1e-11 * abs(t2)
