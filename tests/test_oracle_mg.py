"""Pins for the oracle's multigrid hierarchy (Sec. 3.1) and its reference
preconditioner."""
import numpy as np
import pytest

from conftest import read_golden
from lattice_inputs import free_theta, metropolis_u1
from oracle import mg


@pytest.fixture(scope="module")
def hier3():
    th = metropolis_u1(8, 8, 3.0, 50, 31)
    return mg.setup_hierarchy(th, -0.05, blocks=[(2, 2), (2, 2)], ntv=[2, 2], seed=5)


def test_qr_plus_is_unique_normalisation():
    rs = np.random.default_rng(0)
    A = rs.standard_normal((20, 5)) + 1j * rs.standard_normal((20, 5))
    Q = mg.qr_plus(A)
    R = Q.conj().T @ A
    assert np.allclose(Q.conj().T @ Q, np.eye(5), atol=1e-13)
    assert np.allclose(np.tril(R, -1), 0, atol=1e-13)
    assert np.all(np.abs(np.diag(R).imag) < 1e-13) and np.all(np.diag(R).real > 0)
    # unique: a column-phase change of the input does not change Q up to that phase
    ph = np.exp(1j * rs.uniform(0, 2 * np.pi, 5))
    assert np.allclose(mg.qr_plus(A * ph[None, :]), Q * ph[None, :], atol=1e-12)


def test_orthonormal_prolongations(hier3):
    for P in hier3.P:
        assert np.allclose((P.conj().T @ P).toarray(), np.eye(P.shape[1]), atol=1e-13)


def test_coarse_chirality_and_gamma5_hermiticity(hier3):
    # P^H sigma_3 P is diagonal +-1 (aggregates split the chirality) and the
    # Galerkin operators stay gamma5-hermitian: D_c^H = s3c D_c s3c.
    for l, P in enumerate(hier3.P):
        fine = hier3.levels[l]
        s3 = np.diag(fine.chirality())
        s3c = P.conj().T @ (s3 @ P.toarray())
        coarse = hier3.levels[l + 1]
        assert np.allclose(s3c, np.diag(coarse.chirality()), atol=1e-13)
        Dc = coarse.D.toarray()
        S = np.diag(coarse.chirality())
        assert np.allclose(Dc.conj().T, S @ Dc @ S, atol=1e-13)


def test_galerkin_coarse_sizes_match_table1():
    # Table 1: n_l = 2*128^2, 4*32^2, 8*8^2, 8*2^2 -- 4x4 aggregates with
    # 2, 4, 4 test vectors per chirality.
    vals = dict(ln.split() for ln in read_golden("table1_sizes.txt"))
    th = free_theta(128, 128)
    h = mg.setup_hierarchy(th, 0.5, blocks=[(4, 4), (4, 4), (4, 4)], ntv=[2, 4, 4], seed=1,
                           setup_iters=1)
    assert [lev.n for lev in h.levels] == [int(vals[k]) for k in ("n1", "n2", "n3", "n4")]


def test_telescoping_reduced_form(hier3):
    # sum_l tr(D_l^{-1} - P_l D_{l+1}^{-1} P_l^H) + tr(D_L^{-1}) = tr(D^{-1}),
    # each level difference is real (eq. mlmc_dec_trace_reduced)
    Dinv = [np.linalg.inv(lev.D.toarray()) for lev in hier3.levels]
    total = 0.0
    for l, P in enumerate(hier3.P):
        Pd = P.toarray()
        term = np.trace(Dinv[l] - Pd @ Dinv[l + 1] @ Pd.conj().T)
        assert abs(term.imag) < 1e-10 * max(1.0, abs(term))
        total += term
    total += np.trace(Dinv[-1])
    ref = np.trace(Dinv[0])
    assert abs(total - ref) < 1e-12 * abs(ref)
    assert abs(mg.coarsest_trace(hier3.levels[-1]) - np.trace(Dinv[-1])) < 1e-12 * abs(ref)


def test_level_difference_invariant_under_aggregate_unitaries(hier3):
    rs = np.random.default_rng(3)
    P = hier3.P[0].toarray()
    nc = P.shape[1]
    ntv = 2
    W = np.zeros((nc, nc), dtype=complex)
    for b in range(nc // ntv):
        X = rs.standard_normal((ntv, ntv)) + 1j * rs.standard_normal((ntv, ntv))
        W[b * ntv:(b + 1) * ntv, b * ntv:(b + 1) * ntv] = np.linalg.qr(X)[0]
    D = hier3.levels[0].D.toarray()
    A1 = np.linalg.inv(D) - P @ np.linalg.inv(P.conj().T @ D @ P) @ P.conj().T
    P2 = P @ W
    A2 = np.linalg.inv(D) - P2 @ np.linalg.inv(P2.conj().T @ D @ P2) @ P2.conj().T
    assert np.allclose(A1, A2, atol=1e-11)


def test_square_prolongation_gives_zero_difference():
    # 1x1 aggregates with one test vector per spin: P is square and unitary,
    # so A_0 = D^{-1} - P (P^H D P)^{-1} P^H vanishes.
    th = metropolis_u1(4, 4, 3.0, 20, 41)
    h = mg.setup_hierarchy(th, 0.1, blocks=[(1, 1)], ntv=[1], seed=2)
    P = h.P[0].toarray()
    assert P.shape[0] == P.shape[1]
    D = h.levels[0].D.toarray()
    A0 = np.linalg.inv(D) - P @ np.linalg.inv(h.levels[1].D.toarray()) @ P.conj().T
    assert np.max(np.abs(A0)) < 1e-12


def test_setup_is_deterministic(hier3):
    th = metropolis_u1(8, 8, 3.0, 50, 31)
    h2 = mg.setup_hierarchy(th, -0.05, blocks=[(2, 2), (2, 2)], ntv=[2, 2], seed=5)
    for a, b in zip(hier3.Pb, h2.Pb):
        assert np.array_equal(a, b)


def test_test_vectors_capture_low_modes(hier3):
    # after inverse iteration the span of V holds much of the smallest
    # singular vectors' energy: ||D V|| per column is small vs a random vector
    lev = hier3.levels[0]
    V = hier3.V[0]
    rs = np.random.default_rng(1)
    Rn = mg.qr_plus(rs.standard_normal(V.shape) + 1j * rs.standard_normal(V.shape))
    assert np.linalg.norm(lev.D @ V) < 0.5 * np.linalg.norm(lev.D @ Rn)


# --- reference preconditioner (solver choice; pinned by special cases) ---

def test_sap_single_block_is_exact_inverse():
    th = metropolis_u1(4, 4, 3.0, 20, 5)
    h = mg.setup_hierarchy(th, 0.1, blocks=[(2, 2)], ntv=[2], seed=3)
    lev = h.levels[0]
    blocks = mg.sap_blocks(lev, 4, 4)
    r = np.random.default_rng(2).standard_normal((lev.n, 2)) + 0j
    x = mg.sap_smooth(lev, blocks, r, np.zeros_like(r), 1)
    assert np.allclose(lev.D @ x, r, atol=1e-12)


def test_sap_converges_as_stationary_iteration():
    th = metropolis_u1(8, 8, 3.0, 20, 5)
    h = mg.setup_hierarchy(th, 0.8, blocks=[(2, 2)], ntv=[2], seed=3)
    lev = h.levels[0]
    blocks = mg.sap_blocks(lev, 2, 2)
    r = np.random.default_rng(2).standard_normal((lev.n, 1)) + 0j
    x = mg.sap_smooth(lev, blocks, r, np.zeros_like(r), 60)
    assert np.linalg.norm(r - lev.D @ x) < 1e-10 * np.linalg.norm(r)


def test_fgmres_fixed_full_dimension_is_exact():
    rs = np.random.default_rng(4)
    n = 12
    D = np.eye(n) * 3 + rs.standard_normal((n, n)) + 1j * rs.standard_normal((n, n))
    b = rs.standard_normal((n, 2)) + 0j
    x = mg.fgmres_fixed(D, b, n, lambda v: v)
    assert np.allclose(D @ x, b, atol=1e-10)


def test_kcycle_special_cases(hier3):
    L = hier3.L
    rs = np.random.default_rng(8)
    r = rs.standard_normal((hier3.levels[0].n, 2)) + 1j * rs.standard_normal((hier3.levels[0].n, 2))
    # no fine smoothing + a full-dimension inner FGMRES (whose own
    # preconditioner is non-singular) = exact two-grid coarse correction
    n1 = hier3.levels[1].n
    kc = mg.KCycle(hier3, mg.CycleParams(sap_block=[(2, 2), (1, 1)], sap_cycles=[0, 1],
                                         inner_iters=[0, n1]))
    P0 = hier3.P[0].toarray()
    want = P0 @ np.linalg.solve(hier3.levels[1].D.toarray(), P0.conj().T @ r)
    assert np.allclose(kc.apply(0, r), want, atol=1e-10)
    # with smoothing: x = P e, then SAP on the residual equation
    kc2 = mg.KCycle(hier3, mg.CycleParams(sap_block=[(2, 2), (1, 1)], sap_cycles=[2, 1],
                                          inner_iters=[0, 3]))
    y = kc2.apply(0, r)
    x0 = hier3.P[0] @ kc2.coarse(1, hier3.P[0].conj().T @ r)
    assert np.allclose(y, mg.sap_smooth(hier3.levels[0], kc2.blocks[0], r, x0, 2), atol=1e-12)
    # the preconditioner improves on the unpreconditioned residual
    D = hier3.levels[0].D
    assert np.linalg.norm(r - D @ y) < 0.5 * np.linalg.norm(r)
