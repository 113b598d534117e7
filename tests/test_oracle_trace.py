"""Pins for the oracle's trace estimators (Alg. 1, Sec. 2 variance formulas,
Hutch++ Sec. 2.4, MG-MLMC Sec. 3.1, MG-MLMC++ Alg. 2)."""
import numpy as np
import pytest

from lattice_inputs import metropolis_u1
from oracle import mg, rng
from oracle import trace as tr


@pytest.fixture(scope="module")
def small():
    th = metropolis_u1(4, 4, 3.0, 40, 51)
    h = mg.setup_hierarchy(th, 0.05, blocks=[(2, 2)], ntv=[2], seed=4)
    Dinv = np.linalg.inv(h.levels[0].D.toarray())
    return h, Dinv


def _samples(A, kind, N, seed=11, level=0):
    n = A.shape[0]
    Z = rng.noise_block(kind, seed, rng.PURPOSE_SAMPLE, level, 0, N, n)
    return np.einsum("ij,ij->j", Z.conj(), A @ Z)


def test_hutchinson_variance_formulas_and_unbiasedness(small):
    # Sec. 2: Rademacher variance 1/2 ||offdiag(A + A^T)||_F^2, Z4 (and
    # Z2xZ2 = exp(i pi/4) Z4) variance ||offdiag(A)||_F^2
    _, A = small
    off = lambda M: M - np.diag(np.diag(M))
    sig2 = {rng.RADEMACHER: 0.5 * np.linalg.norm(off(A + A.T)) ** 2,
            rng.Z2Z2: np.linalg.norm(off(A)) ** 2}
    N = 40000
    for kind, s2 in sig2.items():
        t = _samples(A, kind, N)
        assert abs(t.mean() - np.trace(A)) < 4.5 * np.sqrt(s2 / N)
        v = np.sum(np.abs(t - t.mean()) ** 2) / (N - 1)
        assert abs(v / s2 - 1) < 0.05
    # the two formulas differ for this non-symmetric A (the test can tell them apart)
    assert abs(sig2[rng.RADEMACHER] / sig2[rng.Z2Z2] - 1) > 0.05


def test_alg1_plumbing_matches_dense_samples(small):
    h, Dinv = small
    prm = tr.TraceParams(variant="hutchinson", eps=1e-2, noise=rng.Z2Z2, seed=3,
                         fixed_samples=[50])
    out = tr.estimate(h, prm)
    want = _samples(Dinv, rng.Z2Z2, 50, seed=3)
    assert np.allclose(out["samples"][0], want, rtol=1e-11, atol=1e-11)
    assert abs(out["tau"] - want.mean()) < 1e-11 * abs(want.mean())


def test_alg1_stopping_rule(small):
    h, Dinv = small
    out = tr.estimate(h, tr.TraceParams(variant="hutchinson", eps=2e-2, seed=9))
    t = np.array(out["samples"][0])
    s = len(t)
    V = lambda u: np.sum(np.abs(u - u.mean()) ** 2) / (len(u) - 1)
    assert V(t) / s <= (2e-2 * abs(t.mean())) ** 2
    u = t[:-1]
    assert s == 2 or V(u) / len(u) > (2e-2 * abs(u.mean())) ** 2


def test_hutchpp_full_rank_sketch_is_exact(small):
    # d >= rank: Q spans everything, tau_lr = tr A and every sample is 0
    h, Dinv = small
    n = Dinv.shape[0]
    Q, tau_lr = tr.low_rank(lambda X: Dinv @ X, n, n, 2, rng.Z2Z2, 5, 0)
    assert abs(tau_lr - np.trace(Dinv)) < 1e-11 * abs(np.trace(Dinv))
    lvl = tr.StochLevel(lambda X: Dinv @ X, n, n, 1.0, Q=Q)
    assert abs(tr.sample(lvl, rng.Z2Z2, 5, 0, 0)) < 1e-10


def test_hutchpp_projected_variance_formula(small):
    # the stochastic part samples zeta^H (I - QQ^H) A zeta: mean tr((I-QQ^H)A),
    # variance ||offdiag((I-QQ^H)A)||_F^2 for Z2xZ2
    h, A = small
    n = A.shape[0]
    Q, _ = tr.low_rank(lambda X: A @ X, n, 6, 2, rng.Z2Z2, 5, 0)
    M = A - Q @ (Q.conj().T @ A)
    lvl = tr.StochLevel(lambda X: A @ X, n, 6, 1.0, Q=Q)
    N = 20000
    t = np.array([tr.sample(lvl, rng.Z2Z2, 8, 0, i) for i in range(N)])
    s2 = np.linalg.norm(M - np.diag(np.diag(M))) ** 2
    assert abs(t.mean() - np.trace(M)) < 4.5 * np.sqrt(s2 / N)
    assert abs(np.var(t, ddof=1) / s2 - 1) < 0.06


def _variance_slope(make_estimator, Ns, reps):
    var = []
    for N in Ns:
        vals = [make_estimator(N, r) for r in range(reps)]
        var.append(np.var(vals, ddof=1))
    return np.polyfit(np.log(Ns), np.log(var), 1)[0]


@pytest.mark.slow
def test_variance_slopes_hutchinson_vs_hutchpp():
    # Abstract / Sec. 2.4: O(1/N) for Hutchinson, O(1/N^2) for Hutch++ with
    # d = N/3 on an HPD matrix with decaying spectrum (lambda_i = 1/i)
    n = 400
    rs = np.random.default_rng(0)
    U = np.linalg.qr(rs.standard_normal((n, n)) + 1j * rs.standard_normal((n, n)))[0]
    A = (U * (1.0 / np.arange(1, n + 1))) @ U.conj().T
    Ns = np.array([24, 48, 96, 192])

    def hutch(N, r):
        Z = rng.noise_block(rng.Z2Z2, 1000 + r, rng.PURPOSE_SAMPLE, 0, 0, N, n)
        return np.mean(np.einsum("ij,ij->j", Z.conj(), A @ Z)).real

    def hpp(N, r):
        d = N // 3
        Q, tau_lr = tr.low_rank(lambda X: A @ X, n, d, 1, rng.Z2Z2, 2000 + r, 0)
        Z = rng.noise_block(rng.Z2Z2, 2000 + r, rng.PURPOSE_SAMPLE, 0, 0, N - 2 * d, n)
        Zp = Z - Q @ (Q.conj().T @ Z)
        return (tau_lr + np.mean(np.einsum("ij,ij->j", Zp.conj(), A @ Z))).real

    s1 = _variance_slope(hutch, Ns, 150)
    s2 = _variance_slope(hpp, Ns, 150)
    assert -1.3 < s1 < -0.7
    assert s2 < -1.7


def test_mlmc_fixed_samples_equal_dense_level_samples():
    th = metropolis_u1(8, 8, 3.0, 40, 61)
    h = mg.setup_hierarchy(th, -0.05, blocks=[(2, 2), (2, 2)], ntv=[2, 2], seed=6)
    Dinv = [np.linalg.inv(lev.D.toarray()) for lev in h.levels]
    Pd = [P.toarray() for P in h.P]
    A = [Dinv[l] - Pd[l] @ Dinv[l + 1] @ Pd[l].conj().T for l in range(2)]
    prm = tr.TraceParams(variant="mlmc", fixed_samples=[30, 20], seed=4, noise=rng.Z2Z2)
    out = tr.estimate(h, prm)
    total = np.trace(Dinv[-1])
    for l in range(2):
        want = _samples(A[l], rng.Z2Z2, prm.fixed_samples[l], seed=4, level=l)
        assert np.allclose(out["samples"][l], want, rtol=1e-10, atol=1e-10)
        total += want.mean()
    assert abs(out["tau"] - total) < 1e-10 * abs(total)
    assert abs(out["tau_exact"] - np.trace(Dinv[-1])) < 1e-10 * abs(total)


def test_mlmcpp_full_and_reduced_forms_agree_with_exact_trace():
    th = metropolis_u1(8, 8, 3.0, 40, 71)
    h = mg.setup_hierarchy(th, 0.05, blocks=[(2, 2), (2, 2)], ntv=[2, 2], seed=7)
    exact = np.trace(np.linalg.inv(h.levels[0].D.toarray()))
    for form in ("reduced", "full"):
        vals = []
        for seed in range(6):
            out = tr.estimate(h, tr.TraceParams(variant="mlmcpp", form=form, eps=5e-3,
                                                d=[4, 4], k_power=2, seed=100 + seed))
            vals.append(out["tau"])
            # every run stops near its accuracy target: sum_l V_l/s_l ~ (eps |tau|)^2
            # (each level meets rho_l^2 when it stops; tau and the weights
            # move a little afterwards, so the final sum is only close to it)
            sd2 = sum(v / s for v, s in zip(out["level_var"], out["level_samples"]))
            assert sd2 <= 1.25 * (5e-3 * abs(out["tau"])) ** 2
        err = np.abs(np.array(vals) - exact) / abs(exact)
        assert np.max(err) < 4 * 5e-3


def test_optimal_vs_uniform_targets_weights():
    lv = [tr.StochLevel(None, 1, 0, 4.0, samples=[1.0, 3.0]),
          tr.StochLevel(None, 1, 0, 1.0, samples=[0.0, 4.0])]
    # V = 2 and 8; sqrt(C V) = sqrt(8), sqrt(8)
    w = tr._target_weights(lv, "optimal")
    assert np.allclose(w, [0.5, 0.5])
    assert np.allclose(tr._target_weights(lv, "uniform"), [0.5, 0.5])
    lv[1].cost = 4.0
    w = tr._target_weights(lv, "optimal")
    assert np.allclose(w, [np.sqrt(8) / (np.sqrt(8) + np.sqrt(32)), np.sqrt(32) / (np.sqrt(8) + np.sqrt(32))])


def test_two_sided_projection_mean_and_variance(small):
    # one-sided z^H A zeta samples (I - QQ^H) A, two-sided z^H A z samples
    # (I - QQ^H) A (I - QQ^H): both have mean tr((I - QQ^H) A); their Z2xZ2
    # variances are ||offdiag(M)||_F^2 of the respective M (Sec. 2)
    h, A = small
    n = A.shape[0]
    Q, _ = tr.low_rank(lambda X: A @ X, n, 5, 2, rng.Z2Z2, 5, 0)
    P = np.eye(n) - Q @ Q.conj().T
    N = 30000
    off = lambda M: M - np.diag(np.diag(M))
    for two, M in ((False, P @ A), (True, P @ A @ P)):
        lvl = tr.StochLevel(lambda X: A @ X, n, 5, 1.0, Q=Q)
        assert abs(tr.sample(lvl, rng.Z2Z2, 7, 0, 3, two_sided=two)
                   - (lambda z: np.vdot(P @ z, A @ ((P @ z) if two else z)))(
                       rng.noise_vector(rng.Z2Z2, 7, rng.PURPOSE_SAMPLE, 0, 3, n))) < 1e-12
        Z = rng.noise_block(rng.Z2Z2, 9, rng.PURPOSE_SAMPLE, 0, 0, N, n)
        t = np.einsum("ij,ij->j", Z.conj(), M @ Z)
        s2 = np.linalg.norm(off(M)) ** 2
        assert abs(t.mean() - np.trace(P @ A)) < 4.5 * np.sqrt(s2 / N)
        assert abs(np.sum(np.abs(t - t.mean()) ** 2) / (N - 1) / s2 - 1) < 0.05
    # same mean, different variances (the test can tell the two forms apart)
    assert abs(np.trace(P @ A) - np.trace(P @ A @ P)) < 1e-12 * abs(np.trace(A))
    assert abs(np.linalg.norm(off(P @ A)) / np.linalg.norm(off(P @ A @ P)) - 1) > 0.02


def test_adaptive_d_choice_rule():
    # the adaptive choice of d_l: the pilot variance and the low-rank work of
    # each candidate, recomputed here from their definitions, decide; the
    # chosen candidate minimises T(d) = W(d) + V(d) C(d) / rho^2 along the
    # doubling path up to where T first rises, and the estimate uses its Q
    th = metropolis_u1(8, 8, 3.0, 40, 81)
    h = mg.setup_hierarchy(th, -0.02, blocks=[(2, 2)], ntv=[2], seed=4)
    A = np.linalg.inv(h.levels[0].D.toarray())
    P = h.P[0].toarray()
    A = A - P @ np.linalg.inv(h.levels[1].D.toarray()) @ P.conj().T
    n = A.shape[0]
    prm = dict(variant="mlmcpp", eps=1e-2, d=[2], k_power=2, noise=rng.Z2Z2, seed=3, d_max=64, pilot=24,
               fixed_samples=[8])
    out = tr.estimate(h, tr.TraceParams(**prm))
    ca = tr.static_cost(h, 0, n, 0, 2)

    def T_of(d, rho2):
        Q, tlr = tr.low_rank(lambda X: A @ X, n, d, 2, rng.Z2Z2, 3, 0)
        Z = rng.noise_block(rng.Z2Z2, 3, rng.PURPOSE_PILOT, 0, 0, 24, n)
        t = np.einsum("ij,ij->j", (Z - Q @ (Q.conj().T @ Z)).conj(), A @ Z)
        V = np.sum(np.abs(t - t.mean()) ** 2) / 23
        return 3 * d * ca + V * (ca + 2 * n * d) / rho2, t.mean(), tlr, Q

    _, m0, lr0, _ = T_of(2, 1.0)
    tau0 = out["tau_exact"] + m0 + lr0
    rho2 = (1e-2 * abs(tau0)) ** 2
    path = [2]
    Ts = [T_of(2, rho2)[0]]
    while path[-1] * 2 <= 64:
        path.append(path[-1] * 2)
        Ts.append(T_of(path[-1], rho2)[0])
        if Ts[-1] >= Ts[-2]:
            break
    best = path[int(np.argmin(Ts))]
    assert out["level_d"] == [best]
    Qb = T_of(best, rho2)[3]
    assert np.allclose(out["Q"][0] @ out["Q"][0].conj().T, Qb @ Qb.conj().T, atol=1e-10)
    # larger d only ever lowers the pilot variance here, down to 0 at d = n
    Vs = []
    for d in (2, 8, 32, n):
        Q, _ = tr.low_rank(lambda X: A @ X, n, d, 2, rng.Z2Z2, 3, 0)
        Z = rng.noise_block(rng.Z2Z2, 3, rng.PURPOSE_PILOT, 0, 0, 24, n)
        t = np.einsum("ij,ij->j", (Z - Q @ (Q.conj().T @ Z)).conj(), A @ Z)
        Vs.append(np.sum(np.abs(t - t.mean()) ** 2) / 23)
    assert Vs[-1] < 1e-20 * Vs[0] and Vs[2] < Vs[0]
