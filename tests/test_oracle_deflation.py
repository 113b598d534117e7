"""Pins for the deflated-Hutchinson oracle (Sec. 2.1-2.3): exact deflation
by singular triplets, the subspace iteration that approximates them, and the
estimator on the projected remainder."""
import numpy as np
import pytest

from lattice_inputs import metropolis_u1
from oracle import deflation, mg, rng
from oracle import trace as tr


@pytest.fixture(scope="module")
def op():
    th = metropolis_u1(8, 8, 3.0, 40, 71)
    h = mg.setup_hierarchy(th, -0.02, blocks=[], ntv=[], seed=1)
    D = h.levels[0].D.toarray()
    return h, D, np.linalg.inv(D)


def test_full_deflation_is_exact(op):
    # k = n: Pi = I, the deflated part is the whole trace, the remainder 0
    h, D, Dinv = op
    n = D.shape[0]
    assert abs(deflation.exact_deflated_trace(D, n) - np.trace(Dinv)) < 1e-10 * abs(np.trace(Dinv))
    _, _, V = deflation.exact_triplets(D, n)
    lvl = tr.StochLevel(lambda X: Dinv @ X, n, n, 1.0, Q=V)
    assert abs(tr.sample(lvl, rng.Z2Z2, 3, 0, 0)) < 1e-10


def test_deflation_removes_smallest_singular_values_from_frobenius_norm(op):
    # ||(I - V_k V_k^H) D^{-1}||_F^2 = sum_{i > k} sigma_i^{-2} (Sec. 2.1),
    # less than for any other rank-k orthogonal projector
    h, D, Dinv = op
    n = D.shape[0]
    s = np.sort(np.linalg.svd(D, compute_uv=False))
    for k in (1, 5, 20):
        _, _, V = deflation.exact_triplets(D, k)
        M = Dinv - V @ (V.conj().T @ Dinv)
        assert abs(np.linalg.norm(M) ** 2 - np.sum(s[k:] ** -2.0)) < 1e-9 * np.sum(s ** -2.0)
        R = np.linalg.qr(np.random.default_rng(k).standard_normal((n, k)) + 0j)[0]
        assert np.linalg.norm(Dinv - R @ (R.conj().T @ Dinv)) > np.linalg.norm(M)


def test_exact_deflation_trace_identity(op):
    # tr(Pi D^{-1}) = tr(V^H D^{-1} V) = sum u_i^H v_i / sigma_i (Sec. 2.2)
    h, D, Dinv = op
    for k in (1, 7, 30):
        _, _, V = deflation.exact_triplets(D, k)
        a = np.trace(V.conj().T @ Dinv @ V)
        b = deflation.exact_deflated_trace(D, k)
        assert abs(a - b) < 1e-10 * max(1.0, abs(a))


def test_gamma5_gives_the_adjoint_inverse(op):
    h, D, Dinv = op
    g5 = h.levels[0].chirality()
    assert np.allclose(g5[:, None] * Dinv * g5[None, :], Dinv.conj().T, atol=1e-12)


def test_subspace_iteration_converges_to_singular_subspace(op):
    # at a gap of the singular spectrum the iterated basis spans the exact
    # right singular subspace, and its Ritz triplets give the exact trace
    h, D, Dinv = op
    s = np.sort(np.linalg.svd(D, compute_uv=False))
    ratios = s[1:11] / s[:10]
    k = int(np.argmax(ratios)) + 1          # gap between sigma_k and sigma_{k+1}
    sweeps = int(np.ceil(np.log(1e-12) / np.log((s[k - 1] / s[k]) ** 2))) + 2
    g5 = h.levels[0].chirality().astype(complex)
    Q = deflation.subspace_basis(lambda X: np.linalg.solve(D, X), g5, D.shape[0], k, sweeps, rng.Z2Z2, 9)
    _, _, V = deflation.exact_triplets(D, k)
    assert np.linalg.norm(Q @ Q.conj().T - V @ V.conj().T, 2) < 1e-6
    t, sr = deflation.ritz_triplet_trace(D, Q)
    assert np.allclose(sr, s[:k], rtol=1e-8)
    ref = deflation.exact_deflated_trace(D, k)
    assert abs(t - ref) < 1e-8 * abs(ref)
    # and with one sweep the basis is only approximate, yet the split through
    # tr(Q^H D^{-1} Q) stays exact (Sec. 2.3)
    Q1 = deflation.subspace_basis(lambda X: np.linalg.solve(D, X), g5, D.shape[0], k, 1, rng.Z2Z2, 9)
    M = Dinv - Q1 @ (Q1.conj().T @ Dinv)
    assert abs(np.trace(M) + np.trace(Q1.conj().T @ Dinv @ Q1) - np.trace(Dinv)) < 1e-10 * abs(np.trace(Dinv))


def test_deflated_estimator_plumbing_and_variance(op):
    h, D, Dinv = op
    k, sweeps = 6, 3
    out = tr.estimate(h, tr.TraceParams(variant="deflated", d=[k], k_power=sweeps, noise=rng.Z2Z2, seed=4,
                                        fixed_samples=[40]))
    g5 = h.levels[0].chirality().astype(complex)
    Q = deflation.subspace_basis(lambda X: Dinv @ X, g5, D.shape[0], k, sweeps, rng.Z2Z2, 4)
    assert np.allclose(out["Q"][0] @ out["Q"][0].conj().T, Q @ Q.conj().T, atol=1e-10)
    assert abs(out["level_lr"][0] - np.trace(Q.conj().T @ Dinv @ Q)) < 1e-10 * abs(np.trace(Dinv))
    Z = rng.noise_block(rng.Z2Z2, 4, rng.PURPOSE_SAMPLE, 0, 0, 40, D.shape[0])
    want = np.einsum("ij,ij->j", (Z - Q @ (Q.conj().T @ Z)).conj(), Dinv @ Z)
    assert np.allclose(out["samples"][0], want, rtol=1e-10, atol=1e-10)
    # remainder variance: ||offdiag((I - QQ^H) D^{-1})||_F^2 for Z2xZ2 noise,
    # and the estimator is unbiased
    M = Dinv - Q @ (Q.conj().T @ Dinv)
    sig2 = np.linalg.norm(M - np.diag(np.diag(M))) ** 2
    N = 20000
    Z = rng.noise_block(rng.Z2Z2, 8, rng.PURPOSE_SAMPLE, 0, 0, N, D.shape[0])
    t = np.einsum("ij,ij->j", (Z - Q @ (Q.conj().T @ Z)).conj(), Dinv @ Z)
    assert abs(t.mean() - np.trace(M)) < 4.5 * np.sqrt(sig2 / N)
    assert abs(np.sum(np.abs(t - t.mean()) ** 2) / (N - 1) / sig2 - 1) < 0.05
    # adaptive: within 4 sigma of the exact trace
    est = tr.estimate(h, tr.TraceParams(variant="deflated", d=[k], k_power=sweeps, eps=1e-2, noise=rng.Z2Z2, seed=5))
    exact = np.trace(Dinv)
    assert abs(est["tau"] - exact) < 4e-2 * abs(exact)
