"""GPU parity of deflated Hutchinson (Sec. 2.2, the reference method of
Sec. 4) against the oracle on identical seeds: the subspace-iteration basis,
tr(Q^H D^{-1} Q), the Ritz exact-deflation value, per-sample values and
counts; and, with enough sweeps at a spectral gap, the exact singular
triplets from a dense SVD."""
import numpy as np
import pytest

from gpu_util import Recipe, log
from lattice_inputs import WORKLOADS, gauge_for
from oracle import deflation, rng
from oracle import trace as otr

pytestmark = pytest.mark.gpu

SOLVE_TOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    from paper_2303_11512_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def s16(ctx):
    cfg = WORKLOADS["schwinger16"]
    rec = Recipe(gauge_for(cfg), cfg["m0"], cfg["blocks"], cfg["ntv"], seed=3, sap_block=[(4, 4), (1, 1)])
    log("deflation: setup schwinger16")
    hier = rec.oracle()
    return rec.gpu(ctx), hier, hier.levels[0].D.toarray()


def _gpu(ctx, gid, **kw):
    from paper_2303_11512_amd import solve_params
    return ctx.trace_estimate(gid, variant="deflated", solve=solve_params(tol=SOLVE_TOL, restart=24),
                              max_dump=4096, **kw)


def _basis(hier, d, sweeps, noise, seed):
    g5 = hier.levels[0].chirality().astype(complex)
    return deflation.subspace_basis(hier.levels[0].solve, g5, hier.levels[0].n, d, sweeps, noise, seed)


@pytest.mark.parametrize("noise,sweeps", [("rademacher", 2), ("z2z2", 4)])
def test_deflated_replay_parity(ctx, s16, noise, sweeps):
    gid, hier, D = s16
    kw = dict(d=[8], k_power=sweeps, noise=noise, seed=6, fixed_samples=[30])
    log(f"deflated replay {noise} sweeps {sweeps}")
    got = _gpu(ctx, gid, batch=16, **kw)
    want = otr.estimate(hier, otr.TraceParams(variant="deflated", **kw))
    scale = abs(want["tau"])
    assert got["level_samples"] == want["level_samples"] == [30]
    assert abs(got["tau"] - want["tau"]) < 1e-8 * scale
    assert abs(got["level_lr"][0] - want["level_lr"][0]) < 1e-8 * scale
    ws, gs = np.array(want["samples"][0]), np.asarray(got["samples"][0])
    assert np.max(np.abs(gs - ws)) < 1e-8 * max(np.max(np.abs(ws)), scale / len(ws))
    # Ritz triplets of D on the oracle's basis
    t, sr = deflation.ritz_triplet_trace(D, want["Q"][0])
    log(f"  Ritz trace GPU {got['defl_ritz']:.10f} oracle {t:.10f}")
    assert abs(got["defl_ritz"] - t) < 1e-8 * abs(t)
    assert np.allclose(got["sigma"], sr, rtol=1e-8)


def test_deflated_adaptive_parity(ctx, s16):
    gid, hier, D = s16
    kw = dict(d=[8], k_power=3, noise="z2z2", seed=11, eps=1e-2)
    got = _gpu(ctx, gid, batch=16, **kw)
    want = otr.estimate(hier, otr.TraceParams(variant="deflated", **kw))
    assert got["level_samples"] == want["level_samples"]
    assert abs(got["tau"] - want["tau"]) < 1e-8 * abs(want["tau"])
    exact = np.trace(np.linalg.inv(D))
    assert abs(got["tau"] - exact) < 4e-2 * abs(exact)


def test_converged_basis_gives_exact_triplets(ctx, s16):
    # at the largest gap among the 10 smallest singular values, enough sweeps
    # make the basis the exact right singular subspace: the Ritz value and
    # tr(Q^H D^{-1} Q) both equal sum u_i^H v_i / sigma_i of the dense SVD
    gid, hier, D = s16
    s = np.sort(np.linalg.svd(D, compute_uv=False))
    ratios = s[1:11] / s[:10]
    k = int(np.argmax(ratios)) + 1
    sweeps = min(60, int(np.ceil(np.log(1e-12) / np.log((s[k - 1] / s[k]) ** 2))) + 2)
    log(f"deflation: k = {k} at gap {ratios[k - 1]:.3f}, {sweeps} sweeps")
    got = _gpu(ctx, gid, batch=8, d=[k], k_power=sweeps, noise="z2z2", seed=2, fixed_samples=[4])
    ref = deflation.exact_deflated_trace(D, k)
    assert abs(got["defl_ritz"] - ref) < 1e-7 * abs(ref)
    assert abs(got["level_lr"][0] - ref) < 1e-7 * abs(ref)
    assert np.allclose(got["sigma"], s[:k], rtol=1e-7)
