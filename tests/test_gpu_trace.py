"""GPU parity of the trace estimators (Alg. 1, Hutch++, MG-MLMC, MG-MLMC++
Alg. 2) against the oracle on identical seeds: per-sample values, the
low-rank parts, sample counts and the final estimate (1e-8 relative)."""
import numpy as np
import pytest

from gpu_util import Recipe, log
from lattice_inputs import WORKLOADS, gauge_for, metropolis_u1
from oracle import trace as otr

pytestmark = pytest.mark.gpu

SOLVE_TOL = 1e-12  # tight solves so that solver error stays far below 1e-8


@pytest.fixture(scope="module")
def ctx():
    from paper_2303_11512_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def s16(ctx):
    """The 16x16 plain-method workload: beta 3.0 Metropolis field, m0 = -0.05,
    4x4 aggregates with 4 test vectors per chirality, Rademacher noise."""
    cfg = WORKLOADS["schwinger16"]
    th = gauge_for(cfg)
    rec = Recipe(th, cfg["m0"], cfg["blocks"], cfg["ntv"], seed=3, sap_block=[(4, 4), (1, 1)])
    log("setup schwinger16")
    return cfg, rec, rec.gpu(ctx), rec.oracle()


@pytest.fixture(scope="module")
def s32(ctx):
    th = metropolis_u1(32, 32, 3.0, 100, 932)
    rec = Recipe(th, -0.08, [(4, 4), (2, 2)], [8, 8], seed=11,
                 sap_block=[(4, 4), (1, 1), (1, 1)], inner_iters=[4, 4, 4])
    log("setup s32")
    return rec, rec.gpu(ctx), rec.oracle()


def _gpu(ctx, gid, **kw):
    from paper_2303_11512_amd import solve_params
    return ctx.trace_estimate(gid, solve=solve_params(tol=SOLVE_TOL, restart=24), max_dump=4096,
                              **kw)


def _cmp(got, want, tol=1e-8):
    scale = max(abs(want["tau"]), 1e-300)
    assert abs(got["tau"] - want["tau"]) < tol * scale, (got["tau"], want["tau"])
    for l in range(len(want["level_samples"])):
        assert got["level_samples"][l] == want["level_samples"][l]
        ws = np.array(want["samples"][l])
        gs = got["samples"][l]
        # samples are differences of two solves: compare on the scale of the level
        sc = max(np.max(np.abs(ws)), 1e-300)
        assert np.max(np.abs(gs - ws)) < tol * max(sc, scale / max(1, len(ws))), l
        assert abs(got["level_lr"][l] - want["level_lr"][l]) < tol * scale


@pytest.mark.parametrize("variant,form", [("hutchinson", "reduced"), ("hutchpp", "reduced"),
                                          ("mlmc", "reduced"), ("mlmcpp", "reduced"),
                                          ("mlmcpp", "full")])
def test_replay_parity_s16(ctx, s16, variant, form):
    cfg, rec, gid, hier = s16
    log(f"trace replay {variant}/{form}")
    fixed = [37]
    kw = dict(variant=variant, form=form, eps=cfg["eps"], d=[cfg["d"][0]], k_power=2,
              noise="rademacher", seed=cfg["trace_seed"], fixed_samples=fixed)
    got = _gpu(ctx, gid, batch=16, **kw)
    want = otr.estimate(hier, otr.TraceParams(**kw))
    _cmp(got, want)


def test_adaptive_parity_s16(ctx, s16):
    """The full plain-method workload: Hutch++ (8 vectors) + MG-MLMC,
    Rademacher noise, rel. accuracy 1e-2, optimal targets."""
    cfg, rec, gid, hier = s16
    kw = dict(variant="mlmcpp", form="reduced", eps=cfg["eps"], d=[cfg["d"][0]], k_power=2,
              noise="rademacher", seed=cfg["trace_seed"])
    got = _gpu(ctx, gid, batch=8, **kw)
    want = otr.estimate(hier, otr.TraceParams(**kw))
    _cmp(got, want)
    # and the estimate is within 4 sigma (sigma = eps |tau|) of the exact trace
    exact = np.trace(np.linalg.inv(hier.levels[0].D.toarray()))
    assert abs(got["tau"] - exact) < 4 * cfg["eps"] * abs(exact)


@pytest.mark.parametrize("batch", [3, 64])
def test_batching_does_not_change_result(ctx, s16, batch):
    cfg, rec, gid, hier = s16
    kw = dict(variant="mlmcpp", eps=3e-2, d=[4], k_power=1, noise="z2z2", seed=5)
    a = _gpu(ctx, gid, batch=batch, **kw)
    b = _gpu(ctx, gid, batch=1, **kw)
    assert a["level_samples"] == b["level_samples"]
    assert abs(a["tau"] - b["tau"]) < 1e-12 * abs(b["tau"])


def test_three_level_mlmcpp_parity(ctx, s32):
    rec, gid, hier = s32
    for targets in ("optimal", "uniform"):
        kw = dict(variant="mlmcpp", eps=2e-2, d=[8, 8], k_power=2, noise="z2z2", seed=21,
                  targets=targets)
        log(f"trace s32 mlmcpp {targets}")
        got = _gpu(ctx, gid, batch=32, **kw)
        want = otr.estimate(hier, otr.TraceParams(**kw))
        _cmp(got, want)
    assert abs(got["tau_exact"] - want["tau_exact"]) < 1e-9 * abs(want["tau"])


@pytest.mark.parametrize("precision,mlmc", [("fp64", 3), ("fp16", 3), ("fp64", 4)])
def test_concurrent_level_solves_match_sequential(ctx, precision, mlmc):
    """The reduced form solves each level once per phase; with `concurrent`
    the coarse levels run on the field's second stream (own workspaces and
    graphs) while the fine level runs on the first.  Per-sample values, the
    low-rank parts and the counts must not depend on that, over repeated
    estimates (graphs captured on the second, replayed from the third)."""
    th = metropolis_u1(32, 32, 3.0, 100, 951)
    rec = Recipe(th, -0.08, [(4, 4), (2, 2), (2, 2)], [8, 8, 8], seed=17,
                 sap_block=[(4, 4), (2, 1), (1, 1), (1, 1)], inner_iters=[0, 0, 0, 0],
                 mlmc_levels=mlmc, precision=precision)
    log(f"setup concurrent {precision} mlmc levels {mlmc}")
    gid = rec.gpu(ctx)
    nd = mlmc - 1  # level differences
    kw = dict(variant="mlmcpp", eps=2e-2, d=[8] * nd, k_power=2, noise="z2z2", batch=16)
    for rep in range(3):
        a = _gpu(ctx, gid, seed=40 + rep, concurrent=True, **kw)
        b = _gpu(ctx, gid, seed=40 + rep, concurrent=False, **kw)
        assert a["level_samples"] == b["level_samples"]
        assert abs(a["tau"] - b["tau"]) <= 1e-13 * abs(b["tau"])
        for l in range(nd):
            assert np.max(np.abs(a["samples"][l] - b["samples"][l])) <= 1e-12 * np.max(np.abs(b["samples"][l]))
            assert abs(a["level_lr"][l] - b["level_lr"][l]) <= 1e-12 * abs(b["tau"])
    if precision == "fp64":
        hier = rec.oracle()
        want = otr.estimate(hier, otr.TraceParams(seed=42, **{k: v for k, v in kw.items() if k != "batch"},
                                                  levels=mlmc))
        _cmp(a, want)


def test_solver_only_coarse_level_and_vcycles(ctx):
    """A 4-level solver hierarchy whose MLMC sum closes on level 2 (exact
    dense trace there); level 3 only serves the preconditioner, and levels 1-2
    use plain V-cycles instead of inner FGMRES."""
    th = metropolis_u1(32, 32, 3.0, 100, 944)
    rec = Recipe(th, -0.08, [(4, 4), (2, 2), (2, 2)], [8, 8, 8], seed=13,
                 sap_block=[(4, 4), (1, 1), (1, 1), (1, 1)], inner_iters=[0, 0, 0, 0],
                 mlmc_levels=3)
    log("setup 4-level / mlmc 3")
    gid = rec.gpu(ctx)
    hier = rec.oracle()
    kc = rec.kcycle(hier)
    from gpu_util import empty, rel_err, to_dev, to_host
    from lattice_inputs import rhs_vectors
    r = rhs_vectors(hier.levels[0].n, 2, 5)
    x = empty(2, hier.levels[0].n)
    ctx.precondition(gid, 0, to_dev(r), x)
    assert rel_err(to_host(x), kc.apply(0, r.T).T) < 1e-7
    kw = dict(variant="mlmcpp", eps=2e-2, d=[8, 8], k_power=2, noise="z2z2", seed=31, levels=3)
    got = _gpu(ctx, gid, batch=16, **{k: v for k, v in kw.items() if k != "levels"})
    want = otr.estimate(hier, otr.TraceParams(**kw))
    _cmp(got, want)
    assert abs(got["tau_exact"] - want["tau_exact"]) < 1e-9 * abs(want["tau"])


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_low_precision_preconditioner_keeps_fp64_results(ctx, precision):
    """Mixed precision: the whole multigrid cycle in FP32 (and, for fp16, the
    coarse blocks in FP16 on the matrix cores) inside FP64 FGMRES.  Every
    solve still meets its FP64 residual tolerance, so the estimate matches
    the FP64 oracle on the same seeds."""
    th = metropolis_u1(32, 32, 3.0, 100, 932)
    rec = Recipe(th, -0.08, [(4, 4), (2, 2)], [8, 8], seed=11, sap_block=[(4, 4), (1, 1), (1, 1)],
                 inner_iters=[0, 4, 4], precision=precision)
    gid = rec.gpu(ctx)
    hier = rec.oracle()
    from gpu_util import empty, to_dev, to_host
    from lattice_inputs import rhs_vectors
    from paper_2303_11512_amd import solve_params
    lev = hier.levels[0]
    b = rhs_vectors(lev.n, 6, 17)
    x = empty(6, lev.n)
    st, its, rel = ctx.solve_batch(gid, 0, to_dev(b), x, solve_params(tol=1e-10, restart=24))
    res = np.linalg.norm(b - (lev.D @ to_host(x).T).T, axis=1) / np.linalg.norm(b, axis=1)
    assert np.all(res <= 1e-10)
    kw = dict(variant="mlmcpp", eps=2e-2, d=[8, 8], k_power=2, noise="z2z2", seed=21)
    got = _gpu(ctx, gid, batch=32, **kw)
    want = otr.estimate(hier, otr.TraceParams(**kw))
    _cmp(got, want)


def test_fixed_cost_and_full_form_s32(ctx, s32):
    rec, gid, hier = s32
    kw = dict(variant="mlmcpp", form="full", eps=5e-2, d=[4, 4], k_power=1, noise="z2z2", seed=8,
              fixed_cost=[3.0, 1.0], fixed_samples=[12, 20])
    got = _gpu(ctx, gid, batch=8, **kw)
    want = otr.estimate(hier, otr.TraceParams(**kw))
    _cmp(got, want)


def test_fp16_blocks_change_only_the_preconditioner(ctx):
    """The FP16 mode differs from the FP32 one in the coarse blocks only: its
    preconditioner output moves by about FP16 rounding (not more), and its
    solves still reach the FP64 tolerance."""
    from gpu_util import empty, to_dev, to_host
    from lattice_inputs import rhs_vectors
    from paper_2303_11512_amd import solve_params
    th = metropolis_u1(32, 32, 3.0, 100, 933)
    rec = Recipe(th, -0.08, [(4, 4), (2, 2)], [8, 8], seed=11, sap_block=[(4, 4), (1, 1), (1, 1)],
                 inner_iters=[0, 0, 0], precision="fp64")
    gid = rec.gpu(ctx)
    hier = rec.oracle()
    lev = hier.levels[0]
    r = to_dev(rhs_vectors(lev.n, 5, 19))
    out = {}
    for prec in ("fp64", "fp32", "fp16"):
        ctx.set_precision(gid, prec)
        z = empty(5, lev.n)
        ctx.precondition(gid, 0, r, z)
        out[prec] = to_host(z)
    ref = np.linalg.norm(out["fp64"])
    e32 = np.linalg.norm(out["fp32"] - out["fp64"]) / ref
    e16 = np.linalg.norm(out["fp16"] - out["fp64"]) / ref
    log(f"preconditioner rel. change: fp32 {e32:.2e}, fp16 {e16:.2e}")
    assert e32 < 1e-5 and 1e-6 < e16 < 2e-2
    b = rhs_vectors(lev.n, 6, 23)
    x = empty(6, lev.n)
    st, its, rel = ctx.solve_batch(gid, 0, to_dev(b), x, solve_params(tol=1e-10, restart=24))
    res = np.linalg.norm(b - (lev.D @ to_host(x).T).T, axis=1) / np.linalg.norm(b, axis=1)
    assert np.all(res <= 1e-10)


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_mixed_precision_cut_of_the_512_workload(ctx, precision):
    """The 64^2 cut of the 512^2 mixed-precision workload (beta 4.0, m0 -0.08,
    gauge seed 4001, 4x4 then 2x2 aggregation): the estimate with the low
    precision preconditioner equals the FP64 oracle's on the same seeds."""
    th = metropolis_u1(64, 64, 4.0, 200, 4001)
    rec = Recipe(th, -0.08, [(4, 4), (2, 2)], [8, 8], seed=4018, sap_block=[(4, 4), (1, 1), (1, 1)],
                 sap_cycles=[3, 3, 3], inner_iters=[0, 0, 0], precision=precision)
    log(f"cut 64^2 {precision}: setup")
    gid = rec.gpu(ctx)
    hier = rec.oracle()
    kw = dict(variant="mlmcpp", eps=1e-2, d=[16, 16], k_power=2, noise="z2z2", seed=5,
              fixed_samples=[6, 10])
    got = _gpu(ctx, gid, batch=16, **kw)
    want = otr.estimate(hier, otr.TraceParams(**kw))
    _cmp(got, want)


@pytest.mark.parametrize("variant,batch,fixed", [("hutchpp", 16, [25]), ("hutchpp", 8, None),
                                                 ("mlmcpp", 32, None)])
def test_two_sided_projection_parity(ctx, s16, s32, variant, batch, fixed):
    """tau_s = z^H (A z) (the samples are projected before their solves, so
    they do not ride with the last Hutch++ round): parity with the oracle on
    identical seeds, replay and adaptive."""
    if variant == "hutchpp":
        cfg, rec, gid, hier = s16
        kw = dict(variant="hutchpp", eps=1e-2, d=[8], k_power=2, noise="rademacher", seed=13)
    else:
        rec, gid, hier = s32
        kw = dict(variant="mlmcpp", eps=2e-2, d=[8, 8], k_power=2, noise="z2z2", seed=23)
    if fixed:
        kw["fixed_samples"] = fixed
    log(f"two-sided {variant} batch {batch} fixed {fixed}")
    got = _gpu(ctx, gid, batch=batch, projection="two-sided", **kw)
    want = otr.estimate(hier, otr.TraceParams(projection="two-sided", **kw))
    _cmp(got, want)
    # and the one-sided samples of the same seeds differ (another estimator)
    one = _gpu(ctx, gid, batch=batch, **kw)
    assert np.max(np.abs(np.asarray(one["samples"][0])[:5] - np.asarray(got["samples"][0])[:5])) > 1e-6 * abs(got["tau"])


@pytest.mark.parametrize("case", ["hutchpp", "mlmcpp", "mlmcpp-fixed"])
def test_adaptive_d_parity(ctx, s16, s32, case):
    """Adaptive number of Hutch++ vectors per level difference: the same
    candidates, pilot variances and choices as the oracle's (static or fixed
    cost model), then Alg. 2 with the chosen bases."""
    if case == "hutchpp":
        cfg, rec, gid, hier = s16
        kw = dict(variant="hutchpp", eps=1e-2, d=[2], k_power=2, noise="rademacher", seed=17, d_max=32, pilot=16)
    else:
        rec, gid, hier = s32
        kw = dict(variant="mlmcpp", eps=2e-2, d=[2, 4], k_power=1, noise="z2z2", seed=29, d_max=64, pilot=24)
        if case == "mlmcpp-fixed":
            kw.update(fixed_cost=[5.0, 1.0], cost="fixed")
    log(f"adaptive d {case}")
    got = _gpu(ctx, gid, batch=16, **kw)
    want = otr.estimate(hier, otr.TraceParams(**kw))
    log(f"  chosen d GPU {got['level_d']} oracle {want['level_d']}")
    assert got["level_d"] == want["level_d"]
    _cmp(got, want)
