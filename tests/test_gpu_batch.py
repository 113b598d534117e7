"""Batching across gauge fields and lattice sizes: mgm_solve_jobs (one call,
fields on concurrent streams), HIP-graph replay of the preconditioner, and
the RHS-block autotuner.  Every solve is checked with the oracle's operator."""
import numpy as np
import pytest

from gpu_util import Recipe, empty, log, to_dev, to_host
from lattice_inputs import metropolis_u1, rhs_vectors
from oracle import trace as otr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2303_11512_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def fields(ctx):
    """Three fields of different sizes and couplings, each with its hierarchy."""
    specs = [
        (16, 16, 2.0, -0.06, [(4, 4)], [4], [(4, 4), (1, 1)]),
        (32, 32, 4.0, -0.05, [(4, 4), (2, 2)], [8, 8], [(4, 4), (1, 1), (1, 1)]),
        (32, 16, 3.0, -0.04, [(4, 4), (2, 2)], [4, 4], [(4, 4), (1, 1), (1, 1)]),
    ]
    out = []
    for k, (Lx, Lt, beta, m0, blocks, ntv, sap) in enumerate(specs):
        th = metropolis_u1(Lx, Lt, beta, 60, 7000 + k)
        rec = Recipe(th, m0, blocks, ntv, seed=20 + k, sap_block=sap, inner_iters=[0, 3, 3])
        log(f"setup field {k}: {Lx}x{Lt}")
        gid = rec.gpu(ctx)
        out.append((rec, gid, rec.oracle()))
    return out


def test_solve_jobs_matches_separate_solves(ctx, fields):
    from paper_2303_11512_amd import solve_params
    sp = solve_params(tol=1e-10, restart=20)
    jobs, want_b, order = [], [], []
    for k, (rec, gid, hier) in enumerate(fields):
        for level, nrhs in [(0, 5), (1, 3)]:
            n = hier.levels[level].n
            b = rhs_vectors(n, nrhs, 300 + 10 * k + level)
            jobs.append((gid, level, to_dev(b), empty(nrhs, n)))
            want_b.append(b)
            order.append((k, level))
    log("solve_jobs over 3 fields")
    st, its = ctx.solve_jobs(jobs, sp)
    assert st == 0 and len(its) == sum(b.shape[0] for b in want_b)
    for (k, level), (gid, lvl, b_dev, x_dev), b in zip(order, jobs, want_b):
        lev = fields[k][2].levels[level]
        x = to_host(x_dev)
        res = np.linalg.norm(b - (lev.D @ x.T).T, axis=1) / np.linalg.norm(b, axis=1)
        assert np.all(res <= 1e-10), (k, level, res)
        # the same solve issued alone gives the same bits
        x2 = empty(*b.shape)
        ctx.solve_batch(gid, level, b_dev, x2, sp)
        assert np.array_equal(to_host(x2), x)


def test_graph_replay_gives_identical_estimates(ctx):
    th = metropolis_u1(32, 32, 3.0, 60, 7100)
    kw = dict(variant="mlmcpp", eps=3e-2, d=[4, 4], k_power=1, noise="z2z2", seed=4)
    outs = []
    for graphs in (True, False):
        from paper_2303_11512_amd import mg_params, solve_params
        gid = ctx.set_gauge(to_dev(np.exp(1j * th)), -0.07, True)
        ctx.setup_mg(gid, mg_params(3, [(4, 4), (2, 2)], [8, 8], sap_block=[(4, 4), (1, 1), (1, 1)],
                                    inner_iters=[0, 3, 3], seed=5, graphs=graphs))
        outs.append(ctx.trace_estimate(gid, batch=16, solve=solve_params(tol=1e-10, restart=16), **kw))
    assert outs[0]["level_samples"] == outs[1]["level_samples"]
    assert outs[0]["tau"] == outs[1]["tau"]
    assert outs[0]["iters"] == outs[1]["iters"]


def test_autotuner_picks_a_width_and_solves(ctx, fields):
    from paper_2303_11512_amd import solve_params
    rec, gid, hier = fields[1]
    best = ctx.autotune_rhs_block(gid, 0, 24, solve_params(tol=1e-10, restart=16))
    assert best in (8, 16, 24)
    lev = hier.levels[0]
    b = rhs_vectors(lev.n, 24, 401)
    x = empty(24, lev.n)
    ctx.solve_batch(gid, 0, to_dev(b), x, solve_params(tol=1e-10, restart=16, rhs_block=-1))
    res = np.linalg.norm(b - (lev.D @ to_host(x).T).T, axis=1) / np.linalg.norm(b, axis=1)
    assert np.all(res <= 1e-10)


def test_free_gauge_releases_the_field(ctx):
    from paper_2303_11512_amd import MGMError, mg_params
    th = metropolis_u1(16, 16, 3.0, 20, 7200)
    gid = ctx.set_gauge(to_dev(np.exp(1j * th)), -0.05, True)
    ctx.setup_mg(gid, mg_params(2, [(4, 4)], [4], seed=2))
    ctx.free_gauge(gid)
    with pytest.raises(MGMError):
        ctx.level_info(gid, 0)
    with pytest.raises(MGMError):
        ctx.free_gauge(gid)
    gid2 = ctx.set_gauge(to_dev(np.exp(1j * th)), -0.05, True)
    assert gid2 != gid and ctx.level_info(gid2, 0)["n"] == 2 * 16 * 16


def test_trace_jobs_match_separate_estimates(ctx, fields):
    """mgm_trace_jobs: one estimate per field at once (different variants,
    targets and seeds per job) gives, job by job, the bits of separate
    mgm_trace_estimate calls; the estimates match the oracle's Alg. 2."""
    from paper_2303_11512_amd import solve_params
    sp = solve_params(tol=1e-12, restart=24)
    kws = [dict(variant="mlmcpp", eps=3e-2, d=[4], k_power=1, noise="z2z2", seed=5, batch=16),
           dict(variant="mlmc", eps=3e-2, noise="rademacher", seed=6, batch=8, targets="uniform"),
           dict(variant="mlmcpp", eps=3e-2, d=[4, 4], k_power=2, noise="z2z2", seed=7, batch=16,
                cost="flops")]
    jobs = [(gid, dict(kw, solve=sp, max_dump=512)) for (_, gid, _), kw in zip(fields, kws)]
    log("trace_jobs over 3 fields")
    got = ctx.trace_jobs(jobs)
    for k, ((rec, gid, hier), (_, kw)) in enumerate(zip(fields, jobs)):
        alone = ctx.trace_estimate(gid, **kw)
        assert got[k]["tau"] == alone["tau"], k
        assert got[k]["level_samples"] == alone["level_samples"], k
        for a, b in zip(got[k]["samples"], alone["samples"]):
            assert np.array_equal(a, b), k
        if kw.get("cost", "static") == "static":
            want = otr.estimate(hier, otr.TraceParams(**{q: v for q, v in kw.items()
                                                         if q not in ("solve", "max_dump", "batch")}))
            assert got[k]["level_samples"] == want["level_samples"], k
            assert abs(got[k]["tau"] - want["tau"]) < 1e-8 * abs(want["tau"]), k


def test_trace_jobs_rejects_a_shared_field(ctx, fields):
    from paper_2303_11512_amd import MGMError
    gid = fields[0][1]
    with pytest.raises(MGMError):
        ctx.trace_jobs([(gid, dict(eps=1e-1)), (gid, dict(eps=1e-1))])
