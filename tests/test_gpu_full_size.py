"""Solves at full workload sizes.  128^2 plain-method-at-scale workload (beta
3.0 Metropolis field, m0 = -0.1, 4x4 then 2x2 aggregates with 8 test
vectors, solver-only 2x2 coarsenings below), in the hierarchy, SAP schedule
and 64-RHS batch of the timed estimator step.  The solver stops on its own
FP64 residual; here every solution's true residual is recomputed on the CPU
with the oracle's Wilson-Dirac operator (Sec. 4's Schwinger discretisation),
for the FP16-block preconditioner the step uses and for the plain FP64 one,
and the two solutions are compared with each other.  512^2 mixed-precision
workload (beta 4.0, m0 = -0.08, 4x4 then 4x4 aggregates): 256 RHS in blocks
of 64 with the FP64, FP32 and FP16-block preconditioners inside FP64
FGMRES, the same check per RHS and the low-precision solutions against the
FP64 one."""
import numpy as np
import pytest

from bench import mg_setup_kwargs
from gpu_util import empty, log, rel_err, to_dev, to_host
from lattice_inputs import WORKLOADS, gauge_for, links_from_theta, rhs_vectors
from oracle.dirac import wilson_dirac

pytestmark = pytest.mark.gpu

TOL = 1e-10
NRHS = 64
# the CPU recomputation of ||b - D x|| / ||b|| differs from the GPU's only by
# summation order: |D| ~ 4 and |x| / |b| < 1e3 here give well under 1e-12
RES_SLACK = 1e-12


@pytest.fixture(scope="module")
def full128():
    from paper_2303_11512_amd import Context, mg_params
    cfg = WORKLOADS["schwinger128"]
    th = gauge_for(cfg)
    ctx = Context(0)
    gid = ctx.set_gauge(to_dev(links_from_theta(th)), cfg["m0"], True)
    log("setup schwinger128 (fp16 blocks)")
    ctx.setup_mg(gid, mg_params(**mg_setup_kwargs(cfg), precision="fp16"))
    D = wilson_dirac(th, cfg["m0"], True)
    yield ctx, gid, D
    ctx.close()


def _solve(ctx, gid, b):
    from paper_2303_11512_amd import solve_params
    x = empty(b.shape[0], b.shape[1])
    st, its, rel = ctx.solve_batch(gid, 0, to_dev(b), x, solve_params(tol=TOL, restart=32, max_restarts=50))
    return to_host(x), np.asarray(its), np.asarray(rel)


def test_full_size_solves_meet_tolerance_with_oracle_operator(full128):
    ctx, gid, D = full128
    b = rhs_vectors(D.shape[0], NRHS, 128)
    xs = {}
    try:
        for prec in ("fp16", "fp64"):
            ctx.set_precision(gid, prec)
            log(f"schwinger128: solve {NRHS} RHS, {prec} preconditioner")
            x, its, rel = _solve(ctx, gid, b)
            res = np.linalg.norm(b - (D @ x.T).T, axis=1) / np.linalg.norm(b, axis=1)
            log(f"  iterations {its.min()}-{its.max()}, oracle residual max {res.max():.3e}")
            assert np.all(np.isfinite(x))
            assert np.all(rel <= TOL), rel.max()
            assert np.all(res <= TOL + RES_SLACK), res.max()
            assert np.all(np.abs(res - rel) <= RES_SLACK), np.abs(res - rel).max()
            xs[prec] = x
    finally:
        ctx.set_precision(gid, "fp16")
    # both solve the same systems to 1e-10: they agree to within the
    # condition number times the tolerance
    d = rel_err(xs["fp16"], xs["fp64"])
    log(f"  fp16 vs fp64 preconditioner solutions: rel. difference {d:.2e}")
    assert d < 1e-6



def test_fp16_cycle_sees_unit_vectors_whatever_the_rhs_scale(full128):
    """Range of the FP16 path: the outer FGMRES hands the low-precision cycle
    its Arnoldi vectors, which have unit norm whatever the scale of b, so the
    FP16 operands never see the right-hand side's magnitude.  With b scaled
    by 2^-480 and 2^+480 (far outside the FP16 and FP32 ranges; squares
    still within FP64, so ||b|| scales exactly) the
    solutions are exactly the scaled unscaled solution, bit for bit."""
    ctx, gid, D = full128
    b = rhs_vectors(D.shape[0], 8, 129)
    x0, its0, _ = _solve(ctx, gid, b)
    for e in (-480, 480):
        a = 2.0 ** e
        log(f"schwinger128 fp16: b scaled by 2^{e}")
        x, its, rel = _solve(ctx, gid, b * a)
        assert np.array_equal(its, its0)
        assert np.all(rel <= TOL)
        assert np.array_equal(x, x0 * a), e


@pytest.fixture(scope="module")
def full512():
    from paper_2303_11512_amd import Context, mg_params
    cfg = WORKLOADS["schwinger512"]
    th = gauge_for(cfg)
    ctx = Context(0)
    gid = ctx.set_gauge(to_dev(links_from_theta(th)), cfg["m0"], True)
    log("setup schwinger512")
    ctx.setup_mg(gid, mg_params(**mg_setup_kwargs(cfg)))
    D = wilson_dirac(th, cfg["m0"], True)
    yield ctx, gid, D
    ctx.close()


def test_full_size_mixed_precision_solves_512(full512):
    from paper_2303_11512_amd import solve_params
    ctx, gid, D = full512
    nrhs = 256
    b = rhs_vectors(D.shape[0], nrhs, 512)
    bn = np.linalg.norm(b, axis=1)
    bd = to_dev(b)
    xs = {}
    try:
        for prec in ("fp64", "fp32", "fp16"):
            ctx.set_precision(gid, prec)
            log(f"schwinger512: solve {nrhs} RHS in blocks of 64, {prec} preconditioner")
            x = empty(nrhs, D.shape[0])
            st, its, rel = ctx.solve_batch(gid, 0, bd, x, solve_params(tol=TOL, restart=16, max_restarts=50,
                                                                       rhs_block=64))
            xh = to_host(x)
            del x
            res = np.linalg.norm(b - (D @ xh.T).T, axis=1) / bn
            its, rel = np.asarray(its), np.asarray(rel)
            log(f"  iterations {its.min()}-{its.max()}, oracle residual max {res.max():.3e}")
            assert np.all(np.isfinite(xh))
            assert np.all(rel <= TOL), rel.max()
            assert np.all(res <= TOL + RES_SLACK), res.max()
            xs[prec] = xh
    finally:
        ctx.set_precision(gid, "fp64")
    for prec in ("fp32", "fp16"):
        d = rel_err(xs[prec], xs["fp64"])
        log(f"  {prec} vs fp64 preconditioner solutions: rel. difference {d:.2e}")
        assert d < 1e-6


@pytest.fixture(scope="module")
def oracle128():
    from oracle import mg as omg
    cfg = WORKLOADS["schwinger128"]
    log("schwinger128: oracle hierarchy")
    return omg.setup_hierarchy(gauge_for(cfg), cfg["m0"], cfg["blocks"], cfg["ntv"],
                               mg_setup_kwargs(cfg)["seed"])


def test_bench_configuration_parity_128(full128, oracle128):
    """The timed step exactly as bench.py runs it: adaptive MG-MLMC++ (Alg. 2,
    reduced form, optimal targets weighed by the Sec. 4 cost model, at least
    16 samples per level), FGMRES(32) to 1e-10, FP16-block preconditioner,
    batch 64, 128^2.  The oracle solves exactly and replays the GPU's
    per-sample costs, which it first recomputes from the GPU's iteration
    counts with its own cost model: the sample counts are equal, the
    estimate and every kept sample agree to 1e-8 relative."""
    from bench import BATCH, SOLVE, method_kwargs
    from oracle import cost as ocost
    from oracle import trace as otr
    from paper_2303_11512_amd import solve_params
    ctx, gid, D = full128
    cfg = WORKLOADS["schwinger128"]
    mk = mg_setup_kwargs(cfg)
    kw = method_kwargs(cfg, 7)
    log("schwinger128: GPU estimate in the bench configuration")
    got = ctx.trace_estimate(gid, solve=solve_params(**SOLVE), batch=BATCH, max_dump=4096, **kw)
    shape = ocost.shape_from_blocks(cfg["Lx"], cfg["Lt"], mk["blocks"], mk["ntv"], mk["sap_block"],
                                    [max(1, v) for v in mk["sap_cycles"]], inner_iters=mk["inner_iters"],
                                    mlmc_levels=mk["mlmc_levels"], restart=SOLVE["restart"])
    costs = []
    for l, its in enumerate(got["sample_iters"]):
        want_c = [ocost.sample(shape, l, int(a), int(b), kw["d"][l]) for a, b in its]
        assert np.array_equal(np.asarray(got["sample_costs"][l]), np.asarray(want_c, dtype=float)), l
        costs.append(want_c)
    log(f"  GPU samples {got['level_samples']}, C_l {got['level_cost']}; oracle estimate (replayed costs)")
    want = otr.estimate(oracle128, otr.TraceParams(**kw, sample_costs=costs))
    scale = abs(want["tau"])
    log(f"  tau GPU {got['tau']:.10f} oracle {want['tau']:.10f}, "
        f"rel. difference {abs(got['tau'] - want['tau']) / scale:.2e}")
    assert got["level_samples"] == want["level_samples"]
    assert min(got["level_samples"]) >= kw["min_samples"]
    assert abs(got["tau"] - want["tau"]) < 1e-8 * scale
    for l in range(len(want["level_samples"])):
        assert abs(got["level_lr"][l] - want["level_lr"][l]) < 1e-8 * scale, l
        ws, gs = np.array(want["samples"][l]), np.asarray(got["samples"][l])
        sc = max(np.max(np.abs(ws)), scale / len(ws))
        log(f"  level {l}: max sample difference / scale {np.max(np.abs(gs - ws)) / sc:.2e}")
        assert np.max(np.abs(gs - ws)) < 1e-8 * sc, l


def test_full_size_trace_replay_128(full128, oracle128):
    """MG-MLMC++ (Alg. 2, reduced form) on the 128^2 workload in the timed
    step's hierarchy, FP16-block preconditioner and batch of 64, replayed with
    8 samples per level difference (Hutch++ with 32 vectors and two power
    steps first): the estimate, the low-rank parts and every sample match the
    oracle's on identical seeds to 1e-8 relative.  Solves are taken to 1e-12
    so that solver error stays far below that."""
    from oracle import trace as otr
    from paper_2303_11512_amd import solve_params
    ctx, gid, D = full128
    cfg = WORKLOADS["schwinger128"]
    kw = dict(variant="mlmcpp", form="reduced", eps=cfg["eps"], d=list(cfg["d"]), k_power=cfg["k_power"],
              noise=cfg["noise"], seed=cfg["trace_seed"] + 40, fixed_samples=[8, 8])
    log("schwinger128: GPU estimate (replay, 8 samples per level)")
    got = ctx.trace_estimate(gid, solve=solve_params(tol=1e-12, restart=32, max_restarts=50), batch=64,
                             max_dump=4096, **kw)
    log("schwinger128: oracle estimate")
    want = otr.estimate(oracle128, otr.TraceParams(**kw))
    scale = abs(want["tau"])
    log(f"  tau GPU {got['tau']:.10f} oracle {want['tau']:.10f}, "
        f"rel. difference {abs(got['tau'] - want['tau']) / scale:.2e}")
    assert abs(got["tau"] - want["tau"]) < 1e-8 * scale
    for l in range(len(want["level_samples"])):
        assert got["level_samples"][l] == want["level_samples"][l] == 8
        assert abs(got["level_lr"][l] - want["level_lr"][l]) < 1e-8 * scale, l
        ws, gs = np.array(want["samples"][l]), np.asarray(got["samples"][l])
        sc = max(np.max(np.abs(ws)), scale / len(ws))
        log(f"  level {l}: max sample difference / scale {np.max(np.abs(gs - ws)) / sc:.2e}")
        assert np.max(np.abs(gs - ws)) < 1e-8 * sc, l
