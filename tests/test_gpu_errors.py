"""Failure handling through the C ABI: every condition is forced from the host
(a tolerance no solver can meet, a non-finite right-hand side, a hierarchy
that does not tile the lattice, an unknown precision), and every kernel still
exits normally.  Status codes: MGM_EINVAL -1, MGM_ESTATE -4, MGM_ENOTCONV -5,
MGM_ENONFINITE -6."""
import numpy as np
import pytest

from gpu_util import Recipe, empty, log, to_dev, to_host
from lattice_inputs import links_from_theta, metropolis_u1, rhs_vectors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2303_11512_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def field(ctx):
    th = metropolis_u1(16, 16, 3.0, 50, 8100)
    rec = Recipe(th, -0.05, [(4, 4)], [4], seed=3, sap_block=[(4, 4), (1, 1)], inner_iters=[0, 0])
    log("error tests: setup 16^2")
    return rec, rec.gpu(ctx), rec.oracle()


def test_unreachable_tolerance_returns_enotconv_and_the_iterate(ctx, field):
    from paper_2303_11512_amd import solve_params
    rec, gid, hier = field
    lev = hier.levels[0]
    b = rhs_vectors(lev.n, 3, 5)
    x = empty(3, lev.n)
    st, its, rel = ctx.solve_batch(gid, 0, to_dev(b), x,
                                   solve_params(tol=1e-30, restart=2, max_restarts=1), check=False)
    assert st == -5
    # the returned x is the last iterate: its residual is the one reported
    xh = to_host(x)
    res = np.linalg.norm(b - (lev.D @ xh.T).T, axis=1) / np.linalg.norm(b, axis=1)
    assert np.allclose(res, rel, rtol=1e-6)
    assert np.all(res < 1.0) and np.all(its == 4)


def test_nonfinite_rhs_returns_enonfinite(ctx, field):
    from paper_2303_11512_amd import MGMError, solve_params
    rec, gid, hier = field
    n = hier.levels[0].n
    b = rhs_vectors(n, 2, 6)
    b[1, 17] = np.nan
    with pytest.raises(MGMError) as e:
        ctx.solve_batch(gid, 0, to_dev(b), empty(2, n), solve_params(tol=1e-10))
    assert e.value.code == -6


def test_zero_rhs_gives_zero_solution(ctx, field):
    from paper_2303_11512_amd import solve_params
    rec, gid, hier = field
    n = hier.levels[0].n
    b = rhs_vectors(n, 3, 7)
    b[1] = 0
    x = empty(3, n)
    st, its, rel = ctx.solve_batch(gid, 0, to_dev(b), x, solve_params(tol=1e-10))
    assert st == 0 and np.all(to_host(x)[1] == 0) and rel[1] == 0 and its[1] == 0


def test_hierarchy_must_tile_the_lattice(ctx):
    from paper_2303_11512_amd import MGMError, mg_params
    th = metropolis_u1(12, 12, 3.0, 5, 8200)
    gid = ctx.set_gauge(to_dev(links_from_theta(th)), -0.05, True)
    with pytest.raises(MGMError) as e:
        ctx.setup_mg(gid, mg_params(2, [(5, 4)], [4], seed=1))  # 5 does not divide 12
    assert e.value.code == -1
    ctx.free_gauge(gid)


def test_unknown_precision_and_calls_out_of_order(ctx, field):
    from paper_2303_11512_amd import MGMError, _lib
    rec, gid, hier = field
    with pytest.raises(MGMError) as e:
        ctx._chk(ctx.lib.mgm_set_precision(ctx.h, gid, 7), "set_precision")
    assert e.value.code == -1
    th = metropolis_u1(16, 16, 3.0, 5, 8300)
    g2 = ctx.set_gauge(to_dev(links_from_theta(th)), -0.05, True)
    with pytest.raises(MGMError) as e:
        ctx.set_precision(g2, "fp32")  # no hierarchy yet
    assert e.value.code == -4
    with pytest.raises(MGMError) as e:
        ctx.time_kernel(g2, "sap", 0, 4)
    assert e.value.code == -4
    ctx.free_gauge(g2)
    # the context keeps working after errors
    n = hier.levels[0].n
    y = empty(1, n)
    ctx.apply_D(gid, 0, to_dev(rhs_vectors(n, 1, 9)), y)
    assert np.all(np.isfinite(to_host(y)))
