"""GPU parity of the single kernels against the oracle: noise (bit-exact),
the fine Schwinger stencil (Sec. 4), and qr+ (CholQR)."""
import numpy as np
import pytest

from gpu_util import empty, log, rel_err, to_dev, to_host
from lattice_inputs import links_from_theta, metropolis_u1, rhs_vectors
from oracle import mg, rng
from oracle.dirac import wilson_dirac

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2303_11512_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("kind", ["rademacher", "z2z2"])
def test_noise_bit_exact(ctx, kind):
    n, nrhs = 3001, 5
    for (seed, purpose, level, index0) in [(1, rng.PURPOSE_SAMPLE, 0, 0), (2000, rng.PURPOSE_SKETCH, 2, 17),
                                           (2 ** 63 + 5, rng.PURPOSE_SETUP, 1, 2 ** 40)]:
        log(f"noise {kind} seed={seed} purpose={purpose} level={level} index0={index0}")
        out = empty(nrhs, n)
        ctx.noise(kind, seed, purpose, level, index0, out)
        got = to_host(out)
        want = np.stack([rng.noise_vector(kind, seed, purpose, level, index0 + r, n) for r in range(nrhs)])
        assert np.array_equal(got, want)


# Lx a multiple of 64 (<= 256) takes the row-strip kernel, whose strip height
# (1..16 rows) follows Lt and the RHS count: the cases below reach every height
# on MI355X, including a ragged count of strips (Lt = 40) and the fallback
# when no height keeps every workgroup resident (Lt = 12, 700 RHS).  Wider rows
# take the strip kernel with 2 (Lx = 384, 512) or 4 (Lx = 768, 1024) columns
# per thread; Lx = 640 has no such split and takes the thread-per-site kernel.
# Many RHS on a short lattice (64 x 128, 640 RHS) need strips of 32 or 64 rows.
@pytest.mark.parametrize("Lx,Lt,nrhs,m0", [(8, 8, 1, -0.05), (10, 6, 5, 0.2), (34, 18, 3, -0.1),
                                           (128, 128, 64, -0.1), (64, 64, 16, -0.1),
                                           (192, 24, 7, 0.1), (64, 40, 200, -0.05),
                                           (64, 256, 96, -0.1), (128, 12, 700, 0.0),
                                           (256, 32, 3, -0.08), (384, 16, 5, -0.1),
                                           (512, 64, 9, -0.08), (768, 8, 3, 0.1),
                                           (1024, 16, 4, -0.05), (640, 8, 2, 0.0),
                                           (64, 128, 640, -0.1), (512, 128, 64, -0.08)])
def test_wilson_apply_matches_oracle(ctx, Lx, Lt, nrhs, m0):
    log(f"wilson apply {Lx}x{Lt} nrhs={nrhs}")
    th = metropolis_u1(Lx, Lt, 3.0, 30, 17 + Lx)
    gid = ctx.set_gauge(to_dev(links_from_theta(th)), m0, True)
    n = 2 * Lx * Lt
    x = rhs_vectors(n, nrhs, 5) * (1 + np.arange(nrhs))[:, None]
    y = empty(nrhs, n)
    ctx.apply_D(gid, 0, to_dev(x), y)
    D = wilson_dirac(th, m0)
    want = (D @ x.T).T
    assert rel_err(to_host(y), want) < 1e-14


@pytest.mark.parametrize("Lx,Lt", [(8, 8), (64, 16), (512, 8)])
def test_wilson_periodic_bc(ctx, Lx, Lt):
    th = metropolis_u1(Lx, Lt, 2.0, 20, 3)
    gid = ctx.set_gauge(to_dev(links_from_theta(th)), 0.3, False)
    n = 2 * Lx * Lt
    x = rhs_vectors(n, 2, 9)
    y = empty(2, n)
    ctx.apply_D(gid, 0, to_dev(x), y)
    assert rel_err(to_host(y), (wilson_dirac(th, 0.3, bc_t_anti=False) @ x.T).T) < 1e-14


@pytest.mark.parametrize("n,d", [(1000, 7), (4097, 32), (300, 1), (70001, 64), (20000, 48), (32768, 32)])
def test_orthonormalize_is_qr_plus(ctx, n, d):
    log(f"orthonormalize n={n} d={d}")
    rs = np.random.default_rng(n + d)
    Y = rs.standard_normal((n, d)) + 1j * rs.standard_normal((n, d))
    Y[:, -1] += 1e-3 * Y[:, 0]  # mildly ill-conditioned
    Q = empty(d, n)
    ctx.orthonormalize(to_dev(Y.T), Q)
    got = to_host(Q).T
    want = mg.qr_plus(Y)
    assert np.max(np.abs(got - want)) < 1e-11


def test_bad_arguments_return_errors(ctx):
    from paper_2303_11512_amd import MGMError
    th = metropolis_u1(8, 8, 2.0, 5, 3)
    gid = ctx.set_gauge(to_dev(links_from_theta(th)), 0.1, True)
    x = empty(1, 128)
    with pytest.raises(MGMError) as e:
        ctx.apply_D(gid, 1, x, empty(1, 128))  # no coarse level before setup_mg
    assert e.value.code in (-1, -4)
    with pytest.raises(MGMError):
        ctx.trace_estimate(gid)  # needs setup_mg
