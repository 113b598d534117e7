"""mgm_orthonormalize_noalloc (CholQR in the library's static device
workspace, no allocation) against mgm_orthonormalize on the same input: two
calls in a row, the second on a smaller block, so that the first call's
leftovers in the shared workspace would show; and sizes beyond the
workspace are rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _block(ctx, d, n, seed):
    import torch
    Y = torch.empty((d, n), dtype=torch.complex128, device="cuda")
    ctx.noise("z2z2", seed, 0, 0, 0, Y)
    return Y


def test_noalloc_orthonormalize_matches_allocating_call():
    import torch
    from paper_2303_11512_amd import Context
    from paper_2303_11512_amd._lib import EINVAL, MGMError
    ctx = Context(0)
    try:
        # the largest block the workspace takes (n d = 2^20: the Hutch++
        # sketch of the 128^2 workload), then a smaller, ragged one
        for n, d, seed in ((32768, 32, 1), (5003, 7, 2)):
            print(f"[no-alloc] n={n} d={d}", flush=True)
            Y = _block(ctx, d, n, seed)
            Qa = torch.empty_like(Y)
            Qb = torch.empty_like(Y)
            ctx.orthonormalize(Y, Qa)
            ctx.orthonormalize_noalloc(Y, Qb)
            torch.cuda.synchronize()
            qa, qb, y = Qa.cpu().numpy(), Qb.cpu().numpy(), Y.cpu().numpy()
            diff = np.max(np.abs(qa - qb))
            print(f"[no-alloc]   max |Q_noalloc - Q| = {diff:.3e}", flush=True)
            assert diff <= 1e-14
            # and it is the thin QR factor: orthonormal rows spanning Y's rows
            assert np.max(np.abs(qb.conj() @ qb.T - np.eye(d))) < 1e-12
            R = qb.conj() @ y.T
            assert np.linalg.norm(y.T - qb.T @ R) < 1e-11 * np.linalg.norm(y)
            assert np.max(np.abs(np.tril(R, -1))) < 1e-10 * np.max(np.abs(R))
        # beyond the workspace: n d > 2^20
        Y = _block(ctx, 64, 16385, 3)
        with pytest.raises(MGMError) as e:
            ctx.orthonormalize_noalloc(Y, torch.empty_like(Y))
        assert e.value.code == EINVAL
    finally:
        ctx.close()
