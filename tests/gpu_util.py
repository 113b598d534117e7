"""Helpers shared by the GPU parity tests: device transfer, the library
context, and matching multigrid parameters on both sides."""
import sys

import numpy as np

from lattice_inputs import links_from_theta


def log(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda")


def to_host(t):
    return t.detach().cpu().numpy()


def empty(nrhs, n):
    import torch
    return torch.empty((nrhs, n), dtype=torch.complex128, device="cuda")


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# One multigrid recipe used by both sides of a parity test.
class Recipe:
    def __init__(self, theta, m0, blocks, ntv, seed=7, sap_block=None, sap_cycles=None,
                 inner_iters=None, inner_tol=0.0, precision="fp64", mlmc_levels=0):
        self.theta, self.m0, self.blocks, self.ntv, self.seed = theta, m0, blocks, ntv, seed
        self.mlmc_levels = mlmc_levels
        L = len(blocks) + 1
        self.L = L
        self.sap_block = sap_block or [blocks[0]] + [(1, 1)] * (L - 1)
        self.sap_cycles = sap_cycles or [2] * L
        self.inner_iters = inner_iters or [4] * L
        self.inner_tol = inner_tol
        self.precision = precision

    def gpu(self, ctx):
        from paper_2303_11512_amd import mg_params
        gid = ctx.set_gauge(to_dev(links_from_theta(self.theta)), self.m0, True)
        ctx.setup_mg(gid, mg_params(self.L, self.blocks, self.ntv, sap_block=self.sap_block,
                                    sap_cycles=self.sap_cycles, inner_iters=self.inner_iters,
                                    inner_tol=self.inner_tol, seed=self.seed,
                                    precision=self.precision, mlmc_levels=self.mlmc_levels))
        return gid

    def oracle(self):
        from oracle import mg
        return mg.setup_hierarchy(self.theta, self.m0, self.blocks, self.ntv, self.seed)

    def kcycle(self, hier):
        from oracle import mg
        return mg.KCycle(hier, mg.CycleParams(sap_block=self.sap_block[:self.L - 1],
                                              sap_cycles=self.sap_cycles[:self.L - 1],
                                              inner_iters=self.inner_iters))
