"""Benchmark: MG-MLMC++ trace estimates per second on one MI355X.

One step = one full MG-MLMC++ estimate of tr(D^{-1}) to the workload's relative
accuracy (Hutch++ low-rank parts on every level difference, then the adaptive
stochastic part of Alg. 2 with optimal target variances), with the gauge
field and the multigrid hierarchy already resident in HBM (the hierarchy
setup is timed separately and reported as ``setup_s``).

Prints one JSON line (see the fields below).  ``--gpus N`` with N > 1 is not
supported: the build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# red/black SAP cycles per level of the V-cycle (fine, first coarse, deeper)
# and the SAP blocks below the fine level (2x2 sites on the first coarse
# level, single sites deeper): a sweep on the 128^2 workload (fine-level
# solves concurrent with the coarse-level ones) puts the minimum of time per
# estimate at 4 / 6 / 3 with 2x2 blocks (6 cycles: 5 / 6 iterations on levels
# 0 / 1; 7 or 8: 5 / 5 but no faster; 4: the fine level needs 5-6), ahead of
# 2x1 blocks (best at 10 cycles, 5 / 5 iterations, 5% slower)
SAP_CYCLES = (4, 6, 3, 3, 3, 3)
COARSE_SAP_BLOCKS = [(2, 2), (1, 1), (1, 1), (1, 1), (1, 1)]


def mg_setup_kwargs(cfg):
    """The workload's MLMC hierarchy plus, while its coarsest level is large,
    solver-only 2x2 coarsenings below it (the MLMC sum still closes on the
    workload's coarsest level, whose trace is computed exactly); plain
    V-cycles with 3 red/black SAP cycles per level."""
    blocks, ntv = list(cfg["blocks"]), list(cfg["ntv"])
    mlmc = len(blocks) + 1
    Nx, Nt = cfg["Lx"], cfg["Lt"]
    for (bx, bt) in blocks:
        Nx, Nt = Nx // bx, Nt // bt
    while Nx * Nt * 2 * ntv[-1] > 2048 and Nx % 4 == 0 and Nt % 4 == 0 and len(blocks) < 5:
        blocks.append((2, 2))
        ntv.append(ntv[-1])
        Nx, Nt = Nx // 2, Nt // 2
    L = len(blocks) + 1
    return dict(
        nlevels=L, blocks=blocks, ntv=ntv, mlmc_levels=mlmc,
        sap_block=[blocks[0]] + COARSE_SAP_BLOCKS,
        sap_cycles=list(SAP_CYCLES), inner_iters=[0] * 6, inner_tol=0.0,
        setup_iters=3, setup_tol=1e-10, setup_restart=32, setup_max_restarts=200,
        seed=cfg["gauge_seed"] + 17,
    )


# samples per level per GPU batch (the speculative batch of the estimator)
BATCH = 64
# Alg. 2's stop test V_l / s <= rho_l^2 is not applied before this many
# samples per level: the literal reading allows a test at s = 2, where a
# 2-sample variance can stop the estimate long before it holds its accuracy
MIN_SAMPLES = 16
# the solves of the timed step: FGMRES(32), true FP64 residual 1e-10
SOLVE = dict(tol=1e-10, restart=32, max_restarts=50)


def method_kwargs(cfg, step):
    """Alg. 2 as timed (MG-MLMC++, reduced form, optimal target variances
    weighed by the Sec. 4 cost model), the same for the oracle."""
    return dict(variant="mlmcpp", form="reduced", eps=cfg["eps"], d=cfg["d"], k_power=cfg["k_power"],
                noise=cfg["noise"], targets="optimal", cost="flops", min_samples=MIN_SAMPLES,
                seed=cfg["trace_seed"] + step)


def trace_kwargs(cfg, step):
    return dict(method_kwargs(cfg, step), batch=BATCH)


KERNEL_RHS = 64
# the kernel with the largest share of the step's GPU time (rocprofv3 of the
# 128^2 step) per preconditioner precision: one colour of the SAP sweep on the
# first coarse level (16 dofs per site, 2x2-site blocks, premultiplied form)
DOMINANT = {"fp64": "sap_l1", "fp32": "saplow_l1", "fp16": "saplow_l1"}
KERNEL_NAME = {"fp64": "k_sap4p<double, false>", "fp32": "k_sap4p<float, false>", "fp16": "k_sap4p_h<false>"}
# counter summaries of those kernels (FETCH_SIZE / WRITE_SIZE runs, scaled by
# the copy-kernel calibration), keyed to the source file they were measured from
TRAFFIC_SUMMARY = {p: os.path.join(ROOT, "profiles", KERNEL_NAME[p].replace(", ", "_").replace("<", "_")
                                   .replace(">", "") + "_l1_schwinger128_traffic.txt") for p in DOMINANT}
KERNEL_SOURCE = os.path.join(ROOT, "paper_2303_11512_amd", "csrc", "ops.hip")


STENCIL512_SUMMARY = os.path.join(ROOT, "profiles", "k_wilson_strip_schwinger512_traffic.txt")


def measured_traffic(precision=None, path=None):
    """HBM bytes per launch of a kernel from its committed counter summary
    (the dominant kernel of the step for `precision`, or the file `path`);
    None when there is none or the kernel source has changed since the
    counters were taken."""
    import hashlib
    try:
        fields = {}
        with open(path or TRAFFIC_SUMMARY[precision]) as f:
            for ln in f:
                if ":" in ln and not ln.startswith((" ", "#")):
                    k, v = ln.split(":", 1)
                    fields[k.strip()] = v.strip()
        with open(KERNEL_SOURCE, "rb") as f:
            src = hashlib.sha256(f.read()).hexdigest()
        if fields.get("source_sha256") != src:
            return None
        return float(fields["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


STEP_PROFILE = os.path.join(ROOT, "profiles", "schwinger128_step_kernel_stats.txt")


def in_step_average(precision, alg_bytes):
    """Average duration of the dominant kernel inside the timed step, from
    the committed rocprofv3 kernel trace of the step (None when it is missing
    or the kernel source changed since it was taken)."""
    import hashlib
    try:
        with open(KERNEL_SOURCE, "rb") as f:
            src = hashlib.sha256(f.read()).hexdigest()
        name = KERNEL_NAME[precision]
        calls = total = 0.0
        sha = None
        in_step = False
        with open(STEP_PROFILE) as f:
            for ln in f:
                if ln.startswith("source_sha256:"):
                    sha = ln.split(":", 1)[1].strip()
                if ln.startswith("## "):
                    in_step = "timed step" in ln
                    continue
                parts = ln.split()
                if in_step and len(parts) >= 4 and " ".join(parts[3:]) == name:
                    total += float(parts[0])
                    calls += float(parts[1])
        if sha != src or calls == 0:
            return None
        us = total / calls * 1e3
        return {"avg_us": us, "calls": int(calls), "GB/s": alg_bytes / (us * 1e-6) / 1e9,
                "frac": alg_bytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS}
    except (OSError, ValueError, KeyError):
        return None


def ensemble_run(ctx, cfg, mgkw, args):
    """Production mode for an ensemble: `--ensemble` gauge fields of the
    workload (gauge seeds seed, seed + 1, ...), one estimate per field at once
    through mgm_trace_jobs (each field on its own streams and host thread),
    `--steps` rounds, same estimator settings as the timed step."""
    import torch
    from lattice_inputs import gauge_for, links_from_theta
    from paper_2303_11512_amd import mg_params, solve_params
    sp = solve_params(**SOLVE)
    gids = []
    for f in range(args.ensemble):
        c = dict(cfg, gauge_seed=cfg["gauge_seed"] + f)
        g = ctx.set_gauge(torch.from_numpy(links_from_theta(gauge_for(c))).to("cuda"), cfg["m0"], True)
        ctx.setup_mg(g, mg_params(**mgkw, precision=args.precision))
        gids.append(g)
    ctx.trace_jobs([(g, dict(solve=sp, **trace_kwargs(cfg, 1000 + f))) for f, g in enumerate(gids)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rounds = [ctx.trace_jobs([(g, dict(solve=sp, **trace_kwargs(cfg, k))) for g in gids])
              for k in range(args.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the same estimates one after the other (the first field alone is the
    # headline's workload)
    t1 = time.perf_counter()
    seq = [[ctx.trace_estimate(g, solve=sp, **trace_kwargs(cfg, k)) for g in gids] for k in range(args.steps)]
    torch.cuda.synchronize()
    dts = time.perf_counter() - t1
    same = all(a["tau"] == b["tau"] for r, q in zip(rounds, seq) for a, b in zip(r, q))
    for g in gids:
        ctx.free_gauge(g)
    n = args.ensemble * args.steps
    return {"what": f"{args.ensemble} fields of the workload (gauge seeds {cfg['gauge_seed']}.."
                    f"{cfg['gauge_seed'] + args.ensemble - 1}), one estimate per field at once (mgm_trace_jobs)",
            "estimates_per_s": n / dt, "sequential_estimates_per_s": n / dts,
            "gain_over_sequential": dts / dt, "bitwise_equal_to_sequential": same,
            "tau_per_field": [[o["tau"].real, o["tau"].imag] for o in rounds[0]]}


def plain_fp64_run(ctx, th, cfg, mgkw, steps, ref):
    """Plain FP64 MG-FGMRES on the same GPU and seeds: FP64 preconditioner,
    no captured graphs, one stream, and Alg. 2's stochastic loop one sample
    per level at a time (batch 1; the Hutch++ sketch is one block of d
    vectors, as Alg. 2 writes it)."""
    import torch
    from lattice_inputs import links_from_theta
    from paper_2303_11512_amd import mg_params, solve_params
    gid = ctx.set_gauge(torch.from_numpy(links_from_theta(th)).to("cuda"), cfg["m0"], True)
    ctx.setup_mg(gid, mg_params(**dict(mgkw, graphs=False), precision="fp64"))
    sp = solve_params(**SOLVE)
    kw = lambda k: dict(trace_kwargs(cfg, k), batch=1, concurrent=False)
    ctx.trace_estimate(gid, solve=sp, **kw(1000))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [ctx.trace_estimate(gid, solve=sp, **kw(k)) for k in range(steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.free_gauge(gid)
    return {"what": "FP64 preconditioner, no graphs, one stream, one sample per level at a time",
            "estimates_per_s": steps / dt, "ms_per_step": dt / steps * 1e3, "steps": steps,
            "max_tau_rel_diff": max(abs(a["tau"] - b["tau"]) / abs(b["tau"]) for a, b in zip(outs, ref))}


def kernel_table(ctx, gid, nrhs=KERNEL_RHS, mlmc_coarsest=None, precision="fp64"):
    """Average launch duration (HIP events on the library's stream, 50
    back-to-back launches), algorithmic bytes and flops of the step's hot
    kernels at the step's shape."""
    L = 0
    while True:
        try:
            ctx.level_info(gid, L + 1)
            L += 1
        except Exception:
            break
    t = {
        "stencil_l0": ctx.time_kernel(gid, "stencil", 0, nrhs),
        "sap_l0": ctx.time_kernel(gid, "sap", 0, nrhs),
        "sap_l1": ctx.time_kernel(gid, "sap", 1, nrhs),
        "stencil_l1": ctx.time_kernel(gid, "stencil", 1, nrhs),
        "cgs16_l0": ctx.time_kernel(gid, "cgs", 0, nrhs),
        "copy_l0": ctx.time_kernel(gid, "copy", 0, nrhs),
        "dense_l%d" % L: ctx.time_kernel(gid, "dense", L, nrhs),
    }
    if mlmc_coarsest is not None and mlmc_coarsest != L:
        t["dense_l%d" % mlmc_coarsest] = ctx.time_kernel(gid, "dense", mlmc_coarsest, nrhs, reps=10)
    if precision != "fp64":
        for l in range(min(L, 3)):
            t["saplow_l%d" % l] = ctx.time_kernel(gid, "sap_low", l, nrhs)
    return t


def cpu_baseline(cfg, gpu_samples, budget_s=25.0):
    """Time the oracle (1 thread) on a bounded sample of the same workload and
    scale to one estimate with the GPU run's per-level sample counts."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    code = (
        "import json,sys; sys.path.insert(0, %r); import bench; "
        "print(json.dumps(bench._oracle_sample(%r, %r, %r)))" % (ROOT, cfg["name"], gpu_samples, budget_s)
    )
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=900)
    if r.returncode != 0:
        return {"error": r.stderr[-400:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def _oracle_sample(name, gpu_samples, budget_s):
    import numpy as np
    from lattice_inputs import WORKLOADS, gauge_for
    from oracle import mg as omg
    from oracle import rng
    from oracle import trace as otr
    cfg = dict(WORKLOADS[name], name=name)
    th = gauge_for(cfg)
    hier = omg.setup_hierarchy(th, cfg["m0"], cfg["blocks"], cfg["ntv"], cfg["gauge_seed"] + 17)
    # reduced-form level differences A_l = D_l^-1 - P_l D_{l+1}^-1 P_l^H (the
    # coarsest exact trace belongs to the setup, excluded on both sides)
    ops = []
    for l in range(hier.L - 1):
        fine, coarse, P = hier.levels[l], hier.levels[l + 1], hier.P[l]
        ops.append((lambda X, f=fine, c=coarse, P=P: f.solve(X) - P @ c.solve(P.conj().T @ X),
                    fine.n))
    # warm the sparse LU factorisations (setup, excluded like the GPU setup)
    for lev in hier.levels:
        lev.solve(np.ones((lev.n, 1), dtype=complex))
    noise = cfg["noise"]
    total, parts = 0.0, []
    t_start = time.perf_counter()
    for l, (A, n) in enumerate(ops):
        d = cfg["d"][l]
        t0 = time.perf_counter()
        Q, _ = otr.low_rank(A, n, d, cfg["k_power"], noise, cfg["trace_seed"], l)
        t_lr = time.perf_counter() - t0
        lv = otr.StochLevel(A, n, d, 1.0, Q=Q)
        k = 0
        t0 = time.perf_counter()
        while k < 4 or (time.perf_counter() - t_start < budget_s and k < 64):
            otr.sample(lv, noise, cfg["trace_seed"], l, k)
            k += 1
        t_s = (time.perf_counter() - t0) / k
        total += t_lr + gpu_samples[l] * t_s
        parts.append(dict(level=l, lowrank_s=t_lr, per_sample_s=t_s, timed_samples=k))
    return dict(seconds_per_estimate=total, parts=parts)


def solver_hierarchy(L):
    """4x4 then 2x2 aggregation with 8 test vectors, plus solver-only 2x2
    levels until the coarsest level has at most 1024 dofs."""
    blocks, ntv, N = [(4, 4), (2, 2)], [8, 8], L // 8
    while N * N * 16 > 1024 and N % 4 == 0:
        blocks.append((2, 2))
        ntv.append(8)
        N //= 2
    return blocks, ntv


def run_batch8(args):
    """8 independent fields on 64^2 / 128^2 / 256^2 lattices, 64-256 RHS each
    (1280 RHS), solved to 1e-10 in one mgm_solve_jobs call with autotuned RHS
    blocks, against a per-field loop of mgm_solve_batch on the same GPU."""
    import torch
    from lattice_inputs import links_from_theta
    from lattice_inputs.workloads import BATCH8, batch8_fields
    from paper_2303_11512_amd import Context, mg_params, solve_params
    ctx = Context(0)
    jobs = []
    t0 = time.perf_counter()
    for i, (th, m0, nrhs) in enumerate(batch8_fields()):
        L = th.shape[1]
        blocks, ntv = solver_hierarchy(L)
        gid = ctx.set_gauge(torch.from_numpy(links_from_theta(th)).to("cuda"), m0, True)
        ctx.setup_mg(gid, mg_params(len(blocks) + 1, blocks, ntv, sap_block=[(4, 4)] + COARSE_SAP_BLOCKS,
                                    sap_cycles=list(SAP_CYCLES), inner_iters=[0] * 6, setup_tol=1e-10,
                                    seed=3100 + i))
        n = ctx.level_info(gid, 0)["n"]
        b = torch.empty((nrhs, n), dtype=torch.complex128, device="cuda")
        ctx.noise("z2z2", 7, 0, 0, 0, b)
        jobs.append((gid, 0, b, torch.empty_like(b)))
        print(f"# field {i}: {L}^2, {nrhs} RHS, setup done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    total = sum(j[2].shape[0] for j in jobs)
    plain = solve_params(tol=1e-10, restart=32, max_restarts=50, rhs_block=0)
    tuned = solve_params(tol=1e-10, restart=32, max_restarts=50, rhs_block=-1)
    widths = [ctx.autotune_rhs_block(gid, 0, b.shape[0], tuned) for gid, _, b, _ in jobs]
    # per-field loop (the reference), then the batched call
    for gid, lvl, b, x in jobs:
        ctx.solve_batch(gid, lvl, b, x, plain)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for gid, lvl, b, x in jobs:
            ctx.solve_batch(gid, lvl, b, x, plain)
    torch.cuda.synchronize()
    loop_rate = total * args.steps / (time.perf_counter() - t0)
    ctx.solve_jobs(jobs, tuned)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, its = ctx.solve_jobs(jobs, tuned)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rate = total * args.steps / dt
    # roofline: the fine-level kernels of the largest field at its RHS count
    # (HIP events on the library stream, back to back)
    big = max(range(len(jobs)), key=lambda k: jobs[k][2].shape[0] * jobs[k][2].shape[1])
    gid_b, nrhs_b = jobs[big][0], jobs[big][2].shape[0]
    kern = {k: ctx.time_kernel(gid_b, k, 0, nrhs_b) for k in ("stencil", "sap", "copy")}
    st = kern["stencil"]
    st_gbs = st["bytes"] / (st["us"] * 1e-6) / 1e9
    print(json.dumps({
        "metric": "RHS solves/s (tol 1e-10)", "value": rate, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batch8: 8 quenched U(1) fields (beta, m0, L, nRHS) = "
                               + ", ".join(str(t) for t in BATCH8) + "; MG 4x4 then 2x2, 8 vectors",
                   "per_field_loop_solves_per_s": loop_rate, "speedup_vs_loop": rate / loop_rate,
                   "rhs_blocks": widths, "mean_iters": float(np.mean(its)), "setup_s": setup_s},
        "roofline": {"bound": "hbm", "achieved": st_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": st_gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": f"fine stencil, FP64, field {big} ({nrhs_b} RHS)", "launch_us": st["us"],
                     "alg_bytes": st["bytes"],
                     "others": {k: {"us": round(v["us"], 2), "GB/s": round(v["bytes"] / (v["us"] * 1e-6) / 1e9, 1)}
                                for k, v in kern.items()}},
        "cpu_baseline": None,
    }))
    ctx.close()


MFMA_FP32_PEAK_TFS = 157.3
MFMA_FP16_PEAK_TFS = 2500.0  # dense FP16 matrix-core peak (no sparsity)


def run_mixed(args):
    """Mixed precision at 512^2 (beta 4.0, m0 -0.08): 256 Z2xZ2 RHS solved to
    1e-10 with the FP64, FP32 and FP16-coarse-block preconditioners (outer
    FGMRES FP64 in all), and one MG-MLMC++ estimate to 1e-3 in each."""
    import torch
    from lattice_inputs import WORKLOADS, gauge_for, links_from_theta
    from paper_2303_11512_amd import Context, mg_params, solve_params
    cfg = dict(WORKLOADS["schwinger512"], name="schwinger512")
    th = gauge_for(cfg)
    ctx = Context(0)
    gid = ctx.set_gauge(torch.from_numpy(links_from_theta(th)).to("cuda"), cfg["m0"], True)
    if args.roofline_only:
        # counter runs: the fine stencil and the copy kernel at 512^2, 64 RHS
        # (no multigrid needed)
        out = {k: ctx.time_kernel(gid, k, 0, KERNEL_RHS, reps=5) for k in ("stencil", "copy")}
        print(json.dumps(out))
        ctx.close()
        return
    kw = mg_setup_kwargs(cfg)
    t0 = time.perf_counter()
    ctx.setup_mg(gid, mg_params(**kw))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    print(f"# setup {setup_s:.2f}s, levels {kw['blocks']}", file=sys.stderr, flush=True)
    n = ctx.level_info(gid, 0)["n"]
    nrhs = 256
    b = torch.empty((nrhs, n), dtype=torch.complex128, device="cuda")
    ctx.noise("z2z2", 13, 0, 0, 0, b)
    sp = solve_params(tol=1e-10, restart=16, max_restarts=50, rhs_block=64)
    res = {}
    for prec in ("fp64", "fp32", "fp16"):
        ctx.set_precision(gid, prec)
        x = torch.empty_like(b)
        ctx.solve_batch(gid, 0, b, x, sp)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            _, its, rel = ctx.solve_batch(gid, 0, b, x, sp)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / args.steps
        t1 = time.perf_counter()
        est = ctx.trace_estimate(gid, solve=solve_params(tol=1e-10, restart=16, rhs_block=64),
                                 **trace_kwargs(cfg, 0))
        torch.cuda.synchronize()
        res[prec] = dict(solve_s=dt, solves_per_s=nrhs / dt, iters=float(np.mean(its)),
                         max_relres=float(np.max(rel)), x=x,
                         trace_s=time.perf_counter() - t1, tau=est["tau"],
                         samples=est["level_samples"])
        print(f"# {prec}: {nrhs / dt:.1f} solves/s, {np.mean(its):.2f} it, max relres {np.max(rel):.2e}, "
              f"estimate {est['tau']:.6f} in {res[prec]['trace_s']:.2f}s", file=sys.stderr, flush=True)
    # the fine stencil at this size: 64 RHS are 1.07 GB of input, far beyond
    # the 256 MB Infinity Cache, so this is the HBM-bound figure
    ctx.set_precision(gid, "fp64")
    st = ctx.time_kernel(gid, "stencil", 0, KERNEL_RHS)
    ach = st["bytes"] / (st["us"] * 1e-6) / 1e9
    cp = ctx.time_kernel(gid, "copy", 0, KERNEL_RHS)
    copy_gbs = cp["bytes"] / (cp["us"] * 1e-6) / 1e9
    roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": measured_traffic(path=STENCIL512_SUMMARY),
            "kernel": f"fine stencil, FP64, 512x512, {KERNEL_RHS} RHS",
            "launch_us": st["us"], "alg_bytes": st["bytes"],
            "copy_GBs": copy_gbs, "frac_of_copy": ach / copy_gbs}
    print(f"# stencil 512^2: {st['us']:.1f} us, {ach:.0f} GB/s", file=sys.stderr, flush=True)
    xn = torch.linalg.norm(res["fp64"]["x"])
    tau64 = res["fp64"]["tau"]
    for p in ("fp32", "fp16"):
        res[p]["x_rel_diff_vs_fp64"] = float(torch.linalg.norm(res[p]["x"] - res["fp64"]["x"]) / xn)
        res[p]["tau_rel_diff_vs_fp64"] = abs(res[p]["tau"] - tau64) / abs(tau64)
        res[p]["speedup_vs_fp64"] = res["fp64"]["solve_s"] / res[p]["solve_s"]
    for r in res.values():
        r.pop("x")
        r["tau"] = [r["tau"].real, r["tau"].imag]
    print(json.dumps({
        "metric": "RHS solves/s (tol 1e-10), FP32/FP16 preconditioner in FP64 FGMRES",
        "value": res["fp16"]["solves_per_s"],
        "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": res["fp16"]["solve_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32+f16", "data": "synthetic",
        "config": {"workload": f"mixed512: 512x512 Schwinger, beta {cfg['beta']}, m0 {cfg['m0']}, MG "
                               f"{kw['blocks']} (MLMC closes on level {kw['mlmc_levels'] - 1}), 256 Z2xZ2 RHS "
                               f"in blocks of 64, FGMRES(16) tol 1e-10; one MG-MLMC++ estimate to {cfg['eps']}",
                   "fp64": res["fp64"], "fp32": res["fp32"], "fp16": res["fp16"], "setup_s": setup_s},
        "roofline": roof, "cpu_baseline": None,
    }))
    ctx.close()


def run_cnn(args):
    """Learned preconditioner: train the network on quenched 128^2 fields
    (beta 3.0, m0 -0.10, Z2xZ2 right-hand sides solved to 1e-10 by multigrid),
    then solve 64 RHS on each unseen 256^2 and 512^2 field with multigrid
    alone, from the learned initial guess, and with the network as the first
    stage of every level-0 preconditioner call of the flexible FGMRES
    (multigrid as its fallback).  Per field: time and mean iterations of each
    mode and the gain (plain time / mode time)."""
    import torch
    from lattice_inputs import cnn_init_params, links_from_theta
    from lattice_inputs.cnn import EVAL_FIELDS, TRAIN_FIELDS, field
    from paper_2303_11512_amd import Context, adam_params, mg_params, solve_params
    ctx = Context(0)

    def setup(spec, seed):
        blocks, ntv = solver_hierarchy(spec["L"])
        gid = ctx.set_gauge(torch.from_numpy(links_from_theta(field(spec))).to("cuda"), spec["m0"], True)
        ctx.setup_mg(gid, mg_params(len(blocks) + 1, blocks, ntv, sap_block=[(4, 4)] + COARSE_SAP_BLOCKS,
                                    sap_cycles=list(SAP_CYCLES), inner_iters=[0] * 6, setup_tol=1e-10, seed=seed,
                                    precision=args.precision))
        return gid

    t0 = time.perf_counter()
    train = [setup(s, 6000 + i) for i, s in enumerate(TRAIN_FIELDS[:args.train_fields])]
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    print(f"# {len(train)} training fields set up in {setup_s:.1f}s", file=sys.stderr, flush=True)
    ctx.cnn_set_params(cnn_init_params(1))
    t0 = time.perf_counter()
    losses = ctx.cnn_train(train, pairs_per_field=args.pairs, batch=64, epochs=args.epochs,
                           adam=adam_params(lr=1e-3), seed=5, solve=solve_params(tol=1e-10, restart=32))
    train_s = time.perf_counter() - t0
    print(f"# trained: epoch losses {losses} in {train_s:.1f}s", file=sys.stderr, flush=True)
    conv = ctx.time_kernel(train[0], "conv", 0, 64)
    conv_h = ctx.time_kernel(train[0], "conv_h", 0, 64)
    for gid in train:
        ctx.free_gauge(gid)

    sizes = sorted({s["L"] for s in EVAL_FIELDS})
    evals = [s for L in sizes for s in [e for e in EVAL_FIELDS if e["L"] == L][:args.eval_fields]]
    nrhs = 64
    modes = (("plain", False, "fp16"), ("guess", "guess", "fp16"), ("stage", "stage", "fp16"),
             ("stage_fp32", "stage", "fp32"))
    rows = []
    for i, spec in enumerate(evals):
        gid = setup(spec, 7000 + i)
        n = ctx.level_info(gid, 0)["n"]
        b = torch.empty((nrhs, n), dtype=torch.complex128, device="cuda")
        ctx.noise("z2z2", 11, 0, 0, 0, b)
        x = torch.empty_like(b)
        row = dict(L=spec["L"], seed=spec["seed"])
        for key, use, prec in modes:
            ctx.cnn_set_precision(prec)
            sp = solve_params(tol=1e-10, restart=16, max_restarts=50, use_cnn=use)
            ctx.solve_batch(gid, 0, b, x, sp)   # warm-up (workspaces, graphs)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.steps):
                _, its, rel = ctx.solve_batch(gid, 0, b, x, sp)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t1) / args.steps
            assert float(np.max(rel)) <= 1e-10
            row[key] = dict(s=dt, iters=float(np.mean(its)))
        for key, _, _ in modes[1:]:
            row[key]["gain"] = row["plain"]["s"] / row[key]["s"]
        rows.append(row)
        ctx.free_gauge(gid)
        print(f"# eval {spec['L']}^2 seed {spec['seed']}: " + ", ".join(
            f"{k} {row[k]['iters']:.2f} it {row[k]['s'] * 1e3:.1f} ms" for k, _, _ in modes),
            file=sys.stderr, flush=True)
    total = {k: sum(r[k]["s"] for r in rows) for k, _, _ in modes}
    per_size = {str(L): {k: dict(gain=sum(r["plain"]["s"] for r in rows if r["L"] == L) /
                                 sum(r[k]["s"] for r in rows if r["L"] == L),
                                 iters=float(np.mean([r[k]["iters"] for r in rows if r["L"] == L])))
                         for k, _, _ in modes} for L in sizes}
    achieved = conv_h["flops"] / (conv_h["us"] * 1e-6) / 1e12
    achieved32 = conv["flops"] / (conv["us"] * 1e-6) / 1e12
    print(json.dumps({
        "metric": "RHS solves/s (tol 1e-10), learned network as first FGMRES preconditioner stage",
        "value": nrhs * len(rows) / total["stage"],
        "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": total["stage"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32+f16",
        "data": "synthetic",
        "config": {"workload": f"cnn: train on {len(train)} quenched 128^2 fields (beta 3.0, m0 -0.10, "
                               f"{args.pairs} Z2xZ2 pairs each, {args.epochs} epochs, batch 64, Adam 1e-3); "
                               f"solve 64 RHS on {len(rows)} unseen fields at {sizes}, multigrid "
                               f"preconditioner {args.precision}",
                   "network_precision": "fp16 weights and activations (FP32 accumulation) unless _fp32",
                   "solves_per_s": {k: nrhs * len(rows) / total[k] for k, _, _ in modes},
                   "gain": {k: total["plain"] / total[k] for k, _, _ in modes[1:]},
                   "per_size": per_size,
                   "epoch_losses": losses, "train_s": train_s, "setup_s": setup_s, "fields": rows},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": MFMA_FP16_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": achieved / MFMA_FP16_PEAK_TFS, "traffic": None,
                     "kernel": "k_conv_h<32,32,tanh> (one hidden layer, FP16, 128^2, 64 fields)",
                     "launch_us": conv_h["us"], "alg_flops": conv_h["flops"],
                     "fp32_network": {"kernel": "k_conv<32,32,tanh>", "launch_us": conv["us"],
                                      "TFLOP/s": achieved32, "frac": achieved32 / MFMA_FP32_PEAK_TFS}},
        "cpu_baseline": None,
    }))
    ctx.close()


def run_scan(args):
    """Parameter scan on the 128^2 field (the shapes of the paper's Fig. 2 and
    Fig. 1): for each Wilson mass of `--masses` (the workload's -0.10 and
    values closer to the critical mass, i.e. worse conditioned, as the paper's
    five masses), MG-MLMC (d = 0) and MG-MLMC++ over the number of deflation
    vectors d (the same on every level difference) and block power sweeps k,
    optimal and uniform target variances, and deflated Hutchinson.  Per point:
    the Sec. 4 cost-model work per level difference (MFlop, 8 real flops per
    complex multiply-add), the sample counts and the GPU time per estimate,
    averaged over `--steps` seeds."""
    import torch
    from lattice_inputs import WORKLOADS, gauge_for, links_from_theta
    from paper_2303_11512_amd import Context, MGMError, mg_params, solve_params
    cfg = dict(WORKLOADS["schwinger128"], name="schwinger128")
    ctx = Context(0)
    links = torch.from_numpy(links_from_theta(gauge_for(cfg))).to("cuda")
    sp = solve_params(**SOLVE)
    rows = []
    masses = [float(m) for m in args.masses.split(",")]
    for m0 in masses:
        gid = ctx.set_gauge(links, m0, True)
        try:
            ctx.setup_mg(gid, mg_params(**mg_setup_kwargs(cfg), precision=args.precision))
        except MGMError as e:
            print(f"# m0 {m0}: multigrid setup failed ({e}); mass skipped", file=sys.stderr, flush=True)
            ctx.free_gauge(gid)
            continue

        def point(label, **kw):
            base = dict(method_kwargs(cfg, 0), batch=BATCH)
            base.update(kw)
            try:
                ctx.trace_estimate(gid, solve=sp, **dict(base, seed=cfg["trace_seed"] + 900))  # warm-up
                torch.cuda.synchronize()
                outs = []
                t0 = time.perf_counter()
                for k in range(args.steps):
                    outs.append(ctx.trace_estimate(gid, solve=sp, **dict(base, seed=cfg["trace_seed"] + k)))
                torch.cuda.synchronize()
            except MGMError as e:
                print(f"# m0 {m0} {label}: failed ({e})", file=sys.stderr, flush=True)
                return None
            dt = (time.perf_counter() - t0) / args.steps
            nl = len(outs[0]["level_samples"])
            row = {"m0": m0, "label": label, "ms_per_estimate": dt * 1e3,
                   "d_chosen": [float(np.mean([o["level_d"][l] for o in outs])) for l in range(len(outs[0]["level_d"]))],
                   "samples": [float(np.mean([o["level_samples"][l] for o in outs])) for l in range(nl)],
                   "mflop": [float(np.mean([o["level_work"][l] for o in outs])) * 8e-6 for l in range(nl)],
                   "mflop_lowrank": [float(np.mean([o["level_lr_work"][l] for o in outs])) * 8e-6 for l in range(nl)],
                   "iters_per_solve": [round(sum(o["iters"][l] for o in outs) / max(1, sum(o["solves"][l] for o in outs)), 2)
                                       for l in range(2)],
                   "tau_mean": float(np.mean([o["tau"].real for o in outs]))}
            row["mflop_total"] = sum(row["mflop"])
            rows.append(row)
            print(f"# m0 {m0} {label}: {dt * 1e3:.1f} ms, samples {[round(v, 1) for v in row['samples']]}, "
                  f"MFlop {row['mflop_total']:.0f}, iters {row['iters_per_solve']}", file=sys.stderr, flush=True)
            return row

        pts = [point("mlmc optimal", variant="mlmc", d=[0, 0]), point("mlmc uniform", variant="mlmc", d=[0, 0],
                                                                      targets="uniform")]
        for kp in (1, 2):
            for d in (8, 32, 64):
                pts.append(point(f"mlmcpp d={d} k={kp} optimal", d=[d, d], k_power=kp))
        pp = [r for r in pts[2:] if r]
        if pp:
            best = min(pp, key=lambda r: r["mflop_total"])
            bd = int(best["label"].split("d=")[1].split()[0])
            bk = int(best["label"].split("k=")[1].split()[0])
            point(f"mlmcpp d={bd} k={bk} uniform", d=[bd, bd], k_power=bk, targets="uniform")
        for kp in (1, 2):
            point(f"mlmcpp adaptive d (from 4, <= 64, 16 pilots) k={kp} optimal", d=[4, 4], k_power=kp, d_max=64,
                  pilot=16)
        for d in (32, 64):
            point(f"deflated hutchinson k={d} (3 sweeps)", variant="deflated", d=[d], k_power=3)
        ctx.free_gauge(gid)
    ref = [r for r in rows if r["m0"] == masses[0] and r["label"].startswith("mlmcpp d=32 k=2 optimal")]
    print(json.dumps({
        "metric": "Sec. 4 cost-model MFlop and GPU time per trace estimate at 1e-3 (parameter scan)",
        "value": ref[0]["mflop_total"] if ref else None, "unit": "MFlop (MG-MLMC++ d=32 k=2, first mass)",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": ref[0]["ms_per_estimate"] if ref else None,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32+f16",
        "data": "synthetic",
        "config": {"workload": f"scan128: {cfg['Lx']}x{cfg['Lt']} Schwinger field of the 128^2 workload (beta "
                               f"{cfg['beta']}), masses {masses}, 3-level MG, {cfg['noise']} noise, eps {cfg['eps']}, "
                               f"preconditioner {args.precision}", "points": rows},
        "roofline": None, "cpu_baseline": None}))
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="schwinger128")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--precision", default="fp16", choices=["fp64", "fp32", "fp16"],
                    help="precision of the multigrid preconditioner (outer FGMRES is FP64); fp16 = "
                         "FP32 cycle with FP16 coarse blocks")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the FP64 comparison runs reported next to the value")
    ap.add_argument("--plain-steps", type=int, default=1,
                    help="estimates timed with plain FP64 MG-FGMRES, one sample at a time (0: skip)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="set up, time the hot kernels and exit (for counter runs)")
    ap.add_argument("--train-fields", type=int, default=20, help="cnn workload: training fields")
    ap.add_argument("--pairs", type=int, default=1000, help="cnn workload: pairs per training field")
    ap.add_argument("--epochs", type=int, default=4, help="cnn workload: training epochs")
    ap.add_argument("--eval-fields", type=int, default=8, help="cnn workload: unseen fields per size")
    ap.add_argument("--ensemble", type=int, default=3,
                    help="fields estimated at once in the ensemble comparison (0 or 1: skip)")
    ap.add_argument("--masses", default="-0.10,-0.12,-0.13,-0.14",
                    help="scan128 workload: Wilson masses of the scan")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library drives one GPU per process; --gpus must be 1 (multi-GPU sharding is not built)"}))
        sys.exit(2)
    if args.workload == "batch8":
        run_batch8(args)
        return
    if args.workload == "cnn":
        run_cnn(args)
        return
    if args.workload == "mixed512":
        run_mixed(args)
        return
    if args.workload == "scan128":
        run_scan(args)
        return

    import torch
    from lattice_inputs import WORKLOADS, gauge_for, links_from_theta
    from paper_2303_11512_amd import Context, mg_params, solve_params

    cfg = dict(WORKLOADS[args.workload], name=args.workload)
    th = gauge_for(cfg)
    ctx = Context(0)
    gid = ctx.set_gauge(torch.from_numpy(links_from_theta(th)).to("cuda"), cfg["m0"], True)
    t0 = time.perf_counter()
    mgkw = mg_setup_kwargs(cfg)
    if args.roofline_only:
        # counter runs: skip the dense inverse of the MLMC-closing level (only
        # the timed kernels matter; the profiler struggles with its ~16k
        # Gauss-Jordan dispatches)
        mgkw["mlmc_levels"] = 0
    ctx.setup_mg(gid, mg_params(**mgkw, precision=args.precision))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    print(f"# setup done in {setup_s:.2f}s", file=sys.stderr, flush=True)
    mlmc_coarsest = len(cfg["blocks"])
    if args.roofline_only:
        print(json.dumps(kernel_table(ctx, gid, precision=args.precision)))
        ctx.close()
        return

    sp = solve_params(**SOLVE)
    for w in range(args.warmup):
        ctx.trace_estimate(gid, solve=sp, **trace_kwargs(cfg, 1000 + w))
        print(f"# warmup {w} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = []
    for k in range(args.steps):
        # a named range per step, so that a profiler's kernel trace can be
        # cut into steps (roctx; no cost without a profiler)
        torch.cuda.nvtx.range_push(f"timed step {k}")
        outs.append(ctx.trace_estimate(gid, solve=sp, **trace_kwargs(cfg, k)))
        torch.cuda.nvtx.range_pop()
        print(f"# step {k}: tau={outs[-1]['tau']:.6f} samples={outs[-1]['level_samples']}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    solves = sum(sum(o["solves"]) for o in outs)

    kern = kernel_table(ctx, gid, mlmc_coarsest=mlmc_coarsest, precision=args.precision)
    dom_key = DOMINANT[args.precision]
    dom = kern[dom_key]
    achieved = dom["bytes"] / (dom["us"] * 1e-6) / 1e9

    # spread of the timed estimates (each an independent estimate to eps)
    taus = np.array([o["tau"] for o in outs])
    tau_mean = complex(np.mean(taus))
    spread = {"mean": [tau_mean.real, tau_mean.imag],
              "rel_std": float(np.std(np.abs(taus - tau_mean)) / abs(tau_mean)) if len(outs) > 1 else None,
              "rel_rms_dev": float(np.sqrt(np.mean(np.abs(taus - tau_mean) ** 2)) / abs(tau_mean)),
              "max_rel_dev": float(np.max(np.abs(taus - tau_mean)) / abs(tau_mean)),
              "samples_per_step": [o["level_samples"] for o in outs],
              "cost_model_mflop_per_step": [round(sum(o["level_work"]) * 8e-6, 1) for o in outs]}

    # the same estimates with only the preconditioner's precision changed to
    # FP64 (same schedule: phase-batched level solves, two streams, graphs)
    plain = None
    unbatched = None
    if args.precision != "fp64" and not args.no_compare:
        ctx.set_precision(gid, "fp64")
        ctx.trace_estimate(gid, solve=sp, **trace_kwargs(cfg, 1000))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pouts = [ctx.trace_estimate(gid, solve=sp, **trace_kwargs(cfg, k)) for k in range(args.steps)]
        torch.cuda.synchronize()
        pdt = time.perf_counter() - t1
        plain = {"what": "precision-only comparison: FP64 preconditioner, same batched schedule",
                 "estimates_per_s": args.steps / pdt, "ms_per_step": pdt / args.steps * 1e3,
                 "max_tau_rel_diff": max(abs(a["tau"] - b["tau"]) / abs(b["tau"]) for a, b in zip(outs, pouts))}
        ctx.set_precision(gid, args.precision)
        print(f"# FP64 preconditioner, same schedule: {plain}", file=sys.stderr, flush=True)
        if args.plain_steps > 0:
            unbatched = plain_fp64_run(ctx, th, cfg, mgkw, args.plain_steps, outs)
            print(f"# plain FP64 MG-FGMRES, one sample at a time: {unbatched}", file=sys.stderr, flush=True)

    ensemble = None
    if not args.no_compare and args.ensemble > 1:
        ensemble = ensemble_run(ctx, cfg, mgkw, args)
        print(f"# ensemble: {ensemble}", file=sys.stderr, flush=True)

    samples = [int(sum(o["level_samples"][l] for o in outs) / len(outs)) for l in range(len(outs[0]["level_samples"]))]
    cpu = None
    if not args.no_cpu:
        cb = cpu_baseline(cfg, samples)
        if "seconds_per_estimate" in cb:
            cpu = {"value": 1.0 / cb["seconds_per_estimate"], "unit": "trace estimates/s", "cores": 1,
                   "kind": "oracle",
                   "sample": "oracle Hutch++ phase per level in full + >=4 stochastic samples per level "
                             "(1 thread), scaled to the GPU run's mean per-level sample counts; setup "
                             "and coarsest inverse excluded on both sides",
                   "detail": cb["parts"]}
        else:
            cpu = {"error": cb.get("error")}
    line = {
        "metric": "trace estimates/s at 1e-3 rel. accuracy",
        "value": args.steps / dt,
        "unit": "trace estimates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f64+f32", "fp16": "f64+f32+f16"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {cfg['Lx']}x{cfg['Lt']} Schwinger, beta {cfg['beta']}, "
                               f"m0 {cfg['m0']}, {len(cfg['blocks']) + 1}-level MG, Hutch++ d={cfg['d']}, "
                               f"{cfg['noise']} noise, eps {cfg['eps']}, FGMRES tol 1e-10",
                   "solves_per_s": solves / dt, "setup_s": setup_s,
                   "preconditioner": args.precision, "sap_cycles": list(SAP_CYCLES[:4]),
                   "sap_blocks": [list(b) for b in mg_setup_kwargs(cfg)["sap_block"][:3]],
                   "min_samples": MIN_SAMPLES, "cost_model": "flops (Sec. 4)", "estimates": spread,
                   "fp64_preconditioner_same_schedule": plain,
                   "plain_fp64_mg_fgmres": unbatched,
                   "ensemble_concurrent": ensemble,
                   "solver_levels": mg_setup_kwargs(cfg)["nlevels"],
                   "iters_per_solve": [round(sum(o["iters"][l] for o in outs) / max(1, sum(o["solves"][l] for o in outs)), 2)
                                       for l in range(len(cfg["blocks"]) + 1)],
                   "level_samples": samples, "tau": [outs[-1]["tau"].real, outs[-1]["tau"].imag]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.precision),
                     "kernel": f"{KERNEL_NAME[args.precision]} (level 1, one colour, {KERNEL_RHS} RHS)",
                     "launch_us": dom["us"], "alg_bytes": dom["bytes"],
                     "in_step": in_step_average(args.precision, dom["bytes"]),
                     "others": {k: {"us": round(v["us"], 2),
                                    "GB/s": round(v["bytes"] / (v["us"] * 1e-6) / 1e9, 1),
                                    "TFLOP/s": round(v["flops"] / (v["us"] * 1e-6) / 1e12, 2)}
                                for k, v in kern.items() if k != dom_key}},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))
    ctx.close()


if __name__ == "__main__":
    main()
