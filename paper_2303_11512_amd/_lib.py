"""ctypes binding of libmgmlmc.so (the C ABI in include/mgmlmc.h).

Argument marshalling only: every computation runs in the HIP library.  Device
vectors are torch complex128 CUDA tensors of shape (nrhs, n); the library
enqueues its work on torch's current stream.  If the shared library is missing
the import fails loudly -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgmlmc.so")

MAX_LEVELS = 6
OK, EINVAL, ENOMEM, EHIP, ESTATE, ENOTCONV, ENONFINITE = 0, -1, -2, -3, -4, -5, -6
NOISE_RADEMACHER, NOISE_Z2Z2 = 0, 1
PURPOSE_SETUP, PURPOSE_SKETCH, PURPOSE_SAMPLE, PURPOSE_TRAIN, PURPOSE_DEFLATE = 1, 2, 3, 4, 5
PREC_FP64, PREC_FP32, PREC_FP16 = 0, 1, 2
PRECISIONS = {"fp64": PREC_FP64, "fp32": PREC_FP32, "fp16": PREC_FP16}
VARIANTS = {"hutchinson": 0, "hutchpp": 1, "mlmc": 2, "mlmcpp": 3, "deflated": 4}
FORMS = {"reduced": 0, "full": 1}
TARGETS = {"optimal": 0, "uniform": 1}
COSTS = {"static": 0, "fixed": 1, "flops": 2}
NOISES = {"rademacher": NOISE_RADEMACHER, "z2z2": NOISE_Z2Z2}


class MGParams(C.Structure):
    _fields_ = [
        ("nlevels", C.c_int),
        ("block", (C.c_int * 2) * MAX_LEVELS),
        ("ntv", C.c_int * MAX_LEVELS),
        ("sap_block", (C.c_int * 2) * MAX_LEVELS),
        ("sap_cycles", C.c_int * MAX_LEVELS),
        ("inner_iters", C.c_int * MAX_LEVELS),
        ("inner_tol", C.c_double),
        ("setup_iters", C.c_int),
        ("setup_tol", C.c_double),
        ("setup_restart", C.c_int),
        ("setup_max_restarts", C.c_int),
        ("seed", C.c_uint64),
        ("precision", C.c_int),
        ("mlmc_levels", C.c_int),
        ("graphs", C.c_int),
    ]


class SolveParams(C.Structure):
    _fields_ = [
        ("tol", C.c_double),
        ("restart", C.c_int),
        ("max_restarts", C.c_int),
        ("rhs_block", C.c_int),
        ("use_cnn", C.c_int),
    ]


class AdamParams(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double)]


class CnnTrainParams(C.Structure):
    _fields_ = [
        ("pairs_per_field", C.c_int),
        ("batch", C.c_int),
        ("epochs", C.c_int),
        ("adam", AdamParams),
        ("seed", C.c_uint64),
        ("solve", SolveParams),
    ]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.POINTER(C.c_int)), ("relres", C.POINTER(C.c_double))]


class TraceParams(C.Structure):
    _fields_ = [
        ("variant", C.c_int),
        ("form", C.c_int),
        ("eps", C.c_double),
        ("d", C.c_int * MAX_LEVELS),
        ("k_power", C.c_int),
        ("noise", C.c_int),
        ("targets", C.c_int),
        ("cost", C.c_int),
        ("fixed_cost", C.c_double * MAX_LEVELS),
        ("min_samples", C.c_int),
        ("max_samples", C.c_int),
        ("fixed_samples", C.POINTER(C.c_int)),
        ("seed", C.c_uint64),
        ("batch", C.c_int),
        ("solve", SolveParams),
        ("d_max", C.c_int),
        ("pilot", C.c_int),
        ("projection", C.c_int),
        ("concurrent", C.c_int),
    ]


class TraceResult(C.Structure):
    _fields_ = [
        ("tau", C.c_double * 2),
        ("tau_exact", C.c_double * 2),
        ("nstoch", C.c_int),
        ("lvl_mean", (C.c_double * 2) * MAX_LEVELS),
        ("lvl_lr", (C.c_double * 2) * MAX_LEVELS),
        ("lvl_var", C.c_double * MAX_LEVELS),
        ("lvl_cost", C.c_double * MAX_LEVELS),
        ("lvl_samples", C.c_int * MAX_LEVELS),
        ("lvl_solves", C.c_int64 * MAX_LEVELS),
        ("lvl_iters", C.c_int64 * MAX_LEVELS),
        ("lvl_lr_work", C.c_double * MAX_LEVELS),
        ("lvl_work", C.c_double * MAX_LEVELS),
        ("sample_dump", C.POINTER(C.c_double)),
        ("cost_dump", C.POINTER(C.c_double)),
        ("lvl_d", C.c_int * MAX_LEVELS),
        ("defl_ritz", C.c_double * 2),
        ("sigma_dump", C.POINTER(C.c_double)),
        ("iter_dump", C.POINTER(C.c_int)),
        ("max_dump", C.c_int),
    ]


# exported entry points: name -> (restype, argtypes)
_P = C.c_void_p
SIGNATURES = {
    "mgm_create": (C.c_int, [C.POINTER(_P), C.c_int, _P]),
    "mgm_destroy": (None, [_P]),
    "mgm_last_error": (C.c_char_p, [_P]),
    "mgm_set_gauge": (C.c_int, [_P, C.c_int, C.c_int, _P, C.c_double, C.c_int, C.POINTER(C.c_int)]),
    "mgm_setup_mg": (C.c_int, [_P, C.c_int, C.POINTER(MGParams)]),
    "mgm_free_gauge": (C.c_int, [_P, C.c_int]),
    "mgm_set_precision": (C.c_int, [_P, C.c_int, C.c_int]),
    "mgm_level_info": (C.c_int, [_P, C.c_int, C.c_int, C.POINTER(C.c_int)]),
    "mgm_apply_D": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, _P, _P]),
    "mgm_apply_P": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, _P, _P]),
    "mgm_apply_R": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, _P, _P]),
    "mgm_precondition": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, _P, _P]),
    "mgm_get_prolongator": (C.c_int, [_P, C.c_int, C.c_int, _P]),
    "mgm_coarsest_trace": (C.c_int, [_P, C.c_int, C.POINTER(C.c_double)]),
    "mgm_solve_batch": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, _P, _P, C.POINTER(SolveParams),
                                  C.POINTER(SolveStats)]),
    "mgm_noise": (C.c_int, [_P, C.c_int, C.c_uint64, C.c_int, C.c_int, C.c_int64, C.c_int64, C.c_int,
                            _P]),
    "mgm_orthonormalize": (C.c_int, [_P, C.c_int64, C.c_int, _P, _P]),
    "mgm_orthonormalize_noalloc": (C.c_int, [_P, C.c_int64, C.c_int, _P, _P]),
    "mgm_trace_estimate": (C.c_int, [_P, C.c_int, C.POINTER(TraceParams), C.POINTER(TraceResult)]),
    "mgm_trace_jobs": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(TraceParams),
                                 C.POINTER(TraceResult)]),
    "mgm_time_kernel": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                  C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "mgm_solve_jobs": (C.c_int, [_P, C.c_int, _P, C.POINTER(SolveParams), C.POINTER(C.c_int)]),
    "mgm_autotune_rhs_block": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, C.POINTER(SolveParams),
                                         C.POINTER(C.c_int)]),
    "mgm_cnn_set_params": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "mgm_cnn_get_params": (C.c_int, [_P, C.POINTER(C.c_float)]),
    "mgm_cnn_set_precision": (C.c_int, [_P, C.c_int]),
    "mgm_cnn_apply": (C.c_int, [_P, C.c_int, C.c_int, _P, _P]),
    "mgm_cnn_loss_grad": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, C.POINTER(C.c_double),
                                    C.POINTER(C.c_float)]),
    "mgm_cnn_train_step": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, C.POINTER(AdamParams),
                                     C.POINTER(C.c_double)]),
    "mgm_cnn_train": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(CnnTrainParams),
                                C.POINTER(C.c_double)]),
}

CNN_NPARAMS = 20836


class Job(C.Structure):
    _fields_ = [("gauge_id", C.c_int), ("level", C.c_int), ("nrhs", C.c_int),
                ("b", C.c_void_p), ("x", C.c_void_p)]

KERNELS = {"stencil": 0, "sap": 1, "dense": 2, "cgs": 3, "copy": 4, "conv": 5, "sap_low": 6, "conv_h": 7, "dense_low": 8}

_lib = None


def load_library(path: str = LIB_PATH) -> C.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_2303_11512_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class MGMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _ptr(t) -> int:
    return t.data_ptr()


def _check_vec(t, n: int | None = None):
    import torch
    if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
        raise ValueError("vectors must be contiguous complex128 CUDA tensors")
    if n is not None and (t.dim() != 2 or t.shape[1] != n):
        raise ValueError(f"expected shape (nrhs, {n}), got {tuple(t.shape)}")


def mg_params(nlevels, blocks, ntv, sap_block=None, sap_cycles=None, inner_iters=None,
              inner_tol=0.0, setup_iters=3, setup_tol=1e-12, setup_restart=32,
              setup_max_restarts=200, seed=1, precision="fp64", mlmc_levels=0,
              graphs=True) -> MGParams:
    p = MGParams()
    p.nlevels = nlevels
    p.mlmc_levels = mlmc_levels
    p.graphs = int(bool(graphs))
    for l, (bx, bt) in enumerate(blocks):
        p.block[l][0], p.block[l][1] = bx, bt
    for l, v in enumerate(ntv):
        p.ntv[l] = v
    sap_block = sap_block or [blocks[0]] + [(1, 1)] * (MAX_LEVELS - 1)
    for l, (bx, bt) in enumerate(sap_block[:MAX_LEVELS]):
        p.sap_block[l][0], p.sap_block[l][1] = bx, bt
    for l, v in enumerate((sap_cycles or [2] * MAX_LEVELS)[:MAX_LEVELS]):
        p.sap_cycles[l] = v
    for l, v in enumerate((inner_iters or [8] * MAX_LEVELS)[:MAX_LEVELS]):
        p.inner_iters[l] = v
    p.inner_tol = inner_tol
    p.setup_iters = setup_iters
    p.setup_tol = setup_tol
    p.setup_restart = setup_restart
    p.setup_max_restarts = setup_max_restarts
    p.seed = seed
    p.precision = PRECISIONS[precision]
    return p


CNN_USES = {False: 0, None: 0, True: 1, 2: 2, 3: 3, "guess": 1, "stage": 2, "both": 3}


def solve_params(tol=1e-10, restart=16, max_restarts=50, rhs_block=0, use_cnn=False) -> SolveParams:
    """use_cnn: False, True / "guess" (learned initial guess), "stage" (learned
    first stage of every level-0 preconditioner call) or "both"."""
    if use_cnn not in CNN_USES:
        raise ValueError(f"use_cnn must be one of {list(CNN_USES)}")
    return SolveParams(tol, restart, max_restarts, rhs_block, CNN_USES[use_cnn])


def adam_params(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8) -> AdamParams:
    return AdamParams(lr, beta1, beta2, eps)


class Context:
    """One library context on a CUDA (HIP) device, on torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load_library()
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        h = _P()
        st = self.lib.mgm_create(C.byref(h), device, _P(stream))
        if st != OK:
            raise MGMError(st, "mgm_create failed")
        self.h = h
        self.levels = {}

    def close(self):
        if getattr(self, "h", None):
            self.lib.mgm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st: int, what: str):
        if st != OK:
            msg = self.lib.mgm_last_error(self.h)
            raise MGMError(st, f"{what}: {msg.decode() if msg else ''}")
        return st

    # -- calls of the C ABI -------------------------------------------------
    def set_gauge(self, links, m0: float, bc_t_anti: bool = True) -> int:
        """links: complex128 CUDA tensor [2][Lt][Lx]."""
        import torch
        if not (links.is_cuda and links.dtype == torch.complex128 and links.is_contiguous()
                and links.dim() == 3 and links.shape[0] == 2):
            raise ValueError("links must be a contiguous complex128 CUDA tensor [2][Lt][Lx]")
        gid = C.c_int()
        _, Lt, Lx = links.shape
        self._chk(self.lib.mgm_set_gauge(self.h, Lx, Lt, _P(_ptr(links)), float(m0),
                                         int(bool(bc_t_anti)), C.byref(gid)), "set_gauge")
        return gid.value

    def set_precision(self, gid, precision: str):
        self._chk(self.lib.mgm_set_precision(self.h, gid, PRECISIONS[precision]),
                  "set_precision")

    def free_gauge(self, gid):
        self._chk(self.lib.mgm_free_gauge(self.h, gid), "free_gauge")

    def setup_mg(self, gid: int, prm: MGParams):
        self._chk(self.lib.mgm_setup_mg(self.h, gid, C.byref(prm)), "setup_mg")

    def level_info(self, gid: int, level: int):
        info = (C.c_int * 4)()
        self._chk(self.lib.mgm_level_info(self.h, gid, level, info), "level_info")
        return dict(Nx=info[0], Nt=info[1], M=info[2], n=info[3])

    def apply_D(self, gid, level, x, y):
        n = self.level_info(gid, level)["n"]
        _check_vec(x, n)
        _check_vec(y, n)
        self._chk(self.lib.mgm_apply_D(self.h, gid, level, x.shape[0], _P(_ptr(x)), _P(_ptr(y))),
                  "apply_D")

    def apply_P(self, gid, level, x, y):
        self._chk(self.lib.mgm_apply_P(self.h, gid, level, x.shape[0], _P(_ptr(x)), _P(_ptr(y))),
                  "apply_P")

    def apply_R(self, gid, level, x, y):
        self._chk(self.lib.mgm_apply_R(self.h, gid, level, x.shape[0], _P(_ptr(x)), _P(_ptr(y))),
                  "apply_R")

    def precondition(self, gid, level, r, x):
        self._chk(self.lib.mgm_precondition(self.h, gid, level, r.shape[0], _P(_ptr(r)), _P(_ptr(x))),
                  "precondition")

    def get_prolongator(self, gid, level, out):
        self._chk(self.lib.mgm_get_prolongator(self.h, gid, level, _P(_ptr(out))), "get_prolongator")

    def coarsest_trace(self, gid) -> complex:
        out = (C.c_double * 2)()
        self._chk(self.lib.mgm_coarsest_trace(self.h, gid, out), "coarsest_trace")
        return complex(out[0], out[1])

    def solve_batch(self, gid, level, b, x, prm: SolveParams | None = None, stats: bool = True,
                    check: bool = True):
        prm = prm or solve_params()
        nrhs = b.shape[0]
        its = (C.c_int * nrhs)()
        rel = (C.c_double * nrhs)()
        st_obj = SolveStats(C.cast(its, C.POINTER(C.c_int)), C.cast(rel, C.POINTER(C.c_double)))
        st = self.lib.mgm_solve_batch(self.h, gid, level, nrhs, _P(_ptr(b)), _P(_ptr(x)), C.byref(prm),
                                      C.byref(st_obj) if stats else None)
        if check:
            self._chk(st, "solve_batch")
        return st, np.array(its[:]), np.array(rel[:])

    def solve_jobs(self, jobs, prm: SolveParams | None = None, check: bool = True):
        """jobs: list of (gauge_id, level, b, x) with b, x device tensors
        (nrhs, n_level).  Returns (status, iterations per RHS in job order)."""
        prm = prm or solve_params()
        arr = (Job * len(jobs))()
        total = 0
        for k, (gid, level, b, x) in enumerate(jobs):
            _check_vec(b)
            _check_vec(x)
            arr[k] = Job(gid, level, b.shape[0], _ptr(b), _ptr(x))
            total += b.shape[0]
        its = (C.c_int * max(1, total))()
        st = self.lib.mgm_solve_jobs(self.h, len(jobs), C.cast(arr, _P), C.byref(prm), its)
        if check:
            self._chk(st, "solve_jobs")
        return st, np.array(its[:total])

    def autotune_rhs_block(self, gid, level, nrhs, prm: SolveParams | None = None) -> int:
        prm = prm or solve_params()
        best = C.c_int()
        self._chk(self.lib.mgm_autotune_rhs_block(self.h, gid, level, nrhs, C.byref(prm),
                                                  C.byref(best)), "autotune_rhs_block")
        return best.value

    def noise(self, kind, seed, purpose, level, index0, out):
        k = NOISES[kind] if isinstance(kind, str) else kind
        self._chk(self.lib.mgm_noise(self.h, k, C.c_uint64(seed), purpose, level, index0,
                                     out.shape[1], out.shape[0], _P(_ptr(out))), "noise")

    def time_kernel(self, gid, kind, level, nrhs, reps=50) -> dict:
        """Average launch duration (us), algorithmic bytes and flops of one
        kernel of the path, timed with HIP events on the library's stream."""
        us, by, fl = C.c_double(), C.c_double(), C.c_double()
        self._chk(self.lib.mgm_time_kernel(self.h, gid, KERNELS[kind], level, nrhs, reps, C.byref(us),
                                           C.byref(by), C.byref(fl)), "time_kernel")
        return dict(us=us.value, bytes=by.value, flops=fl.value)

    # ------------------------------------------------------------ learned guess
    def cnn_set_params(self, theta):
        import numpy as np
        th = np.ascontiguousarray(theta, dtype=np.float32)
        if th.shape != (CNN_NPARAMS,):
            raise ValueError(f"expected {CNN_NPARAMS} parameters, got {th.shape}")
        self._chk(self.lib.mgm_cnn_set_params(self.h, th.ctypes.data_as(C.POINTER(C.c_float))),
                  "cnn_set_params")

    def cnn_set_precision(self, precision: str):
        self._chk(self.lib.mgm_cnn_set_precision(self.h, PRECISIONS[precision]), "cnn_set_precision")

    def cnn_get_params(self):
        import numpy as np
        th = np.empty(CNN_NPARAMS, dtype=np.float32)
        self._chk(self.lib.mgm_cnn_get_params(self.h, th.ctypes.data_as(C.POINTER(C.c_float))),
                  "cnn_get_params")
        return th

    def cnn_apply(self, gid, b, y):
        _check_vec(b)
        _check_vec(y, b.shape[1])
        self._chk(self.lib.mgm_cnn_apply(self.h, gid, b.shape[0], _P(_ptr(b)), _P(_ptr(y))), "cnn_apply")

    def cnn_loss_grad(self, gid, b, x):
        """(loss, gradient as float32 numpy array in the parameter packing)."""
        import numpy as np
        _check_vec(b)
        _check_vec(x, b.shape[1])
        loss = C.c_double()
        g = np.empty(CNN_NPARAMS, dtype=np.float32)
        self._chk(self.lib.mgm_cnn_loss_grad(self.h, gid, b.shape[0], _P(_ptr(b)), _P(_ptr(x)),
                                             C.byref(loss), g.ctypes.data_as(C.POINTER(C.c_float))),
                  "cnn_loss_grad")
        return loss.value, g

    def cnn_train_step(self, gid, b, x, adam: AdamParams | None = None) -> float:
        _check_vec(b)
        _check_vec(x, b.shape[1])
        loss = C.c_double()
        self._chk(self.lib.mgm_cnn_train_step(self.h, gid, b.shape[0], _P(_ptr(b)), _P(_ptr(x)),
                                              C.byref(adam or adam_params()), C.byref(loss)),
                  "cnn_train_step")
        return loss.value

    def cnn_train(self, gids, pairs_per_field, batch, epochs, adam: AdamParams | None = None, seed=1,
                  solve: SolveParams | None = None):
        """Per-epoch mean losses of training on the fields' own MG solves."""
        prm = CnnTrainParams(pairs_per_field, batch, epochs, adam or adam_params(), C.c_uint64(seed),
                             solve or solve_params())
        ids = (C.c_int * len(gids))(*gids)
        out = (C.c_double * max(1, epochs))()
        self._chk(self.lib.mgm_cnn_train(self.h, len(gids), ids, C.byref(prm), out), "cnn_train")
        return [out[i] for i in range(epochs)]

    def orthonormalize(self, Y, Q):
        self._chk(self.lib.mgm_orthonormalize(self.h, Y.shape[1], Y.shape[0], _P(_ptr(Y)),
                                              _P(_ptr(Q))), "orthonormalize")

    def orthonormalize_noalloc(self, Y, Q):
        """As orthonormalize, in the library's static workspace (no device
        allocation; n * d <= 2^20)."""
        self._chk(self.lib.mgm_orthonormalize_noalloc(self.h, Y.shape[1], Y.shape[0], _P(_ptr(Y)),
                                                      _P(_ptr(Q))), "orthonormalize_noalloc")

    @staticmethod
    def _trace_in(variant="mlmcpp", form="reduced", eps=1e-2, d=(), k_power=2, noise="z2z2",
                  targets="optimal", cost="static", fixed_cost=None, min_samples=2, max_samples=0,
                  fixed_samples=None, seed=1, batch=64, solve=None, max_dump=0, concurrent=True,
                  projection="one-sided", d_max=0, pilot=16):
        """Parameter and result structs of one estimate plus the host buffers
        they point to (kept alive by the caller until the call returns)."""
        p = TraceParams()
        p.variant = VARIANTS[variant]
        p.form = FORMS[form]
        p.eps = eps
        for i, v in enumerate(d):
            p.d[i] = v
        p.k_power = k_power
        p.noise = NOISES[noise]
        p.targets = TARGETS[targets]
        p.cost = COSTS["fixed" if fixed_cost is not None else cost]
        if fixed_cost is not None:
            for i, v in enumerate(fixed_cost):
                p.fixed_cost[i] = v
        p.min_samples = min_samples
        p.max_samples = max_samples
        keep = {}
        if fixed_samples is not None:
            keep["fs"] = (C.c_int * len(fixed_samples))(*fixed_samples)
            p.fixed_samples = C.cast(keep["fs"], C.POINTER(C.c_int))
        p.seed = seed
        p.batch = batch
        p.solve = solve or solve_params()
        p.concurrent = int(bool(concurrent))
        p.projection = {"one-sided": 0, "two-sided": 1}[projection]
        p.d_max = d_max
        p.pilot = pilot
        r = TraceResult()
        if variant == "deflated" and len(d) > 0 and d[0] > 0:
            keep["sig"] = (C.c_double * d[0])()
            r.sigma_dump = C.cast(keep["sig"], C.POINTER(C.c_double))
        if max_dump > 0:
            keep["dump"] = (C.c_double * (MAX_LEVELS * max_dump * 2))()
            keep["cdump"] = (C.c_double * (MAX_LEVELS * max_dump))()
            keep["idump"] = (C.c_int * (MAX_LEVELS * max_dump * 2))()
            r.sample_dump = C.cast(keep["dump"], C.POINTER(C.c_double))
            r.cost_dump = C.cast(keep["cdump"], C.POINTER(C.c_double))
            r.iter_dump = C.cast(keep["idump"], C.POINTER(C.c_int))
            r.max_dump = max_dump
        return p, r, keep

    @staticmethod
    def _trace_out(r, keep) -> dict:
        ns = r.nstoch
        out = dict(
            tau=complex(r.tau[0], r.tau[1]),
            tau_exact=complex(r.tau_exact[0], r.tau_exact[1]),
            level_mean=[complex(r.lvl_mean[i][0], r.lvl_mean[i][1]) for i in range(ns)],
            level_lr=[complex(r.lvl_lr[i][0], r.lvl_lr[i][1]) for i in range(ns)],
            level_var=[r.lvl_var[i] for i in range(ns)],
            level_cost=[r.lvl_cost[i] for i in range(ns)],
            level_samples=[r.lvl_samples[i] for i in range(ns)],
            solves=[r.lvl_solves[i] for i in range(MAX_LEVELS)],
            iters=[r.lvl_iters[i] for i in range(MAX_LEVELS)],
            level_d=[r.lvl_d[i] for i in range(ns)],
            level_lr_work=[r.lvl_lr_work[i] for i in range(ns)],
            level_work=[r.lvl_work[i] for i in range(ns)],
        )
        if "sig" in keep:
            out["defl_ritz"] = complex(r.defl_ritz[0], r.defl_ritz[1])
            out["sigma"] = np.array(keep["sig"][:])
        if "dump" in keep:
            max_dump = r.max_dump
            arr = np.frombuffer(keep["dump"], dtype=np.float64).reshape(MAX_LEVELS, max_dump, 2)
            out["samples"] = [
                (arr[i, :min(max_dump, out["level_samples"][i]), 0]
                 + 1j * arr[i, :min(max_dump, out["level_samples"][i]), 1]).copy()
                for i in range(ns)
            ]
            carr = np.frombuffer(keep["cdump"], dtype=np.float64).reshape(MAX_LEVELS, max_dump)
            iarr = np.frombuffer(keep["idump"], dtype=np.int32).reshape(MAX_LEVELS, max_dump, 2)
            out["sample_costs"] = [carr[i, :min(max_dump, out["level_samples"][i])].copy() for i in range(ns)]
            out["sample_iters"] = [iarr[i, :min(max_dump, out["level_samples"][i])].copy() for i in range(ns)]
        return out

    def trace_estimate(self, gid, **kw) -> dict:
        """One MG-MLMC(++) estimate on field gid (keywords: see _trace_in)."""
        p, r, keep = self._trace_in(**kw)
        self._chk(self.lib.mgm_trace_estimate(self.h, gid, C.byref(p), C.byref(r)), "trace_estimate")
        return self._trace_out(r, keep)

    def trace_jobs(self, jobs) -> list:
        """Independent estimates at once: jobs is a list of (gid, keywords),
        one distinct field per job; returns one result dict per job."""
        n = len(jobs)
        ins = [self._trace_in(**kw) for _, kw in jobs]
        gids = (C.c_int * max(1, n))(*[g for g, _ in jobs])
        ps = (TraceParams * max(1, n))(*[p for p, _, _ in ins])
        rs = (TraceResult * max(1, n))(*[r for _, r, _ in ins])
        self._chk(self.lib.mgm_trace_jobs(self.h, n, gids, ps, rs), "trace_jobs")
        return [self._trace_out(rs[j], ins[j][2]) for j in range(n)]
