/*
 * mgmlmc.h -- C ABI of the MI355X (gfx950) MG-MLMC++ library.
 *
 * The library estimates tr(D^{-1}) for the 2D Schwinger (U(1) Wilson-Dirac)
 * operator D with the multigrid multilevel Monte Carlo method combined with
 * Hutch++ deflation (MG-MLMC++; Frommer & Nasr Khalil, Alg. 2).  The problem
 * statement (Sec. 1) fixes the interface: D is large, sparse and non-singular,
 * and D^{-1} is reached only through solves D x = zeta.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Vectors are complex128 (interleaved re, im doubles) in DEVICE memory,
 *    caller-owned, in the natural layout [nrhs][n_level]: RHS r occupies
 *    n_level consecutive complex numbers.
 *  - Logical dof index on the fine level (level 0): (t * Lx + x) * 2 + s,
 *    s the spin.  On a coarse level l >= 1 with site grid Nx_l x Nt_l and
 *    ntv test vectors per chirality: ((A * 2 + c) * ntv + k), A = At*NAx+Ax
 *    the aggregate (= coarse site), c the chirality, k the test vector.
 *  - Every call is enqueued on the context's HIP stream (the stream given to
 *    mgm_create).  mgm_apply_* and mgm_noise return without a host sync;
 *    every other call synchronises the stream before returning.
 *  - Calls return MGM_OK (0) or a negative status; they never abort.
 *    mgm_last_error() gives the message of the last failing call.
 *  - One context per host thread; no internal locking.  All internal state
 *    (gauge copy, hierarchy, factorizations, workspaces) is owned by the
 *    context and freed by mgm_destroy.
 *  - FP64 results are bitwise reproducible for the same inputs, GPU and
 *    build: reductions use fixed trees and no atomics.
 */
#ifndef MGMLMC_H
#define MGMLMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MGM_OK 0
#define MGM_EINVAL (-1)     /* bad argument: sizes, pointers, level range      */
#define MGM_ENOMEM (-2)     /* device allocation failed                        */
#define MGM_EHIP (-3)       /* a HIP runtime call failed                       */
#define MGM_ESTATE (-4)     /* wrong order of calls (e.g. no setup_mg yet)     */
#define MGM_ENOTCONV (-5)   /* a solve did not reach its tolerance             */
#define MGM_ENONFINITE (-6) /* NaN or Inf in an input or a residual            */

#define MGM_MAX_LEVELS 6

/* noise kinds (isotropic vectors, Sec. 1 eq. random_props) */
#define MGM_NOISE_RADEMACHER 0 /* z = +-1                                 */
#define MGM_NOISE_Z2Z2 1       /* z = (+-1 +- i)/sqrt(2)                  */

/* noise purposes: field of the counter key */
#define MGM_PURPOSE_SETUP 1
#define MGM_PURPOSE_SKETCH 2
#define MGM_PURPOSE_SAMPLE 3
#define MGM_PURPOSE_TRAIN 4   /* right-hand sides of the network's training pairs */
#define MGM_PURPOSE_DEFLATE 5 /* start block of the deflation subspace iteration */
#define MGM_PURPOSE_PILOT 6   /* pilot samples of the adaptive choice of d_l */

/* precision of the multigrid preconditioner (the outer FGMRES, its residuals,
 * orthogonalisation and every trace sum are always FP64):
 *   FP64  the whole cycle in FP64;
 *   FP32  the whole cycle in FP32 (vectors and operators);
 *   FP16  as FP32, but coarse levels with 16 dofs per site keep their stencil
 *         blocks and SAP block inverses in FP16 and apply them with FP16
 *         matrix-core products (vector operands rounded to FP16, FP32
 *         accumulation).  Vectors whose entries exceed the FP16 range
 *         (|v| > 65504) in the cycle are not supported in this mode. */
#define MGM_PREC_FP64 0
#define MGM_PREC_FP32 1
#define MGM_PREC_FP16 2

typedef struct mgm_ctx mgm_ctx;

/* Create a context on HIP device `device`, enqueuing on `stream` (a
 * hipStream_t; NULL = the default stream). */
int mgm_create(mgm_ctx **out, int device, void *stream);
void mgm_destroy(mgm_ctx *ctx);
const char *mgm_last_error(const mgm_ctx *ctx);

/* ---------------------------------------------------------------------------
 * set_gauge -- the fine operator (Sec. 4: Schwinger discretization shifted by
 * a multiple of the identity):
 *   D = (m0 + 2) I - 1/2 sum_mu [(1 - sigma_mu) U_mu(x) delta_{x+mu,y}
 *                               + (1 + sigma_mu) U_mu(x-mu)^* delta_{x-mu,y}]
 * sigma_0 = Pauli x, sigma_1 = Pauli y; periodic in x; antiperiodic in t when
 * bc_t_anti != 0.
 *   links: DEVICE complex128 [2][Lt][Lx]; links[mu][t][x] = U_mu(x, t), the
 *          link from (x, t) to its neighbour in direction mu.  Copied in.
 *   Lx, Lt even and >= 2, at most 2^30 sites.  Returns a gauge handle in *gauge_id.
 * ------------------------------------------------------------------------- */
int mgm_set_gauge(mgm_ctx *ctx, int Lx, int Lt, const void *links, double m0,
                  int bc_t_anti, int *gauge_id);

/* free_gauge -- release a gauge field and everything built on it (multigrid
 * hierarchy, workspaces, captured graphs) once its queued work has finished.
 * The id is not reused; later calls with it fail with MGM_EINVAL. */
int mgm_free_gauge(mgm_ctx *ctx, int gauge_id);

/* ---------------------------------------------------------------------------
 * setup_mg -- aggregation multigrid hierarchy with R_l = P_l^H, P_l^H P_l = I
 * and Galerkin coarse operators D_{l+1} = P_l^H D_l P_l (Sec. 3.1), built by
 * the deterministic bootstrap documented with the oracle's setup:
 *   V <- Z2xZ2 noise (purpose SETUP, level l, column k)
 *   setup_iters times: V <- qr+(D_l^{-1} V)       (FGMRES solves to setup_tol)
 *   P_l columns of aggregate A, chirality c <- qr+(rows of V in (A, c))
 * then the coarsest operator is inverted densely (Gauss-Jordan with partial
 * pivoting), which gives tr(D_{L-1}^{-1}) (Alg. 2, coarsest level).
 * ------------------------------------------------------------------------- */
typedef struct {
  int nlevels;                        /* L, 1 .. MGM_MAX_LEVELS              */
  int block[MGM_MAX_LEVELS][2];       /* aggregate (bx, bt), step l -> l+1   */
  int ntv[MGM_MAX_LEVELS];            /* test vectors per chirality, step l  */
  int sap_block[MGM_MAX_LEVELS][2];   /* SAP block (sbx, sbt) on level l     */
  int sap_cycles[MGM_MAX_LEVELS];     /* SAP post-smoothing cycles, level l  */
  int inner_iters[MGM_MAX_LEVELS];    /* FGMRES steps of the coarse solve on
                                         level l (1 <= l <= L-2); 0 = one
                                         multigrid cycle on l, no Krylov    */
  double inner_tol;                   /* relative stop of those inner solves
                                         (0: always inner_iters steps)       */
  int setup_iters;                    /* inverse-iteration steps (3)          */
  double setup_tol;                   /* relative residual of setup solves   */
  int setup_restart;                  /* FGMRES restart length in the setup  */
  int setup_max_restarts;
  uint64_t seed;                      /* seed of the SETUP noise             */
  int precision;                      /* MGM_PREC_FP64 | _FP32 | _FP16      */
  int mlmc_levels;                    /* levels 0..mlmc_levels-1 form the
                                         MLMC telescoping sum; level
                                         mlmc_levels-1 is inverted densely
                                         for its exact trace and exact
                                         solves.  Coarser levels only serve
                                         the preconditioner.  0 = nlevels.  */
  int graphs;                         /* 1: replay preconditioner
                                         applications as captured HIP graphs */
} mgm_mg_params;

int mgm_setup_mg(mgm_ctx *ctx, int gauge_id, const mgm_mg_params *prm);

/* set_precision -- switch the preconditioner of a set-up field between
 * MGM_PREC_FP64, MGM_PREC_FP32 and MGM_PREC_FP16 without a new setup
 * (setup_mg keeps every copy); the outer FGMRES stays FP64. */
int mgm_set_precision(mgm_ctx *ctx, int gauge_id, int precision);

/* Level geometry: info[0..3] = Nx, Nt, dof per site M, n = Nx*Nt*M. */
int mgm_level_info(mgm_ctx *ctx, int gauge_id, int level, int *info);

/* ---------------------------------------------------------------------------
 * apply_D -- y = D_level x for nrhs vectors (level 0 = the fine operator,
 * level l >= 1 = the Galerkin operator; Sec. 3.1).  x, y: DEVICE
 * [nrhs][n_level], must not overlap.
 * apply_P -- y = P_level x: coarse (level+1) -> fine (level) vectors.
 * apply_R -- y = P_level^H x: fine (level) -> coarse (level+1) vectors.
 * ------------------------------------------------------------------------- */
int mgm_apply_D(mgm_ctx *ctx, int gauge_id, int level, int nrhs, const void *x, void *y);
int mgm_apply_P(mgm_ctx *ctx, int gauge_id, int level, int nrhs, const void *x, void *y);
int mgm_apply_R(mgm_ctx *ctx, int gauge_id, int level, int nrhs, const void *x, void *y);

/* Apply the multigrid preconditioner M_level ~ D_level^{-1}: coarse
 * correction by inner FGMRES (or the dense inverse on the coarsest level),
 * then sap_cycles red/black SAP cycles with exact block solves.  r, x:
 * DEVICE [nrhs][n_level]. */
int mgm_precondition(mgm_ctx *ctx, int gauge_id, int level, int nrhs, const void *r, void *x);

/* Copy P_level's aggregate blocks to DEVICE `out`:
 * complex128 [nagg][2][bx*bt*M_level/2][ntv]. */
int mgm_get_prolongator(mgm_ctx *ctx, int gauge_id, int level, void *out);

/* tr(D_T^{-1}) of the MLMC coarsest level T = mlmc_levels-1, out[0] = re,
 * out[1] = im (HOST). */
int mgm_coarsest_trace(mgm_ctx *ctx, int gauge_id, double *out);

/* ---------------------------------------------------------------------------
 * solve_batch -- x = D_level^{-1} b for nrhs right-hand sides by right-
 * preconditioned FGMRES(restart) in FP64 with the multigrid preconditioner
 * (Alg. 2 "use mg to solve lin. sys.").  Every RHS stops on its true FP64
 * residual ||b - D x|| <= tol ||b||.  x0 = 0 (or the learned guess, see
 * mgm_cnn_set_params).  On the coarsest level the
 * dense inverse is applied.  b, x: DEVICE [nrhs][n_level].
 * stats (optional, HOST arrays of nrhs entries, caller-owned): FGMRES
 * iterations and final relative residual per RHS.  On MGM_ENOTCONV x holds
 * the last iterate.
 * ------------------------------------------------------------------------- */
typedef struct {
  double tol;        /* relative residual, e.g. 1e-10 */
  int restart;       /* FGMRES restart length m       */
  int max_restarts;
  int rhs_block;     /* RHS solved together (0 = all, -1 = the autotuned
                        width of the level, all if none) */
  int use_cnn;       /* level 0 only, flags (mgm_cnn_*): MGM_CNN_GUESS
                        starts from the learned guess instead of x0 = 0;
                        MGM_CNN_STAGE puts the network in front of the
                        multigrid cycle in every preconditioner call */
} mgm_solve_params;

#define MGM_CNN_GUESS 1
#define MGM_CNN_STAGE 2

typedef struct {
  int *iters;        /* HOST [nrhs] or NULL */
  double *relres;    /* HOST [nrhs] or NULL */
} mgm_solve_stats;

int mgm_solve_batch(mgm_ctx *ctx, int gauge_id, int level, int nrhs, const void *b, void *x,
                    const mgm_solve_params *prm, mgm_solve_stats *stats);

/* ---------------------------------------------------------------------------
 * solve_jobs -- many independent solve batches, possibly on different gauge
 * fields and lattice sizes, in one call.  Each gauge field owns a HIP stream
 * and its workspaces; the jobs of one field run in order on its stream, the
 * fields run concurrently (one host thread each), so small lattices share the
 * GPU.  Every RHS meets prm->tol as in mgm_solve_batch.  iters (optional,
 * HOST, sum of nrhs entries in job order) receives FGMRES iterations.
 * ------------------------------------------------------------------------- */
typedef struct {
  int gauge_id, level, nrhs;
  const void *b;  /* DEVICE [nrhs][n_level] */
  void *x;        /* DEVICE [nrhs][n_level] */
} mgm_job;

int mgm_solve_jobs(mgm_ctx *ctx, int njobs, const mgm_job *jobs, const mgm_solve_params *prm,
                   int *iters);

/* autotune_rhs_block -- time solves of nrhs noise vectors on `level` with RHS
 * block widths 8, 16, 32 and 64 (up to nrhs) and keep the fastest for
 * rhs_block = -1; the width is written to *best. */
int mgm_autotune_rhs_block(mgm_ctx *ctx, int gauge_id, int level, int nrhs,
                           const mgm_solve_params *prm, int *best);

/* ---------------------------------------------------------------------------
 * noise -- nrhs isotropic vectors of length n written to DEVICE out
 * [nrhs][n] (complex128): vector r uses the counter key (seed, purpose,
 * level, index0 + r), element i its SplitMix64 word i.
 * ------------------------------------------------------------------------- */
int mgm_noise(mgm_ctx *ctx, int kind, uint64_t seed, int purpose, int level, int64_t index0,
              int64_t n, int nrhs, void *out);

/* qr+ -- Q = thin QR factor of the d columns of Y (DEVICE [d][n]) with a
 * real positive diagonal of R (CholQR2); Q written to DEVICE [d][n]. */
int mgm_orthonormalize(mgm_ctx *ctx, int64_t n, int d, const void *Y, void *Q);

/* orthonormalize_noalloc -- the same Q = qr+(Y) as mgm_orthonormalize, for
 * callers that cannot allocate device memory (code that must not call
 * hipMalloc, e.g. while a HIP graph is being captured, or a serving loop
 * with a fixed memory budget).  The call allocates nothing: its workspace is
 * one static device array of about 25 MB that each device using the library
 * holds until the process ends.  Limits: 1 <= d <= 64, d <= n, n * d <= 2^20
 * (MGM_EINVAL beyond).  Every call on a device shares that array, so calls
 * that overlap on one device (several host threads or streams) race; calls
 * in order on one stream are safe.  Synchronises the stream, like
 * mgm_orthonormalize. */
int mgm_orthonormalize_noalloc(mgm_ctx *ctx, int64_t n, int d, const void *Y, void *Q);

/* ---------------------------------------------------------------------------
 * trace_estimate -- tr(D^{-1}) by
 *   MGM_VARIANT_HUTCH    Alg. 1 (plain Hutchinson) on D^{-1};
 *   MGM_VARIANT_HUTCHPP  Hutch++ (Sec. 2.4) on D^{-1};
 *   MGM_VARIANT_MLMC     MG-MLMC (Sec. 3.1), i.e. Alg. 2 with d_l = 0;
 *   MGM_VARIANT_MLMCPP   MG-MLMC++ (Alg. 2);
 *   MGM_VARIANT_DEFLATED deflated Hutchinson (Sec. 2.2, the reference method
 *                        of Sec. 4): Pi = Q Q^H with Q (n x d[0]) from k_power
 *                        sweeps of block subspace iteration
 *                        Q <- qr(D^{-1} gamma5 D^{-1} gamma5 Q) (noise purpose
 *                        DEFLATE at the start), which converges to the right
 *                        singular vectors of D of the d[0] smallest singular
 *                        values (D^{-H} = gamma5 D^{-1} gamma5 for this
 *                        operator); tr(Pi D^{-1}) = tr(Q^H D^{-1} Q) from d[0]
 *                        solves (exact for any orthonormal Q, Sec. 2.3) and
 *                        Hutchinson on (I - Pi) D^{-1}.  The exact-deflation
 *                        value sum u_i^H v_i / sigma_i of the Ritz triplets of
 *                        D on span(Q) is reported next to it (defl_ritz).
 * Level differences use the reduced form (eq. mlmc_dec_trace_reduced) or the
 * full form with accumulated prolongations (eq. mlmc_decomp_trace).  Samples
 * are drawn `batch` at a time per active level and Alg. 2's stopping rule is
 * replayed sample by sample, so the result equals the sequential algorithm's
 * on the same seeds.  In the reduced form all right-hand sides one phase
 * needs on a level (the fine part of difference l, the coarse part of
 * difference l-1) are solved as one batch.
 * ------------------------------------------------------------------------- */
#define MGM_VARIANT_HUTCH 0
#define MGM_VARIANT_HUTCHPP 1
#define MGM_VARIANT_MLMC 2
#define MGM_VARIANT_MLMCPP 3
#define MGM_VARIANT_DEFLATED 4
#define MGM_FORM_REDUCED 0
#define MGM_FORM_FULL 1
#define MGM_TARGETS_OPTIMAL 0
#define MGM_TARGETS_UNIFORM 1
#define MGM_PROJ_ONE_SIDED 0
#define MGM_PROJ_TWO_SIDED 1
/* cost C_{s,l} of a stochastic sample (Alg. 2), which weighs the optimal
 * target variances (Sec. 3, eq. optimal_variance):
 *   STATIC  one number per level: nnz(D_l) + nnz(D_{l+1}) + 2 n_l d_l;
 *   FIXED   the given fixed_cost[l];
 *   FLOPS   the cost model of Sec. 4: complex multiply-adds of every
 *           matrix-vector product of the sample -- the operators by their
 *           structural non-zeros (9 per fine row, 5 M^2 per coarse site),
 *           R_l and P_l (n_l ntv_l each), per SAP cycle the residual rows of
 *           both colours and one K x K block-inverse product per block, dense
 *           inverses (n^2), per FGMRES iteration one preconditioner and one
 *           operator product, per restart cycle two residuals, a solve with a
 *           dense inverse one dense product and its residual check, and the
 *           projection 2 n_l d_l.  It depends on the iteration counts of the
 *           sample's own solves; C_l is the running mean over the samples
 *           taken, as Alg. 2 prints. */
#define MGM_COST_STATIC 0
#define MGM_COST_FIXED 1
#define MGM_COST_FLOPS 2

typedef struct {
  int variant, form;
  double eps;                        /* relative accuracy (1 sigma)          */
  int d[MGM_MAX_LEVELS];             /* Hutch++ vectors per difference level */
  int k_power;                       /* block power sweeps                   */
  int noise;                         /* MGM_NOISE_*                          */
  int targets;                       /* MGM_TARGETS_*                        */
  int cost;                          /* MGM_COST_*                           */
  double fixed_cost[MGM_MAX_LEVELS]; /* cost per sample with MGM_COST_FIXED  */
  int min_samples;                   /* no stop test before this many
                                        samples (>= 2; values below 2 mean 2) */
  int max_samples;
  const int *fixed_samples;          /* HOST [levels] exact counts, or NULL  */
  uint64_t seed;
  int batch;                         /* samples per level per GPU batch      */
  mgm_solve_params solve;
  int d_max;                         /* > 0 (HUTCHPP, MLMCPP): adaptive d_l.
                                        Candidates d[l], 2 d[l], ... <= d_max
                                        (<= 64); per candidate the Hutch++
                                        basis, tau_lr and `pilot` pilot
                                        samples (noise purpose PILOT, then
                                        discarded) predict the level's cost
                                        T(d) = W_lr(d) + V(d) C(d) / rho^2,
                                        rho^2 = (eps |tau0|)^2 / (levels),
                                        tau0 from the first candidates; the
                                        doubling stops when T stops falling
                                        and the best candidate's basis is
                                        used.  The choice of d is left open
                                        by the paper (Sec. 5).  0: fixed d. */
  int pilot;                         /* pilot samples per candidate (>= 2)  */
  int projection;                    /* MGM_PROJ_ONE_SIDED: tau_s =
                                        z^H (A zeta) as Alg. 2 prints;
                                        MGM_PROJ_TWO_SIDED: tau_s = z^H (A z),
                                        Hutchinson on (I - QQ^H) A (I - QQ^H):
                                        same mean, another variance; its
                                        samples are solved after Q is final */
  int concurrent;                    /* 1: a phase's solves on different
                                        levels run at once on two streams of
                                        the field (same results as 0)       */
} mgm_trace_params;

typedef struct {
  double tau[2];                       /* the estimate of tr(D^{-1})          */
  double tau_exact[2];                 /* directly computed coarsest part     */
  int nstoch;                          /* stochastic levels                   */
  double lvl_mean[MGM_MAX_LEVELS][2];
  double lvl_lr[MGM_MAX_LEVELS][2];    /* Hutch++ low-rank parts              */
  double lvl_var[MGM_MAX_LEVELS];
  double lvl_cost[MGM_MAX_LEVELS];     /* C_l used by the last stop test      */
  int lvl_samples[MGM_MAX_LEVELS];
  int64_t lvl_solves[MGM_MAX_LEVELS];  /* solves on D_l issued (incl. discarded batch tail) */
  int64_t lvl_iters[MGM_MAX_LEVELS];   /* FGMRES iterations on D_l            */
  double lvl_lr_work[MGM_MAX_LEVELS];  /* Sec. 4 cost model of difference l's
                                          Hutch++ phase (k sweeps and the
                                          low-rank round)                   */
  double lvl_work[MGM_MAX_LEVELS];     /* lvl_lr_work + the costs of the
                                          samples kept (whatever `cost`)    */
  double *sample_dump;                 /* HOST [nstoch][max_dump][2] or NULL  */
  double *cost_dump;                   /* HOST [nstoch][max_dump] or NULL:
                                          each kept sample's Sec. 4 cost     */
  int lvl_d[MGM_MAX_LEVELS];           /* Hutch++ vectors used per level
                                          difference (the adaptive choice)  */
  double defl_ritz[2];                 /* deflated variant: sum u_i^H v_i /
                                          sigma_i over the Ritz singular
                                          triplets of D on span(Q)           */
  double *sigma_dump;                  /* deflated variant: HOST [d[0]] or
                                          NULL, those Ritz singular values
                                          ascending                         */
  int *iter_dump;                      /* HOST [nstoch][max_dump][2] or NULL:
                                          FGMRES iterations of each kept
                                          sample's solves on D_l, D_{l+1}
                                          (0 where a level has no such solve) */
  int max_dump;
} mgm_trace_result;

int mgm_trace_estimate(mgm_ctx *ctx, int gauge_id, const mgm_trace_params *prm,
                       mgm_trace_result *res);

/* ---------------------------------------------------------------------------
 * trace_jobs -- njobs independent estimates (Alg. 2 each) at once, e.g. one
 * per gauge field of an ensemble: job j runs on field gauge_ids[j] with
 * params[j] into results[j] (HOST arrays of njobs entries; the fields must be
 * distinct).  Each job runs on its field's own streams from a host thread of
 * its own, so the latency-bound kernels of the estimates overlap on the GPU.
 * Each result is bit for bit that of a separate mgm_trace_estimate call.
 * Returns the first failing job's status (its index in mgm_last_error).
 * ------------------------------------------------------------------------- */
int mgm_trace_jobs(mgm_ctx *ctx, int njobs, const int *gauge_ids, const mgm_trace_params *params,
                   mgm_trace_result *results);

/* ---------------------------------------------------------------------------
 * time_kernel -- measurement helper for rooflines: launches one kernel of the
 * path `reps` times back to back on the context stream (inputs: seeded noise
 * vectors allocated by the library) and returns, between two HIP events, the
 * average duration per launch in microseconds (*us_out), the algorithmic
 * bytes one launch moves (*bytes_out: every operand counted once) and its
 * algorithmic flops (*flops_out).  Synchronises.
 *   MGM_KERNEL_STENCIL  y = D_level x
 *   MGM_KERNEL_SAP      one red/black SAP colour sweep on `level`
 *   MGM_KERNEL_DENSE    y = D_level^{-1} x with the dense inverse (level must
 *                       have one)
 *   MGM_KERNEL_CGS      one Gram-Schmidt projection pass against 16 vectors
 *   MGM_KERNEL_COPY     y = x, a plain copy of nrhs * n_level complex128
 *   MGM_KERNEL_CONV     one hidden 32 -> 32 3x3 convolution (+ tanh) of the
 *                       learned guess on nrhs fields of level 0 (FP32 matrix
 *                       cores; needs mgm_cnn_set_params)
 *   MGM_KERNEL_SAP_LOW  one SAP colour sweep of the low-precision cycle at the
 *                       field's current precision (FP32 vectors; FP16 blocks on
 *                       16-dof levels in FP16 mode)
 *   MGM_KERNEL_CONV_H   the same hidden convolution with FP16 weights and
 *                       activations (FP16 matrix cores, FP32 accumulation)
 *   MGM_KERNEL_DENSE_LOW the low-precision cycle's coarse solve y = D^{-1} x on
 *                       the coarsest level at the field's current precision
 *                       (FP32 vectors; in FP16 mode the FP16 copy of the
 *                       inverse on the FP16 matrix cores when it exists)
 * ------------------------------------------------------------------------- */
#define MGM_KERNEL_STENCIL 0
#define MGM_KERNEL_SAP 1
#define MGM_KERNEL_DENSE 2
#define MGM_KERNEL_CGS 3
#define MGM_KERNEL_COPY 4
#define MGM_KERNEL_CONV 5
#define MGM_KERNEL_SAP_LOW 6
#define MGM_KERNEL_CONV_H 7
#define MGM_KERNEL_DENSE_LOW 8

int mgm_time_kernel(mgm_ctx *ctx, int gauge_id, int kind, int level, int nrhs, int reps,
                    double *us_out, double *bytes_out, double *flops_out);

/* ---------------------------------------------------------------------------
 * Learned initial guess.  Not part of the paper's method: it changes where a
 * fine-level solve starts, never the tolerance it meets, so the estimator is
 * unchanged (every sample still comes from an FP64 solve to prm->tol).
 *
 * The network y = f(b): four 3x3 convolutions on the fine lattice with
 * 4 -> 32 -> 32 -> 32 -> 4 channels and tanh after the first three.  Its 4
 * channels are (Re, Im) x 2 spins in the order of a level-0 vector, so a
 * complex128 vector [n0] is read as [Lt][Lx][4] reals.  Padding is periodic
 * in x and, in t, follows the field's boundary condition (antiperiodic: a
 * value fetched across the t boundary changes sign).  The network does not
 * see the links.  Parameters: MGM_CNN_NPARAMS floats packed
 * W1 b1 W2 b2 W3 b3 W4 b4 with W[co][ci][dt][dx], where tap (dt, dx) reads
 * site (t + dt - 1, x + dx - 1).  FP32 storage, FP32 matrix-core
 * accumulation.  One network per context; Lx and Lt must be multiples of 16.
 *
 * With mgm_solve_params.use_cnn = 1, a level-0 solve starts from
 * x0 = alpha_r f(b_r), alpha_r = <D f(b_r), b_r> / ||D f(b_r)||^2 per RHS (the
 * minimal residual along f(b_r), so ||b - D x0|| <= ||b||); a zero or
 * non-finite alpha_r gives x0 = 0, i.e. plain multigrid.
 *
 * With MGM_CNN_STAGE the network is the first stage of the level-0
 * preconditioner of the (flexible) outer FGMRES: for an Arnoldi vector v_r
 * (unit norm) z_r = x_r + M(v_r - D x_r) with M the multigrid cycle and
 * x_r = alpha_r f(sqrt(n0) v_r), alpha_r the minimal residual factor as
 * above (sqrt(n0) scales v_r to the size of a Z2 x Z2 vector, the network's
 * training input).  A zero or non-finite alpha_r gives z_r = M v_r, i.e.
 * multigrid alone.  Each iteration then costs one network evaluation and
 * one extra application of D on top of the cycle.
 * ------------------------------------------------------------------------- */
#define MGM_CNN_NPARAMS 20836

/* set_params -- copy HOST theta [MGM_CNN_NPARAMS] into the network and reset
 * the Adam state.  get_params copies the current parameters to HOST theta. */
int mgm_cnn_set_params(mgm_ctx *ctx, const float *theta);
int mgm_cnn_get_params(mgm_ctx *ctx, float *theta);

/* set_precision -- arithmetic of the network's inference (mgm_cnn_apply and
 * the initial guess): MGM_PREC_FP32 (default) or MGM_PREC_FP16 (FP16 weights
 * and activations on the FP16 matrix cores, FP32 accumulation).  Training
 * (loss_grad, train_step, train) always runs in FP32 on the FP32 master
 * parameters.  Needs mgm_cnn_set_params first. */
int mgm_cnn_set_precision(mgm_ctx *ctx, int precision);

/* apply -- y = f(b) for nb level-0 vectors of gauge field gauge_id (its
 * lattice size and boundary condition); b, y: DEVICE complex128 [nb][n0]. */
int mgm_cnn_apply(mgm_ctx *ctx, int gauge_id, int nb, const void *b, void *y);

/* loss_grad -- loss = (1/nb) sum_r ||f(b_r) - x_r||^2 / ||x_r||^2 (written to
 * HOST *loss) and its gradient with respect to the parameters (HOST grad
 * [MGM_CNN_NPARAMS], same packing, or NULL).  b, x: DEVICE complex128
 * [nb][n0]. */
int mgm_cnn_loss_grad(mgm_ctx *ctx, int gauge_id, int nb, const void *b, const void *x,
                      double *loss, float *grad);

typedef struct {
  double lr, beta1, beta2, eps;  /* Adam (Kingma & Ba 2015), bias-corrected */
} mgm_adam_params;

/* train_step -- loss_grad on (b, x), then one Adam step; *loss (HOST) is the
 * loss before the step. */
int mgm_cnn_train_step(mgm_ctx *ctx, int gauge_id, int nb, const void *b, const void *x,
                       const mgm_adam_params *adam, double *loss);

typedef struct {
  int pairs_per_field;      /* Z2xZ2 right-hand sides per field (noise purpose
                               MGM_PURPOSE_TRAIN, level 0, index = pair) */
  int batch;                /* pairs per Adam step */
  int epochs;
  mgm_adam_params adam;
  uint64_t seed;            /* noise seed; also orders the pairs each epoch */
  mgm_solve_params solve;   /* the multigrid solves that make the targets */
} mgm_cnn_train_params;

/* train -- solve D x = b for pairs_per_field noise vectors on each of the
 * nfields fields (all of one lattice size, each with its multigrid set up),
 * keep the pairs in HBM, and run `epochs` passes of Adam over them in a
 * seeded order.  epoch_loss (HOST [epochs] or NULL) receives each epoch's
 * mean mini-batch loss.  MGM_ENOTCONV if a target solve did not converge. */
int mgm_cnn_train(mgm_ctx *ctx, int nfields, const int *gauge_ids, const mgm_cnn_train_params *prm,
                  double *epoch_loss);

#ifdef __cplusplus
}
#endif
#endif /* MGMLMC_H */
