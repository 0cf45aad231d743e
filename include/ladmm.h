/*
 * ladmm.h - batched ADMM for the Gamma Knife planning LP on one MI355X (gfx950).
 *
 * C ABI of the library.  The library solves, for k objective weightings at
 * once, the LP
 *
 *     minimize c'x   subject to   A x <= b,   0 <= x <= u            (Eq. dual_problem)
 *
 * whose blocks are those of App. A: columns of A are the dose points (target
 * surface TS, target interior TI, ring R, low-dose LD, organ at risk O) followed
 * by 8 sector variables per isocentre; rows are 24 shot rows and one beam-on-time
 * (BOT) row per isocentre.  The weights of each plan enter only b and u (Sec. 2.A
 * and the end of Sec. 2.B).  The solver is the scaled-form ADMM of Eq. (admm)
 * with the x-step of Eq. (partial_elimination) and the closed form after it,
 * applied to all plans as matrix columns, with the row normalisation, BOT column
 * scaling and per-plan step size rule of Sec. 3.C.
 *
 * Conventions that hold for every entry point:
 *   - Return value: LADMM_OK (0) on success, LADMM_PENDING (>0) for a request
 *     still running, a negative ladmm_status on error.  Not converging within
 *     the iteration limit is NOT an error: it is a per-plan status.  After an
 *     error, ladmm_last_error() returns a message for the calling thread.
 *   - Pointers named host_* or documented as host memory are read during the
 *     call only and copied; the caller keeps ownership.  Result buffers are
 *     caller-owned host memory written by the library.  Handles are owned by
 *     the library and released by the matching destroy call.
 *   - Matrices are dense and row-major unless stated otherwise.
 *   - Calls on one handle are not thread-safe unless stated; different cases
 *     may be used from different threads.
 */
#ifndef LADMM_H
#define LADMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LADMM_OK = 0,
  LADMM_PENDING = 1,
  LADMM_E_INVALID = -1,   /* malformed argument or descriptor                */
  LADMM_E_NOMEM = -2,     /* HBM budget of the context exceeded, or hipMalloc */
  LADMM_E_DEVICE = -3,    /* a HIP runtime call failed                        */
  LADMM_E_NUMERIC = -4,   /* Schur complement not positive definite, NaN/Inf  */
  LADMM_E_STATE = -5,     /* unknown, destroyed or busy handle / ticket       */
  LADMM_E_CANCELLED = -6
} ladmm_status;

/* Storage and arithmetic of the dose matrix and the dose-point iterates.  The
 * Schur complement, its factor and inverse, and the small per-row iterates are
 * always FP64.
 *   LADMM_F64:    FP64 dose block and iterates, FP64 MFMA.
 *   LADMM_F32:    FP32 dose block and iterates, FP32 MFMA.
 *   LADMM_BF16X3: the dose block and the plan-side operands of the two products
 *                 (z1 - y1, the Schur solution, the shot times) as BF16 pairs
 *                 hi = bf16(x), lo = bf16(x - hi); each product sums
 *                 A_hi B_hi + A_hi B_lo + A_lo B_hi on the BF16 MFMA with FP32
 *                 accumulation (about 2^-16 relative per product); iterates FP32.
 *                 The dose block takes 8 bytes per entry (two pairs, one per
 *                 product layout).
 *   LADMM_BF16:   BF16 dose block with iterative refinement of the x-update
 *                 (the FP32-iteration / FP64-factor split of Sec. 3.A carried
 *                 one step further).  Every iteration but the last of each check
 *                 chunk reads the dose block once per product as a single BF16
 *                 operand (2 bytes per entry; the rows of A are scaled to unit
 *                 norm by E, Sec. 3.C, which is the per-column scale of the BF16
 *                 block) and multiplies it, on the BF16 MFMA with FP32
 *                 accumulation, by the change of the plan-side operand since the
 *                 last refresh: A_s W = G_ref + D_hi' bf16(W - W_ref) and
 *                 A_s' v = X_ref + D_hi bf16(v - v_ref).  The last iteration of
 *                 every chunk is a refresh: three-term pair products (as
 *                 LADMM_BF16X3) that also record G_ref, W_ref, X_ref, v_ref; the
 *                 check statistics and the objective come from it.  The rounding
 *                 then acts on the change alone, so the iterates converge to the
 *                 fixed point of the exact products.  Iterates FP32; the low half
 *                 of the dose block is read by the refresh only. */
typedef enum { LADMM_F64 = 0, LADMM_F32 = 1, LADMM_BF16X3 = 2, LADMM_BF16 = 3 } ladmm_precision;

/* Dose-point group types (App. A subscripts TS, TI, R, LD, O). */
typedef enum { LADMM_PT_TS = 0, LADMM_PT_TI = 1, LADMM_PT_RING = 2, LADMM_PT_LD = 3,
               LADMM_PT_OAR = 4 } ladmm_point_type;

typedef enum { LADMM_PLAN_CONVERGED = 0, LADMM_PLAN_MAX_ITER = 1, LADMM_PLAN_NUMERIC = 2,
               LADMM_PLAN_RUNNING = 3 } ladmm_plan_status;

/* One block of dose points (App. A, including its multi-target extension).
 *   threshold : D_alpha in Gy (for an OAR, its max dose D_O); > 0.
 *   share     : multiplies the plan weight of the group's type: q_k,A for a
 *               target surface, q_k,V for a target interior, 1/n for a ring,
 *               1 for low-dose and OAR groups.  >= 0. */
typedef struct {
  int32_t type;        /* ladmm_point_type */
  int32_t structure;   /* target / LD level / OAR index (informational) */
  double threshold;
  double share;
} ladmm_group;

/* A planning case.  n_t = n_iso * n_sectors * n_collimators shot columns,
 * ordered (i * n_sectors + s) * n_collimators + c (collimator fastest), which
 * is the order of C = I (x) I_8 (x) 1_{1x3} in App. A. */
typedef struct {
  int32_t n_points;           /* N >= 1 dose points                              */
  int32_t n_iso;              /* >= 1                                           */
  int32_t n_sectors;          /* 8 on the Gamma Knife                           */
  int32_t n_collimators;      /* 3 on the Gamma Knife                           */
  const double *dose;         /* host, N x n_t dose rates phi >= 0, finite       */
  const int32_t *point_group; /* host, N entries in [0, n_groups)                */
  int32_t n_groups;
  const ladmm_group *groups;  /* host, n_groups entries                          */
  double prescription_mean;   /* D_T (mean target prescription), > 0             */
  double phi_cal;             /* calibration dose rate, > 0                      */
  int32_t precision;          /* ladmm_precision                                 */
  int32_t row_normalize;      /* 1: unit 2-norm rows of A (Sec. 3.C)             */
  double beta;                /* BOT column scale; <= 0 selects the rule         */
  double beta_denominator;    /*   beta = (non-OAR points) / beta_denominator    */
} ladmm_case_desc;

/* Primal weights of one plan (Sec. 2.A): w_TS = w_TI = w_T. w_BOT > 0. */
typedef struct { double w_t, w_r, w_ld, w_bot; } ladmm_weights;

/* Solver options.  Step size per plan: rho_j = rho0 * sqrt(w0_bot / w_BOT,j)
 * (Eq. rho_rule).  Plan j stops at the first check (every check_every
 * iterations) where rel_gap <= tol_gap, r_pri <= tol_pri and r_dual <= tol_dual
 * (and cert_gap <= tol_cert when tol_cert > 0; a tolerance <= 0 other than
 * tol_gap is not used); tol_gap <= 0 and tol_cert <= 0 run exactly max_iter
 * iterations (the fixed budget of Sec. 3.D). */
typedef struct {
  int32_t max_iter;
  int32_t check_every;
  double tol_gap, tol_pri, tol_dual;
  double rho0, w0_bot;
  int32_t autotune;   /* nonzero: time the tile configurations before the first
                         iteration (see ladmm_batch_tiles); 0: configuration 0 */
  /* Per-plan step-size balancing (extension of the fixed rule of Sec. 3.C):
   * with adapt_rho nonzero, at every check of ladmm_batch_run / solve / serve
   * a running plan's rho is multiplied by adapt_tau when r_pri > adapt_mu *
   * r_dual and divided by it when r_dual > adapt_mu * r_pri, within a factor
   * 1e3 of its starting value; its scaled duals are rescaled so that the
   * multipliers rho * y (and the shot times) do not change.  S does not depend
   * on rho, so nothing is refactored.  adapt_tau = 2 keeps every rescale
   * exact.  adapt_mu > 1, adapt_tau > 1. */
  int32_t adapt_rho;
  double adapt_mu, adapt_tau;
  /* Over-relaxation (an extension; the paper's ADMM has alpha = 1): the z- and
   * y-steps of Eq. (admm) use alpha x + (1 - alpha) z in place of x, z the
   * copies before the step; the residuals keep x.  alpha in (0, 2); 0 means 1.
   * Batches and solves only: ladmm_submit rejects alpha other than 0 or 1. */
  double alpha;
  /* Stopping on the certified gap (see ladmm_result.cert_gap): with tol_cert
   * > 0 a plan also needs cert_gap <= tol_cert to stop, which proves its
   * objective within tol_cert (relative) of the exact optimum F*.  0: not used.
   * A plan stops at the first check where every tolerance in use holds
   * (tol_gap, tol_cert, and tol_pri, tol_dual when > 0); with tol_gap <= 0 and
   * tol_cert <= 0 it runs exactly max_iter iterations. */
  double tol_cert;
} ladmm_opts;

/* Per-plan results; every pointer is caller-owned host memory or NULL.
 *   t        : k x n_t shot times  t = E rho y2 (end of Sec. 2.B), >= 0
 *   bot      : k x n_iso  tau_i = (phi_cal/D_T) max_s sum_c t_isc
 *   objective: F_j(t), the planning objective (hinge terms + w_BOT sum tau)
 *   dual_obj : c'z1, the dual-LP objective at the box-feasible copy
 *   rel_gap  : |F + c'z1| / max(F, 1e-300) (the plain gap: not a bound)
 *   r_pri    : ||x - z|| / max(||x||, ||z||);  r_dual: ||z - z_prev|| / ||y||
 *   iters    : iterations run;  plan_status: ladmm_plan_status
 *   lower_bound: L <= F* by LP duality (App. A): x = (clip(z1, 0, u), sector
 *              values as small as the shot rows allow), scaled by the largest
 *              theta <= 1 that keeps every BOT row within w_BOT, is feasible
 *              for the dual LP, so L = -c'x <= -p* = F*.
 *   cert_gap : (U - L) / U with U an upper bound on F(t~) >= F* for the
 *              OAR-feasible shot times t~ = t / max(1, max_O d_O / D_O):
 *              U = F(t) + (1 - 1/r) sum_targets u d / D when the OAR ratio r
 *              exceeds 1.  Certifies |F(t~) - F*| <= cert_gap * U.
 * lower_bound and cert_gap are evaluated in the iteration precision of the
 * products (FP64 sums); the certificate is as rigorous as those products. */
typedef struct {
  double *t, *bot, *objective, *dual_obj, *rel_gap, *r_pri, *r_dual;
  int32_t *iters, *plan_status;
  double *lower_bound, *cert_gap;
} ladmm_result;

typedef struct ladmm_ctx ladmm_ctx;
typedef struct ladmm_case ladmm_case;
typedef struct ladmm_batch ladmm_batch;

/* Context on one device.  hbm_budget_bytes = 0 means no budget.  Every case
 * and batch allocation is charged to the budget; a request that would exceed it
 * fails with LADMM_E_NOMEM before touching the device. */
int ladmm_ctx_create(int device, size_t hbm_budget_bytes, ladmm_ctx **out);
/* Destroying a context (or a case) that still has live cases (or batches) is
 * allowed: the object is freed when its last dependant is destroyed. */
int ladmm_ctx_destroy(ladmm_ctx *ctx);
/* Bytes currently charged to the context. */
size_t ladmm_ctx_used_bytes(const ladmm_ctx *ctx);

/* Case setup (Sec. 2.B, 3.C): copies the dose matrix to HBM; computes the row
 * scales E, beta, the Schur complement S = A A' + I (FP64), its Cholesky factor
 * and S^-1 = L^-T L^-1 (FP64); stores the scaled dose block in the requested
 * precision.  LADMM_E_INVALID for negative or non-finite doses, bad group
 * indices, non-positive thresholds; LADMM_E_NUMERIC if S is not SPD. */
int ladmm_create_case(ladmm_ctx *ctx, const ladmm_case_desc *desc, ladmm_case **out);
int ladmm_destroy_case(ladmm_case *c);
/* Row scales E (m_A = n_t + n_iso values) and beta of a case, to host memory. */
int ladmm_case_scaling(const ladmm_case *c, double *E, double *beta);
/* Inspection of the cached setup, for verification: the Schur complement
 * S = A_s A_s' + I of the scaled LP (Eq. partial_elimination) and its inverse,
 * each m_A x m_A FP64 host memory (rows: shot rows, then BOT rows).  Either
 * pointer may be NULL. */
int ladmm_case_schur(const ladmm_case *c, double *S, double *S_inv);
/* Setup timing in milliseconds (device time of the setup kernels). */
double ladmm_case_setup_ms(const ladmm_case *c);

/* A batch of k plans on a case, holding the iterates in HBM.
 *   ld_mask: NULL, or host k x ceil(N/64) uint64 words; bit (p % 64) of word
 *            p / 64 of row j set means dose point p is in plan j's low-dose
 *            set p_j (Sec. 2.C.2).  Low-dose points outside p_j get u = 0 and
 *            the LD weight of plan j is spread over |p_j| points.  Bits of
 *            non-LD points are ignored.
 *   rho:     NULL (rule of Eq. rho_rule from opts) or host k values > 0.
 * Iterates start at zero. */
int ladmm_batch_create(ladmm_case *c, int32_t k, const ladmm_weights *w,
                       const uint64_t *ld_mask, const double *rho,
                       const ladmm_opts *opts, ladmm_batch **out);
int ladmm_batch_destroy(ladmm_batch *b);
/* Exactly `iters` ADMM iterations on every active plan, no convergence checks. */
int ladmm_batch_iterate(ladmm_batch *b, int32_t iters);
/* Iterate with checks until every plan has stopped or max_iter is reached. */
int ladmm_batch_run(ladmm_batch *b);
/* The same, returning after at most max_checks check chunks (>= 1) with
 * *running (optional) = plans still running; call again to continue.  Plans
 * that stop keep their results; a run continued in several calls gives the
 * same results as one ladmm_batch_run. */
int ladmm_batch_run_checks(ladmm_batch *b, int32_t max_checks, int32_t *running);
/* Evaluate the per-plan statistics at the current iterate and fill `out`. */
int ladmm_batch_results(ladmm_batch *b, ladmm_result *out);
/* Iterates in the oracle's variables (scaled LP of Sec. 3.C), host FP64,
 * row-major with one column per plan: z1, y1 are n_A x k (points then
 * sectors), z2, y2 are m_A x k (shot rows then BOT rows).  Any pointer may be
 * NULL.  Import requires z1 = clip(z1 + y1, 0, u) and z2 = min(z2 + y2, b),
 * which every ADMM iterate satisfies; the device keeps q = z + y only. */
int ladmm_batch_export(ladmm_batch *b, double *z1, double *y1, double *z2, double *y2);
int ladmm_batch_import(ladmm_batch *b, const double *z1, const double *y1,
                       const double *z2, const double *y2);
/* Device time of the iterations run so far, in milliseconds, and the number of
 * plan-iterations. */
int ladmm_batch_timing(const ladmm_batch *b, double *iterate_ms, int64_t *plan_iterations);
/* Current step size rho_j of every plan (host, k values): the rule of
 * Eq. rho_rule at the start, changed by step-size balancing when adapt_rho is
 * on.  The exported scaled duals y are the multipliers divided by these. */
int ladmm_batch_step_sizes(const ladmm_batch *b, double *rho);

/* Per-kernel timing.  With profiling on, every kernel launch of an iteration
 * is bracketed by HIP events recorded on the batch's stream; the elapsed times
 * are accumulated per kernel class when each run chunk completes.  Classes:
 * 0 GEMM1 (A_s W, the dose-point part of the right-hand side), 1 rhs assembly,
 * 2 S^-1 product, 3 post (small-side update), 4 GEMM2 (closed-form x-step with
 * the fused z- and y-steps), 5 objective product, 6 shot-time scaling,
 * 7 finalize, 8 certificate (z1, its product with the dose block, the sector
 * values of the dual point), 9 GEMM1 and 10 GEMM2 of a refresh iteration of
 * LADMM_BF16 (its other iterations count under 0 and 4).  ms_total and
 * launches are arrays of LADMM_N_KERNEL_CLASSES. */
#define LADMM_N_KERNEL_CLASSES 11
/* Tile configurations chosen for the two dose-matrix products of a batch.
 * Before its first iteration a batch times every tile configuration of the
 * products on its own data and keeps the fastest (cached per case and padded
 * plan count).  The configurations differ only in how the work is split, not
 * in the order of any floating-point sum, so the choice never changes a result.
 * Values are indices into the library's configuration tables. */
int ladmm_batch_tiles(const ladmm_batch *b, int32_t *gemm1, int32_t *gemm2);
/* Pin the tile configurations (no autotuning), for reproducible benchmarks.
 * An index that is not valid for the batch's shapes falls back to 0.
 * LADMM_E_INVALID for an index outside [0, 10) (the FP32 and FP64 products
 * have four configurations, the BF16 products ten, of which 6 to 9 (a
 * ring-pipelined kernel of 64-, 112-, 96- and 448-column tiles) serve
 * LADMM_BF16's single-operand products only; its refresh then runs the pair
 * products in configuration 0). */
int ladmm_batch_set_tiles(ladmm_batch *b, int32_t gemm1, int32_t gemm2);
/* Launch mode of the iterations of the stacked plans (end of Sec. 2.B).  With
 * graphs on (the default) the kernel launches of a run chunk (check_every
 * iterations, the last with statistics) are captured once per chunk length and
 * tile configuration into a HIP graph on the batch's stream and replayed for
 * every later chunk; off, they are launched one by one.  Both
 * run the same kernels on the same arguments, so results are identical.
 * Profiling always launches one by one.  Graphs are destroyed with the batch. */
int ladmm_batch_set_graphs(ladmm_batch *b, int32_t on);
/* Compaction of the running plans (default on).  Between the checks of
 * ladmm_batch_run (and ladmm_solve_batch), when plans have stopped, the
 * running plans' columns (all their state) are moved to the lowest columns and
 * the dose-matrix products launch only as many columns as they occupy (a
 * multiple of 32; for the BF16 blocks one that admits a tile of 64, 96 or 224
 * columns); the plans return to
 * their own columns when the run ends.  A plan's arithmetic does not depend on
 * its column, so results are identical with compaction on or off; only the
 * work on stopped plans is saved. */
int ladmm_batch_set_compaction(ladmm_batch *b, int32_t on);
int ladmm_batch_set_profiling(ladmm_batch *b, int32_t on);
int ladmm_batch_kernel_times(const ladmm_batch *b, double *ms_total, int64_t *launches);

/* One call for the stacked plans of Sec. 2.B: create a batch, run the ADMM
 * iterations of Eq. (admm) to each plan's stopping rule (ladmm_batch_run),
 * write the results as ladmm_batch_results does, destroy the batch.  Errors as
 * ladmm_batch_create, ladmm_batch_run and ladmm_batch_results. */
int ladmm_solve_batch(ladmm_case *c, int32_t k, const ladmm_weights *w,
                      const uint64_t *ld_mask, const ladmm_opts *opts, ladmm_result *out);

/* Low-dose band of Sec. 2.C.1 from the current shot times of a batch: bit v of
 * row j of vol_bits is set iff D_LD <= d_j(v) < D_LD + delta, where
 * d_j = phi_vox t_j is the dose of plan j at candidate voxel v (FP64 product).
 *   phi_vox : host, n_vox x n_t dose rates of the candidate voxels, >= 0.
 *   vol_bits: host output, k x ceil(n_vox/64) words (bit v % 64 of word v/64). */
int ladmm_batch_ld_band(ladmm_batch *b, int64_t n_vox, const double *phi_vox, double d_ld,
                        double delta, uint64_t *vol_bits);

/* Clinical metrics of the batch's plans from their current shot times, on a
 * dose grid (Sec. 2.A; used to compare plans in Sec. 3.B), with the dose
 * d_j(v) = phi_vox(v) t_j computed on the device in FP64:
 *   coverage       = |{v in T : d_j(v) >= D(v)}| / |T|, T the target voxels and
 *                    D(v) the prescription of v's target;
 *   selectivity    = |{v in T : d_j(v) >= D(v)}| / |{v : d_j(v) >= d_ref}|;
 *   gradient index = |{v : d_j(v) >= d_ref / 2}| / |{v : d_j(v) >= d_ref}|;
 *   beam-on time   = sum over isocentres of max over sectors of the summed shot
 *                    times of the sector (in the time unit of the dose rates:
 *                    minutes for Gy/min).
 * With one target (or equal prescriptions) d_ref is the prescription and these
 * are the paper's definitions; with unequal prescriptions the paper defines no
 * global gradient index.
 *   phi_vox:    host, n_vox x n_t dose rates of the grid voxels, >= 0.
 *   vox_target: host, n_vox target indices in [0, n_targets), -1 outside.
 *   presc:      host, n_targets prescription doses > 0.
 *   out:        host, k x 4 (coverage, selectivity, gradient index, beam-on
 *               time); NaN where a denominator is zero.
 * Allocates its scratch for the call. */
int ladmm_batch_metrics(ladmm_batch *b, int64_t n_vox, const double *phi_vox,
                        const int32_t *vox_target, int32_t n_targets, const double *presc,
                        double d_ref, double *out);

/* Algorithm 1 (overlapping low-dose point sampling, Sec. 2.C.2), integer exact.
 * Plans are taken in order of decreasing density w_j = min(1, N_LD,j / |V_j|)
 * (ties: lower index first); a plan with |V_j| = 0 or N_LD,j <= 0 gets no
 * points.  Point counts are round-half-even((N_LD,j / |V_j|) * |X|) in IEEE
 * double, clamped to |X|.  "Randomly select K of X" takes the K members of X
 * with the smallest (h, v), h = sm(sm(sm(seed) ^ step) ^ v), sm the SplitMix64
 * output function, step = 2 r (thinning of the running union) and 2 r + 1
 * (new region) for the plan at rank r.
 *   vol_bits: host, k x ceil(n_vox/64) words, the volumes V_j.
 *   n_ld    : host, k desired point counts N_LD,j.
 *   P       : host output, capacity n_vox; the sorted voxel indices of the union.
 *   nP      : host output, |P|.
 *   masks   : host output, k rows of ceil(n_vox/64) words; bit i % 64 of word
 *             i / 64 of row j is set iff P[i] is in p_j (words past
 *             ceil(|P|/64) are zero).
 * Runs on the context's device; allocates its scratch for the call. */
int ladmm_select_ld_points(ladmm_ctx *ctx, int32_t k, int64_t n_vox, const uint64_t *vol_bits,
                           const int32_t *n_ld, uint64_t seed, int64_t *P, int64_t *nP,
                           uint64_t *masks);

/* The same selection, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, hosts that forbid hipMalloc):
 * it calls no hipMalloc, hipFree or other allocating routine and creates no
 * stream.  Its work arrays, the staged inputs and the outputs live in one
 * library-owned device array of 32 MiB per device (held until the process
 * ends), launched on the null stream.  Arguments, layouts and results are
 * those of ladmm_select_ld_points, bit for bit.  LADMM_E_INVALID when the call
 * needs more than the 32 MiB: 8 (7 + 64 + 3 k) ceil(n_vox/64) + 8 n_vox + 16 k
 * bytes plus alignment, e.g. k = 441 plans of up to 60,000 candidate voxels.
 * Calls on one device share the array and are serialized by the library
 * (the array keeps the last call's contents; every call writes what it reads). */
int ladmm_select_ld_points_static(ladmm_ctx *ctx, int32_t k, int64_t n_vox,
                                  const uint64_t *vol_bits, const int32_t *n_ld, uint64_t seed,
                                  int64_t *P, int64_t *nP, uint64_t *masks);

/* Second pass of the two-pass optimisation (Sec. 2.C): how the low-dose points
 * of the second-pass problem are chosen from the first-pass dose.
 *   n_vox, phi_vox: candidate voxels of the patient volume and their dose rates
 *                   (host, n_vox x n_t, >= 0); the low-dose volume V_j of plan j
 *                   is {v : d_ld <= d_j(v) < d_ld + delta} for the pass-1 dose d_j.
 *   n_ld:           host, k desired point counts N_LD,j (> 0 to sample plan j).
 *   seed:           seed of Algorithm 1's selections.
 *   ld_group:       index (in the pass-1 descriptor's groups) of the low-dose group
 *                   whose points are replaced; every other point is kept as is. */
typedef struct {
  int64_t n_vox;
  const double *phi_vox;
  double d_ld, delta;
  const int32_t *n_ld;
  uint64_t seed;
  int32_t ld_group;
} ladmm_pass2_desc;

/* Both passes for k plans: pass 1 on `pass1`, the band and Algorithm 1 on the
 * device, a new case whose low-dose block is the shared point set P (new row
 * scales, beta, Schur complement and factor, Sec. 2.C.2), and pass 2 with plan
 * j's low-dose bound u restricted to its own subset p_j.  Pass 2 starts from
 * zero iterates.
 *   pass1_out: optional per-plan results of pass 1 (NULL to skip).
 *   out:       per-plan results of pass 2 (t in pass-2 shot order = pass-1 order).
 *   P:         optional host output, capacity n_vox: the selected voxel indices.
 *   n_points2: optional host output: |P| (first), then the pass-2 point count.
 *   times_ms:  optional host output[5]: wall time of pass-1 setup, pass-1 solve,
 *              band + Algorithm 1, pass-2 setup, pass-2 solve.
 * Device memory: pass 1's dose rates (FP64, n_points x n_t x 8 bytes) stay on
 * the device for the whole call, beside the context's budget; the pass-2 block
 * is gathered from them and only the selected rows of phi_vox are uploaded.
 * LADMM_E_DEVICE when these allocations or copies fail. */
int ladmm_two_pass(ladmm_ctx *ctx, const ladmm_case_desc *pass1, int32_t k,
                   const ladmm_weights *w, const ladmm_opts *opts, const ladmm_pass2_desc *p2,
                   ladmm_result *pass1_out, ladmm_result *out, int64_t *P, int64_t *n_points2,
                   double *times_ms);

/* The same with several low-dose groups replaced at once (App. A: two low-dose
 * thresholds D_1,LD and D_2,LD, each with its own volume [D_i,LD, D_i,LD +
 * Delta), in both passes).  Set i gives the threshold, candidates, counts and
 * seed of the group sets[i].ld_group (distinct groups); its band and its
 * Algorithm 1 selection are computed from the same pass-1 dose, and the pass-2
 * case appends the selected points of every set, in set order, each in its own
 * group, with plan j's bound restricted to its own subsets.
 *   P:         optional host output, capacity sum of n_vox: the selected voxel
 *              indices of every set, concatenated in set order (each set's
 *              indices refer to its own candidates).
 *   n_points2: optional host output[n_sets + 1]: |P_i| per set, then the pass-2
 *              point count.
 * ladmm_two_pass is this call with one set. */
int ladmm_two_pass_sets(ladmm_ctx *ctx, const ladmm_case_desc *pass1, int32_t k,
                        const ladmm_weights *w, const ladmm_opts *opts, int32_t n_sets,
                        const ladmm_pass2_desc *sets, ladmm_result *pass1_out, ladmm_result *out,
                        int64_t *P, int64_t *n_points2, double *times_ms);

/* More than two passes (Sec. 2.C repeated): pass p + 1 takes its low-dose
 * points from the dose of pass p by the same band and Algorithm 1 steps (each
 * set with its own threshold and seed), on the points of pass 1 outside the
 * replaced groups; every pass starts from zero iterates.
 *   n_passes:  >= 2 (2 is ladmm_two_pass_sets), at most 64.
 *   pass_out:  optional array of n_passes result records (entry p: pass p + 1;
 *              NULL pointers inside a record are skipped).
 *   P, n_points: as for ladmm_two_pass_sets, for the last pass.
 *   times_ms:  optional host output[2 + 3 (n_passes - 1)]: pass-1 setup and
 *              solve, then per later pass band + Algorithm 1, setup, solve. */
int ladmm_passes(ladmm_ctx *ctx, const ladmm_case_desc *pass1, int32_t k, const ladmm_weights *w,
                 const ladmm_opts *opts, int32_t n_sets, const ladmm_pass2_desc *sets,
                 int32_t n_passes, ladmm_result *pass_out, int64_t *P, int64_t *n_points,
                 double *times_ms);

/* ---- Serving: continuous batching of plan requests ---------------------------
 *
 * Plans of one case are independent columns that share the dose block and the
 * Schur complement inverse (end of Sec. 2.B); only b, u and the step size
 * (Eq. rho_rule) are per plan.  A server keeps one slot batch ("lane") per case
 * with work and one worker thread.  Between chunks of check_every iterations it
 * retires finished plans and admits queued ones (oldest request first) into the
 * free slots; lanes of different cases run on their own streams and overlap on
 * the device.  A plan's arithmetic does not depend on the other slots, so its
 * result is bitwise that of ladmm_solve_batch on the plan alone with the same
 * options (max_iter a multiple of check_every).  Lane memory is charged to the
 * context's HBM budget: when a new lane does not fit, idle lanes are released
 * (least recently used first) and otherwise the request waits for busy lanes;
 * a request that cannot fit even on an otherwise empty device fails with
 * LADMM_E_NOMEM.
 *
 * Warm starts (warm_store > 0): each lane keeps the final iterates of up to
 * warm_store converged plans of its case in HBM (charged to the budget, oldest
 * replaced first).  A newly admitted plan then starts from the stored plan with
 * the nearest weighting instead of from zero: its q = z + y, z2 + y2 and sector
 * columns are copied, z and y follow from its own bounds, and it takes the
 * stored plan's final step size.  The distance is Euclidean over (w_t, w_r,
 * w_ld, log10(w_BOT) / 3), the slider coordinates of a weighting.  ADMM
 * converges from any start, so a warm-started plan reaches the same optimum in
 * fewer iterations; its result matches the plan solved alone within the
 * stopping tolerance, not bitwise.  With warm_store = 0 every plan starts cold
 * and the bitwise statement above holds.
 *
 *   slots:       plan columns per lane, rounded up to a multiple of 32; [1, 4096].
 *   check_every: iterations per chunk; admission, the stopping test and
 *                retirement happen between chunks.  >= 1.
 *   max_lanes:   at most this many cases hold lane memory at once (0: no limit
 *                besides the HBM budget).
 *   autotune:    time the tile configurations when a lane is created.
 *   eager:       nonzero: launch each lane's kernels one by one instead of
 *                replaying a captured graph per chunk (ladmm_batch_set_graphs).
 *   warm_store:  solved plans kept per lane for warm starts; [0, 65536]. */
typedef struct {
  int32_t slots;
  int32_t check_every;
  int32_t max_lanes;
  int32_t autotune;
  int32_t eager;
  int32_t warm_store;
} ladmm_server_opts;

/* Counters of a server.  Latencies (submit to final status, completed requests
 * only) are nearest-rank percentiles in milliseconds; busy_ms is the wall time
 * of worker rounds that ran at least one lane; plan_iterations counts every
 * iteration of every occupied slot; warm_starts counts plans admitted from a
 * stored plan. */
typedef struct {
  int64_t submitted, completed, cancelled, failed;
  int64_t plans_completed, plan_iterations, warm_starts;
  double p50_ms, p99_ms, max_ms, mean_ms, busy_ms;
  int32_t lanes, busy_slots;
} ladmm_server_stats;

typedef struct ladmm_server ladmm_server;

/* Start a server (and its worker thread) on a context.  The context must
 * outlive the server.  LADMM_E_INVALID for options out of range. */
int ladmm_server_create(ladmm_ctx *ctx, const ladmm_server_opts *opts, ladmm_server **out);
/* Stop the worker, cancel every request that is not final, release the lanes
 * and the server.  No other call on the server may be in progress or follow. */
int ladmm_server_destroy(ladmm_server *s);
/* Queue k plans of case c (same context as the server).  w, ld_mask (NULL or
 * k rows of ceil(n_points/64) words, bit p of a row = LD point p kept, as in
 * ladmm_batch_create) and opts are copied.  opts->check_every must be 0 or the
 * server's; max_iter (>= 1) is rounded up to a multiple of it; autotune is the
 * server's.  `out` is copied: its buffers (sized for k plans) must stay valid
 * until the request's final status has been reported, and are written plan by
 * plan as plans finish.  *ticket identifies the request.  The case must not be
 * destroyed before its requests are final (queued requests of a destroyed case
 * whose lane was released fail with LADMM_E_STATE). */
int ladmm_submit(ladmm_server *s, ladmm_case *c, int32_t k, const ladmm_weights *w,
                 const uint64_t *ld_mask, const ladmm_opts *opts, ladmm_result *out,
                 uint64_t *ticket);
/* Non-blocking status: LADMM_PENDING while plans remain, else the final status
 * (LADMM_OK, LADMM_E_CANCELLED or the error that stopped the request).
 * *plans_done (optional) = plans retired so far.  The first call that reports a
 * final status releases the ticket; later calls return LADMM_E_STATE. */
int ladmm_poll(ladmm_server *s, uint64_t ticket, int32_t *plans_done);
/* Block until the request is final (timeout_us < 0: no limit), then as
 * ladmm_poll; LADMM_PENDING on timeout.  One waiter per ticket. */
int ladmm_wait(ladmm_server *s, uint64_t ticket, int64_t timeout_us);
/* Ask for a request to stop: its queued plans are dropped and its running
 * plans are freed at the next chunk boundary; its final status becomes
 * LADMM_E_CANCELLED (plans already retired keep their results).  LADMM_OK
 * also when the request is already final. */
int ladmm_cancel(ladmm_server *s, uint64_t ticket);
int ladmm_server_get_stats(ladmm_server *s, ladmm_server_stats *out);
/* Zero the counters and the latency record (lanes, stores and queued work are
 * kept), e.g. after a warm-up phase. */
int ladmm_server_reset_stats(ladmm_server *s);

/* Message for the last error returned on this thread ("" if none). */
const char *ladmm_last_error(void);
/* Library version string. */
const char *ladmm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LADMM_H */
