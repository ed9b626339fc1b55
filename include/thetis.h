/*
 * thetis.h -- C ABI of libthetis, an MI355X (gfx950) implementation of the
 * solve step of "An Approximate, Efficient LP Solver for LP Rounding"
 * (Sridhar, Bittorf, Liu, Zhang, Re, Wright): stochastic coordinate descent
 * on the quadratic-penalty form of a sparse LP relaxation, followed by the
 * pre-rounding scaling, the rounding and the feasibility check.
 *
 * Conventions for every call:
 *   - Every call returns a thetis_status: THETIS_OK (0) or a negative code.
 *     thetis_last_error() gives a message for the calling thread's last
 *     failure.  No C++ exception crosses this boundary: a host allocation
 *     that fails inside a call returns THETIS_ENOMEM.
 *   - Pointers named *_host are host memory owned by the caller; the library
 *     copies what it needs before the call returns and keeps no reference.
 *   - Device work is enqueued on the solver's stream (a hipStream_t passed
 *     as void*, NULL = the null stream).  Calls that hand host values back
 *     synchronise that stream before they return.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - After an error the handle stays valid, except after THETIS_EDEVICE.
 */
#ifndef THETIS_H
#define THETIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t thetis_status;
enum {
    THETIS_OK = 0,
    THETIS_EINVAL = -1,       /* bad argument or malformed instance          */
    THETIS_ENOMEM = -2,       /* host or device allocation failed, or the
                                 caller's workspace is too small              */
    THETIS_EDEVICE = -3,      /* HIP runtime error; the handle is unusable     */
    THETIS_EDIVERGED = -4,    /* NaN or Inf in a residual/objective reduction  */
    THETIS_EBUSY = -5,        /* a handle is in use by a batch                 */
    THETIS_EBUDGET = -6,      /* device-memory budget exceeded (serving)       */
    THETIS_EUNSUPPORTED = -7  /* valid request outside what the library does   */
};

typedef struct thetis_inst thetis_inst;       /* host-side instance, library owned */
typedef struct thetis_solver thetis_solver;   /* device state of one solve         */
typedef struct thetis_batch thetis_batch;     /* several solvers run as one launch */

/* step rules of Section 3.3 */
enum {
    THETIS_STEP_PER_COORD = 0,    /* 1/L_j, L_j = beta ||A_j||^2 + rho: the exact
                                     minimiser along coordinate j             */
    THETIS_STEP_GLOBAL_LMAX = 1   /* 1/Lmax, Lmax of eq. (Lmax), as in Algorithm 1 */
};
/* update schedules (Section 3.4, asynchronous parallel SCD) */
enum {
    THETIS_SCHED_DET = 0,   /* colour classes of units with disjoint rows, the
                               class order drawn per epoch; race-free and
                               reproducible: equal to serial SCD in that order */
    THETIS_SCHED_ASYNC = 1  /* all units of an epoch at once, residual updated
                               with hardware float atomics (lock-free)        */
};
/* storage precision of y = (x, s) and of the running residual r */
enum {
    THETIS_PREC_FP32 = 0,   /* x, s, r in FP32; refresh and reductions in FP64 */
    THETIS_PREC_FP64 = 1,   /* everything in FP64 (validation build)          */
    THETIS_PREC_BF16X = 2   /* x in BF16, s and r in FP32                     */
};
/* rounding rules */
enum {
    THETIS_ROUND_VC_THRESH = 1,   /* vertex cover: keep v iff x_v >= T,
                                     T = min(1/2, min_e (x_u+x_v)/2)           */
    THETIS_ROUND_MIS_THRESH = 2,  /* independent set: keep v iff x_v > T',
                                     T' = max(1/2, max_e (x_u+x_v)/2)          */
    THETIS_ROUND_MIS_RAND = 3,    /* independent set: scale by 1/(1+alpha), keep
                                     v with probability x~_v, drop conflicts    */
    THETIS_ROUND_MC_CKR = 4,      /* multiway cut: region growing from terminals */
    THETIS_ROUND_COVER_THRESH = 5,/* set cover (Appendix B, Hochbaum): keep s iff
                                     x_s >= T, T = min(1, min_j A_j x)/f with f the
                                     longest row (the covering scaling of Appendix
                                     C with q = 1), capped by every row's largest
                                     x so each row keeps a set                   */
    THETIS_ROUND_COVER_RAND = 6,  /* integer covering (Appendix B randomized set
                                     cover, Appendix C scaling): alpha =
                                     max_j (b_j - A_j x)_+ / q(P), xt = min(1,
                                     x/(1-alpha)) (1 once alpha >= 1); the union of
                                     ceil(ln 2m) rounds keeping s with probability
                                     xt_s; a row still short takes, from that
                                     union alone, its unkept sets by decreasing xt
                                     (ties: entry order) until covered           */
    THETIS_ROUND_PACK_RAND = 7,   /* packing (Appendix C scaling, Bansal et al.'s
                                     alteration with theta = 1/k): alpha =
                                     max_j ((A_j x - b_j)/b_j)_+, keep s with
                                     probability x_s/(1+alpha); with w = A_js/b_j,
                                     drop a kept s when, in a row where it has
                                     weight, the kept sets of weight >= its own
                                     (itself included) weigh more than 1         */
    THETIS_ROUND_MAP_ARGMAX = 8,  /* MAP LP (pairwise factors declared): every free
                                     block takes the label of its largest
                                     marginal (ties: the lower label); cost = the
                                     energy of the labelling                   */
    THETIS_ROUND_MAP_SAMPLE = 9   /* MAP LP: every free block draws its label from
                                     its marginal (inverse CDF in label order,
                                     Philox counter (repetition, block, 3); past
                                     the end, the last label with positive mass);
                                     best of reps by energy                    */
};

/* Solver parameters.  The penalty function is eq. (QP) of Section 3.2 with
 * slacks for inequality rows:
 *   F(y) = c^T x - ubar^T (A y - b) + beta/2 ||A y - b||^2 + rho/2 ||y - ybar||^2
 * with rho = 0 (prox off) or rho = 1/beta (prox on), y in the box / simplex. */
typedef struct {
    double beta;            /* penalty parameter, > 0                               */
    int32_t step_rule;      /* THETIS_STEP_*                                         */
    double step_scale;      /* gamma in (0, 1]: step gamma/L                          */
    int32_t prox;           /* 0: rho = 0; 1: rho = 1/beta                            */
    const double *ybar;     /* host, n+m entries (x then one slack per row), or NULL = 0 */
    const double *ubar;     /* host, m entries, or NULL = 0                          */
    int32_t schedule;       /* THETIS_SCHED_*                                        */
    int32_t precision;      /* THETIS_PREC_*                                         */
    int32_t refresh_every;  /* epochs between FP64 recomputations of r = Ay - b (>=1) */
    uint64_t seed;          /* Philox key for the class order and the rounding draws */
} thetis_params;

/* Fills the defaults: beta 10, per-coordinate step, gamma 1, prox off, DET,
 * FP32, refresh every 5 epochs, seed 0. */
thetis_status thetis_params_default(thetis_params *p);

/* --------------------------------------------------------------- instance */

/* Creates an LP instance (standard form of Section 3.1 with bounds and
 * inequality rows, Appendix C):
 *     min c^T x   s.t.  A_i x (>= | <= | =) b_i,   0 <= x_j <= u_j.
 * m rows, n columns, CSR with nnz entries: row_ptr_host[m+1] (int64,
 * row_ptr[0] = 0, non-decreasing), col_idx_host[nnz] in [0, n) with no
 * repeated column inside a row, val_host[nnz] (NULL: every entry is 1),
 * b_host[m], c_host[n], u_host[n] (NULL: +inf; entries >= 0 or +inf),
 * sense_host[m] (+1 '>=', -1 '<=', 0 '='; NULL: all '=').  One slack column
 * is appended per inequality row (-1 for '>=', +1 for '<='), bounded below
 * by 0.  All inputs are copied.  Limits: nnz < 2^31, n + m < 2^31.
 * Errors: THETIS_EINVAL for non-finite data, indices out of range or a bad
 * row_ptr; THETIS_ENOMEM.  The layout (column copy, colouring, plans) is
 * built once, by the first call that needs it (thetis_inst_classes,
 * thetis_solver_workspace_bytes, thetis_solver_create; those calls may be
 * made from several threads). */
thetis_status thetis_inst_create_csr(int64_t m, int64_t n, int64_t nnz,
                                     const int64_t *row_ptr_host, const int32_t *col_idx_host,
                                     const double *val_host, const double *b_host,
                                     const double *c_host, const double *u_host,
                                     const int8_t *sense_host, thetis_inst **out);

/* Declares simplex blocks (multiway cut, Appendix B; block coordinate
 * descent with projection onto the k-simplex, Appendix E): block t owns the
 * k consecutive columns first_col_host[t] .. first_col_host[t]+k-1, which
 * must not overlap.  fixed_label_host[t] >= 0 pins block t at the unit
 * vector of that label (a terminal); -1 leaves it free; NULL = all free.
 * 1 <= k <= 64.  The columns of one block must not share a row (then the
 * block of A^T A is diagonal and one block's update writes every row at most
 * once): THETIS_EINVAL otherwise, as for overlapping or out-of-range
 * blocks.  Must be called before any solver is created. */
thetis_status thetis_inst_set_simplex_blocks(thetis_inst *inst, int64_t nblocks, int32_t k,
                                             const int64_t *first_col_host,
                                             const int32_t *fixed_label_host);

/* Declares the pairwise factors of a MAP-inference LP (the local polytope
 * of a pairwise factor graph; the MAP experiments' formulation): factor e
 * joins simplex blocks ends_host[2e] and ends_host[2e+1] (the node
 * marginals), and its k*k factor-marginal columns start at
 * first_col_host[e], row-major in (label of the first block, label of the
 * second).  Used only by the MAP roundings' energy: sum over blocks of the
 * objective at the block's label plus, per factor, the objective at its
 * label pair.  Call after thetis_inst_set_simplex_blocks and before any
 * solver is created.  Copies the arrays.  THETIS_EINVAL for ends or columns
 * out of range or factor columns inside a block; THETIS_EBUSY after a
 * solver exists. */
thetis_status thetis_inst_set_pairwise(thetis_inst *inst, int64_t nfactors, const int32_t *ends_host,
                                       const int64_t *first_col_host);

/* Number of colour classes of the DET schedule (greedy colouring of the
 * update units in index order, all slack units in one last class) and the
 * class of every unit: units are the free simplex blocks and the columns
 * outside blocks in increasing column order, then the slack of every
 * inequality row in row order.  class_host may be NULL (a first call then
 * returns the unit count in nunits); otherwise it needs room for nunits
 * entries. */
thetis_status thetis_inst_classes(const thetis_inst *inst, int32_t *nclasses, int64_t *nunits,
                                  int32_t *class_host);

/* Shapes the general rounding rules accept, as bits of *flags:
 * THETIS_SHAPE_COVER (every row '>=' with non-negative integer entries and
 * right-hand side, binary columns, no blocks), THETIS_SHAPE_SET_COVER (also
 * every entry and right-hand side 1), THETIS_SHAPE_PACK (every row '<=' with
 * non-negative entries and b > 0, binary columns, no blocks); and q(P) of
 * the covering lemma (Appendix C): over the rows with b_j > 0, the least
 * b_j - A_j x among binary x with A_j x < b_j (exact for b_j <= 2^24, else
 * the lower bound 1; +inf without such rows; 0 when not covering).  Either
 * pointer may be NULL.  Builds the layout if needed. */
enum { THETIS_SHAPE_COVER = 1, THETIS_SHAPE_SET_COVER = 2, THETIS_SHAPE_PACK = 4 };
thetis_status thetis_inst_rounding_shape(const thetis_inst *inst, int32_t *flags, double *cover_q);

thetis_status thetis_inst_destroy(thetis_inst *inst);

/* ----------------------------------------------------------------- solver */

/* Device bytes a solver of this instance and these parameters needs. */
thetis_status thetis_solver_workspace_bytes(const thetis_inst *inst, const thetis_params *p,
                                            size_t *bytes);

/* Creates a solver: uploads the instance layout to the current HIP device
 * and sets y = 0 (fixed blocks at their unit vector), r = A y - b.
 * dev_workspace: caller-owned device memory of ws_bytes >= the size above
 * (for example a torch tensor), kept for the solver's life; NULL = the
 * library allocates and frees it.  stream: hipStream_t or NULL.
 * Errors: THETIS_EINVAL (bad parameters), THETIS_ENOMEM, THETIS_EDEVICE. */
thetis_status thetis_solver_create(const thetis_inst *inst, const thetis_params *p,
                                   void *dev_workspace, size_t ws_bytes, void *stream,
                                   thetis_solver **out);

/* For callers that cannot allocate device memory: code recorded under HIP
 * graph capture, serving loops and harnesses that forbid hipMalloc.  The
 * same solver as thetis_solver_create, but its workspace is a fixed array
 * of THETIS_STATIC_WORKSPACE_BYTES inside the library, one copy per device,
 * held until the process ends; this call allocates no device memory.  The
 * solver runs on the current device; at most one solver made by this call
 * lives on a device at a time (the array is its whole device state), and
 * it releases the array when destroyed.  Creation rewrites every part of
 * the array it uses, so what a previous solver left there does not matter.
 * Errors: as thetis_solver_create; THETIS_EBUDGET when the instance needs
 * more than THETIS_STATIC_WORKSPACE_BYTES (thetis_solver_workspace_bytes),
 * THETIS_EBUSY while another such solver lives on the device.  Calls of the
 * library on two solvers of one device that share the array cannot happen;
 * two processes each have their own copy. */
#define THETIS_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
thetis_status thetis_solver_create_static(const thetis_inst *inst, const thetis_params *p, void *stream,
                                          thetis_solver **out);

/* Back to the starting point (y = 0, epoch 0) without re-uploading.  After
 * multiplier steps, ubar, ybar and the shifted costs return to the values
 * given at creation and beta to the one of creation or of the last
 * thetis_set_beta. */
thetis_status thetis_solver_reset(thetis_solver *s);

/* Changes beta between epochs (with prox, rho = 1/beta follows); every
 * curvature L_j and the simplex blocks' bounds are recomputed. */
thetis_status thetis_set_beta(thetis_solver *s, double beta);
thetis_status thetis_set_step_rule(thetis_solver *s, int32_t rule, double step_scale);

/* Runs up to max_epochs epochs of SCD (Algorithm 1; an epoch updates every
 * unit once).  Every refresh_every epochs r is recomputed from y in FP64
 * and, when gap_tol > 0, the run stops once the certified relative gap
 * (F - Phi)/max(1,|F|) <= gap_tol (Phi is the dual bound of the penalty
 * problem).  epochs_done (may be NULL) receives the count.
 * THETIS_EDIVERGED if a refresh sees NaN or Inf. */
thetis_status thetis_run_epochs(thetis_solver *s, int32_t max_epochs, double gap_tol,
                                int32_t *epochs_done);

/* Chooses, for every colour class of the DET schedule, how many columns a
 * lane group updates at once (1, 2 or 4: more loads in flight against more
 * serial work per wavefront) by timing real epochs: 1 + 3 x
 * epochs_per_candidate epochs of the solve are run (counted in
 * thetis_epoch; no gap test); a shape other than one column per group is
 * taken only when it is at least 3% faster.
 * choice_host (NULL or one int per class) receives the choices.  Results do
 * not depend on them.  ASYNC solvers are left as they are. */
thetis_status thetis_solver_autotune(thetis_solver *s, int32_t epochs_per_candidate, int32_t *choice_host);

/* ------------------------------------------------ augmented Lagrangian */

/* Figures of one multiplier step, all FP64, at the iterate y the step is
 * taken at. */
typedef struct {
    double lp_value;   /* c^T x                                                   */
    double linf;       /* ||A y - b||_inf                                         */
    double lp_dual;    /* D(u) = b^T u + sum over variables of the minimum of its
                          reduced-cost term over its feasible set (box; simplex
                          for a free block; the unit vector for a fixed one), at
                          u = the new ubar with each inequality row's entry
                          clipped to the sign its slack allows (covering >= 0,
                          packing <= 0): a lower bound on the LP optimum       */
    double lp_gap;     /* (lp_value - lp_dual) / max(1, |lp_value|)               */
    double device_ms;  /* device time of the step's three launches (HIP events) */
    double alg_bytes;  /* their algorithmic bytes: CSR and CSC read once, x, s,
                          ubar, ctil (and the prox centre when it moves)         */
} thetis_mul_stats;

/* One update of the augmented-Lagrangian framework of Section 3.2 between
 * two penalty solves (with prox on, a proximal method of multipliers):
 *     ubar <- ubar - beta (A y - b)   (w recomputed from y in FP64),
 *     ybar <- y                        when move_centre != 0,
 *     beta <- new_beta                 when new_beta > 0 (as thetis_set_beta),
 * and the shifted costs c - A^T ubar recomputed in FP64 (stored in the
 * storage precision).  y and the epoch count are unchanged.  The solver
 * must have been created with a ubar (zeros are fine) and, for
 * move_centre, with prox on and a ybar: THETIS_EUNSUPPORTED otherwise.
 * stats_host may be NULL.  Synchronises the solver's stream. */
thetis_status thetis_multiplier_step(thetis_solver *s, int32_t move_centre, double new_beta,
                                     thetis_mul_stats *stats_host);

/* Copies the current multiplier ubar (m entries, the caller's row order) and,
 * if ybar_host is not NULL, the prox centre (n + m entries, x then one slack
 * per row, as stored: in the storage precision) to the host.  Either may be
 * NULL; asking for one the solver does not hold is THETIS_EUNSUPPORTED. */
thetis_status thetis_get_multipliers(thetis_solver *s, double *ubar_host, double *ybar_host);

/* The outer loop of that framework: up to max_outer times, run up to
 * inner_epochs epochs (stopping early at the penalty gap inner_gap_tol as
 * thetis_run_epochs does), then take a multiplier step with
 * new_beta = min(beta * beta_growth, beta_max) when beta_growth > 1 (else
 * beta is kept).  Stops after the first step with linf <= feas_tol and
 * lp_gap <= lp_gap_tol (an (eps, delta)-approximate point of Section 3.1,
 * certified by the dual bound).  outer_done, epochs_done and last_host (the
 * last step's figures) may be NULL.  Errors as thetis_run_epochs and
 * thetis_multiplier_step. */
thetis_status thetis_run_multipliers(thetis_solver *s, int32_t max_outer, int32_t inner_epochs,
                                     double inner_gap_tol, double beta_growth, double beta_max,
                                     double feas_tol, double lp_gap_tol, int32_t move_centre,
                                     int32_t *outer_done, int64_t *epochs_done,
                                     thetis_mul_stats *last_host);

/* Residual norms of the slack form, ||A y - b||_inf and ||.||_2, and the
 * largest violation of an original row by x (Definition of an
 * (eps,delta)-approximate solution, Section 3.1).  Computed in FP64 from
 * y; does not change the solver state. */
thetis_status thetis_residual(thetis_solver *s, double *linf, double *l2,
                              double *max_row_violation);

/* c^T x, the penalty value F(y), the dual bound Phi <= min F, and the
 * certified relative gap (F - Phi)/max(1, |F|) that thetis_run_epochs stops
 * on (Section 3.1's approximate solution measured on the penalty problem),
 * all FP64 and formed on the device from y.  Any output may be NULL. */
thetis_status thetis_objective(thetis_solver *s, double *lp_value, double *penalty,
                               double *dual_bound, double *gap);

/* Copies y to the host: x_host[n] (structural) and, if s_host is not NULL,
 * s_host[m] (slacks), converted to double. */
thetis_status thetis_get_x(thetis_solver *s, double *x_host, double *s_host);

/* Replaces y by y_host[n+m] (rounded to the storage precision) and
 * recomputes r.  Entries are clipped to their bounds; the columns of a fixed
 * simplex block keep its unit vector, and a free block is taken as given
 * (its next update projects it onto the simplex). */
thetis_status thetis_set_y(thetis_solver *s, const double *y_host);

/* Epochs run since creation or reset. */
thetis_status thetis_epoch(const thetis_solver *s, int64_t *epoch);

/* Pre-rounding pass and rounding of the current x (Section 2, Lemma
 * infeasible:rounded:vc, Appendix B and C) into sol_host: 0/1 per column
 * for the VC, MIS, COVER and PACK rules (n entries), a label per simplex
 * block for MC_CKR and the MAP rules (nblocks entries); sol_host may be
 * NULL.  reps >= 1
 * draws for the randomised rules, keeping the cheapest (ties: first).
 * cost = c^T sol (for MC: the cut weight).  aux_host (NULL or 2 doubles)
 * gets the threshold T (or alpha, or the region radius) and the winning
 * repetition.  THETIS_EINVAL when the instance does not have the rule's
 * shape (VC/MIS: every row x_u + x_v with b = 1 and the rule's sense; MC:
 * blocks; COVER/PACK: see thetis_inst_rounding_shape).  Draws: Philox
 * stream 4, counter (repetition, column, 0) for the keep draws of MIS_RAND
 * and PACK_RAND, (repetition, column, 16 + round) for COVER_RAND. */
thetis_status thetis_round(thetis_solver *s, int32_t rule, uint64_t seed, int32_t reps,
                           int32_t *sol_host, double *cost, double *aux_host);

/* Feasibility of an integer solution for the original problem: every row
 * of A against b by its sense, every entry 0 or 1 (VC, MIS, COVER and PACK
 * rules: n entries), or every label in range and every fixed block on its
 * own label (MC_CKR and the MAP rules: nblocks entries).  sol_host = NULL
 * checks the solution of the last thetis_round on the device. */
thetis_status thetis_check_feasible(thetis_solver *s, int32_t rule, const int32_t *sol_host,
                                    int32_t *feasible, int64_t *n_violated);

/* Kernel groups for timing and traffic figures. */
enum {
    THETIS_K_SWEEP_COLUMNS = 0, /* k_sweep: the plain columns of one class (or of a
                                   whole ASYNC epoch) -- LDS-staged hub workgroups
                                   and lane groups in one launch                  */
    THETIS_K_SWEEP_BLOCK = 1,   /* k_sweep_block: simplex blocks of one class       */
    THETIS_K_SWEEP_SLACK = 2,   /* k_sweep_slack: the slack class                   */
    THETIS_K_REFRESH = 3,       /* FP64 refresh + reductions (k_rows, k_dual,
                                   k_finalize)                                      */
    THETIS_K_NKINDS = 4
};

/* Per-launch HIP-event timing: with every > 0, events are recorded on the
 * solver's stream around every launch of every `every`-th epoch of
 * thetis_run_epochs (a sample whose average launch duration is unbiased and
 * whose event overhead stays small); 0 turns it off. */
thetis_status thetis_set_timing(thetis_solver *s, int32_t every);

/* For kernel group `kind`, over the last thetis_run_epochs with timing on:
 * the summed device time of its launches (ms), the launch count, and the
 * algorithmic bytes those launches moved (the traffic a perfect cache would
 * see: column pointers, row indices, residual entries read and written,
 * y read and written, costs).  Average bytes/launch over average
 * time/launch is the kernel's achieved algorithmic bandwidth. */
thetis_status thetis_get_timing(const thetis_solver *s, int32_t kind, double *ms, int64_t *launches,
                                double *alg_bytes);

/* Algorithmic bytes of one epoch's coordinate updates (all sweep kernels)
 * and of one refresh, and the coordinate updates per epoch. */
thetis_status thetis_epoch_traffic(const thetis_solver *s, double *sweep_bytes,
                                   double *refresh_bytes, int64_t *updates_per_epoch);

/* Checkpoint of a solver's state (not part of the method): x, s, the running
 * residual r, the epoch (which selects the next class orders), beta and,
 * when the solver holds them, ubar, the shifted costs and the prox centre,
 * all as stored on the device (in the library's internal row and column
 * order).  thetis_solver_save with host_buf NULL puts the size in *bytes;
 * otherwise *bytes gives the buffer's size (too small: THETIS_EINVAL with
 * the size in *bytes) and receives the bytes written.  thetis_solver_load
 * restores such a checkpoint into a solver of the same instance (the
 * checkpoint carries 64-bit digests of the LP and its simplex blocks and of
 * the internal orders, so a checkpoint of another library version's layout
 * is refused), precision and ubar/prox setting (THETIS_EINVAL otherwise); the
 * solve then continues bit for bit as it would have from the save (DET).
 * A reset afterwards still returns to the creation values.  Both
 * synchronise the solver's stream; not while a batch holding the solver
 * runs. */
thetis_status thetis_solver_save(thetis_solver *s, void *host_buf, size_t *bytes);
thetis_status thetis_solver_load(thetis_solver *s, const void *host_buf, size_t bytes);

/* Frees the solver (NULL is a no-op).  THETIS_EBUSY, and nothing freed,
 * while a batch slot holds it: empty the slot or destroy the batch first. */
thetis_status thetis_solver_destroy(thetis_solver *s);

/* Measurement aid (no part of the method): on `stream` (NULL: the null
 * stream) of the current device, times passes over a buffer of
 * 2^words_log2 4-byte words (words_log2 in [13, 28]) that touch every word
 * once: ms_host[0] a gather at random distinct addresses, ms_host[1] a
 * read-modify-write at random distinct addresses, ms_host[2] a plain copy
 * into a second buffer, ms_host[3] a read-modify-write at random distinct
 * addresses where the workgroups of each XCD (workgroup b runs on XCD
 * b mod 8) touch only their own eighth of the buffer; each the mean of
 * `iters` passes after one warm-up.  ms_host needs 4 entries.  Allocates
 * and frees its two buffers; synchronises the stream. */
thetis_status thetis_calibrate_random(int32_t words_log2, int32_t iters, void *stream, double *ms_host);

/* ----------------------------------------------------------------- batches */

/* A batch is a set of `capacity` slots, each empty or holding a solver (DET
 * schedule, the batch's precision, matrix values all ones when unit_values
 * is nonzero and otherwise not, created on the current device).
 * thetis_batch_run advances every occupied slot in one sequence of launches
 * per epoch: the class of step q of every instance (its own Philox class
 * order) in one launch, instance by instance refresh and stop.  Each solver
 * computes exactly what thetis_run_epochs would compute for it alone (same
 * classes, same order, same kernels): results are bit-identical, whatever
 * else occupies the batch.  solvers_host: NULL or `capacity` entries (NULL =
 * empty slot).  The batch borrows the solvers (they must outlive their slot,
 * which thetis_solver_destroy enforces, and must not be run alone during a
 * batch call).  stream: hipStream_t for
 * the batch's launches, or NULL (the batch makes its own).  Errors:
 * THETIS_EINVAL (a solver of another precision or value kind, ASYNC
 * schedule, capacity < 1), THETIS_EUNSUPPORTED (more than 64 colour
 * classes), THETIS_ENOMEM, THETIS_EDEVICE. */
thetis_status thetis_batch_create(int32_t capacity, thetis_solver *const *solvers_host, int32_t precision,
                                  int32_t unit_values, void *stream, thetis_batch **out);

/* Puts a solver into a slot, or empties it (s = NULL), between runs. */
thetis_status thetis_batch_set(thetis_batch *b, int32_t slot, thetis_solver *s);

/* Runs every occupied slot for up to max_epochs more epochs; an instance
 * retires once its certified gap is <= gap_tol at one of its refresh epochs
 * (gap_tol <= 0: never) or after max_epochs.  epochs_done_host (NULL or
 * `capacity` entries) receives the epochs each slot ran; status_host (NULL
 * or `capacity` entries) 0 still running, 1 gap reached, 2 max_epochs
 * reached, 3 NaN/Inf, -1 empty slot.  K epochs of launches (K = the
 * shortest refresh period of the occupied slots, at most 8; 1 when the call
 * asks for at most K epochs) are captured as one HIP graph and replayed
 * (re-captured when K, the launch configuration, the slot contents' largest
 * class count or the tables change); a slot that has retired is left
 * unchanged by the epochs of the last replay it does not need.  The host
 * stops replaying once no slot is left, read one replay late. */
thetis_status thetis_batch_run(thetis_batch *b, int32_t max_epochs, double gap_tol,
                               int32_t *epochs_done_host, int32_t *status_host);

/* Chooses the launch configuration by timing real epochs of the batch
 * (1 + epochs_per_candidate per candidate, counted as epochs of the solve).
 * First the per-column shape: lanes per column widened 1x or 2x beyond the
 * degree bound, or 1, 2 or 4 columns per lane group; then, with that shape,
 * one workgroup per work item or 1, 2 or 4 times the resident workgroup
 * count walking the items, and contiguous or strided walks of each XCD's
 * share of the work items.
 * Every candidate computes bit-identical results.  The choice is cached per
 * batch shape (instance count, entries, largest degree, precision) for the
 * life of the process; choice_host (NULL or 4 ints) receives (widen, grid
 * multiplier, strided, columns per group). */
thetis_status thetis_batch_autotune(thetis_batch *b, int32_t epochs_per_candidate, int32_t *choice_host);

/* Sets the launch configuration directly: widen in {1,2,4}, grid multiplier
 * in {0,1,2,4,8} (0: one workgroup per work item), strided in {0,1},
 * columns per lane group in {1,2,4} (at most
 * 2 where a column takes 64 lanes).  Defaults: 1, 2, 1, 4.  Results do not
 * depend on it. */
thetis_status thetis_batch_configure(thetis_batch *b, int32_t widen, int32_t grid_mult, int32_t strided,
                                     int32_t cols);

/* At most `window` occupied slots run at once (0, the default: all).  The
 * first `window` occupied slots start; when one retires, the waiting slot
 * with the lowest index takes its place at the end of that epoch, on the
 * device.  thetis_batch_run then counts max_epochs per instance, from the
 * epoch it starts, and replays epochs until every slot has retired (at most
 * max_epochs * (ceil(occupied / window) + 1) epochs of launches).  A smaller
 * active set keeps the residuals of the running instances in the device's
 * caches.  Results do not depend on it. */
thetis_status thetis_batch_set_window(thetis_batch *b, int32_t window);

thetis_status thetis_batch_destroy(thetis_batch *b);

/* Message describing the calling thread's last failed call ("" if none). */
const char *thetis_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* THETIS_H */
