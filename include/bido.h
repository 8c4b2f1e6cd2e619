/*
 * bido.h - C ABI of the MI355X bidomain per-step solver.
 *
 * The library advances the semi-implicit heart-torso bidomain scheme of
 * C. Pierre, "Preconditioning the bidomain model with almost linear
 * complexity" (Sec. 3.2, resolution algorithm):
 *
 *   Step 1  Y = [0 ; M_H (gamma V^n - chi (I_ion(V^n, W^n) - I_st^n))]
 *   Step 2  Lambda X = Y with Lambda = [[S_1, Pi^T S_i], [S_i Pi, gamma M_H + S_i]],
 *           X = [U^{n+1}; V^{n+1}], normalised so that (M U, 1) = 0 (Prop. 1)
 *   Step 3  W^{n+1} = W^n + dt g(V^n, W^n)
 *
 * with gamma = chi * c / dt.  Step 2 is solved by preconditioned conjugate
 * gradient with the block-LU preconditioner of Def. 2, the Schur complement
 * replaced by the monodomain matrix K_m = gamma M_H + S_m (Sec. 5.2) and the
 * inner solves P_1 ~ S_1, P_K ~ K_m given by hierarchical Cholesky factors
 * built at accuracy eps (Sec. 5.3).
 *
 * Conventions
 *   - Every pointer named "host" is host memory that the library only reads
 *     during the call and copies; the caller keeps ownership.
 *   - Every pointer named "dev" is device memory on the context's device,
 *     borrowed for the duration of the call and used on the context's
 *     stream; the library never frees it.
 *   - u is indexed by the caller's global vertex numbering (length N);
 *     v and w are indexed in the heart-local order returned by
 *     bido_heart_nodes (heart vertices in ascending global id, length N_H).
 *   - All functions return BIDO_OK (0) or a negative bido_status; the text
 *     of the last error of the calling thread is given by bido_last_error.
 *   - A context is not thread safe; distinct contexts are independent.
 */
#ifndef BIDO_H
#define BIDO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int bido_status;
#define BIDO_OK                 0
#define BIDO_ERR_ARG           -1  /* bad argument, size or layout          */
#define BIDO_ERR_DEVICE        -2  /* HIP runtime error, or no device       */
#define BIDO_ERR_NOT_SPD       -3  /* factorisation failed / CG breakdown   */
#define BIDO_ERR_NOT_CONVERGED -4  /* max_iter reached; best iterate kept   */
#define BIDO_ERR_DT_MISMATCH   -5  /* dt differs from the factored one      */
#define BIDO_ERR_RANGE         -6  /* rhs not in Ran(Lambda) (Prop. 1)      */
#define BIDO_ERR_STATE         -7  /* call not valid in the current state   */

/* region code of heart elements; every other code is a torso organ whose
 * isotropic conductivity is region_sigma[code] (Sec. 2, sigma_T = k(x) Id) */
#define BIDO_REGION_HEART 1

#define BIDO_PREC_FP64  0  /* preconditioner applied in FP64               */
#define BIDO_PREC_MIXED 1  /* preconditioner in FP32 (FP64 outer PCG)      */

#define BIDO_PRECOND_PLAIN   0  /* block-LU / monodomain preconditioner    */
#define BIDO_PRECOND_LEARNED 1  /* P_K from K_m + learned stencil C, FCG   */
#define BIDO_PRECOND_LEARNED_ADDITIVE 2  /* P_K^-1 t + network(t), FCG     */

#define BIDO_LEARN_STENCIL  0   /* train the Schur-complement stencil C     */
#define BIDO_LEARN_ADDITIVE 1   /* train the additive correction network    */

typedef struct bido_ctx bido_ctx;

/* Mesh of the thorax Omega (Sec. 3.1): P1 simplices; heart elements form the
 * sub-mesh of H.  For an isolated heart (Sec. 2.2) every element is heart. */
typedef struct {
    int dim;                /* 2 (triangles) or 3 (tetrahedra)              */
    int64_t n_nodes;        /* N                                            */
    const double* xyz;      /* host, n_nodes x dim, row-major [cm]          */
    int64_t n_elems;
    const int32_t* elems;   /* host, n_elems x (dim+1) vertex ids           */
    const int8_t* region;   /* host, n_elems region codes                   */
} bido_mesh;

/* Tissue description (Sec. 2): sigma_i, sigma_e diagonal in the local fibre
 * frame of each heart element; torso isotropic per region code.           */
typedef struct {
    double sigma_i[3];          /* along fibre, sheet, normal [mS/cm]       */
    double sigma_e[3];
    const double* fibre;        /* host, n_elems x dim x dim, row-major;
                                   column k = k-th frame axis               */
    const double* region_sigma; /* host, n_region_sigma entries             */
    int n_region_sigma;
    const uint8_t* stim_mask;   /* host, n_nodes; 1 = stimulated vertex     */
    double stim_amp;            /* [uA/cm^2]                                */
    double stim_t0, stim_t1;    /* active at step n iff
                                   round(t0/dt) <= n < round(t1/dt)          */
} bido_tissue;

typedef struct {
    double chi;        /* membrane surface-to-volume ratio [1/cm]            */
    double cm;         /* membrane capacitance [uF/cm^2]                      */
    double dt;         /* time step [ms]; gamma = chi*cm/dt                   */
    double eps_h;      /* H-matrix accuracy eps (Sec. 5.3); 0 = exact factor */
    double eta;        /* reserved (kept for the layout; not read): the
                          hierarchical top uses weak admissibility, every
                          off-diagonal block of its bisection tree is low-rank */
    double tol;        /* default relative residual |Lambda X - Y| / |Y|     */
    int leaf;          /* nested-dissection leaf size (default 64)           */
    int max_iter;      /* PCG iteration cap (default 200)                    */
    int precision;     /* BIDO_PREC_*                                         */
    int precond;       /* BIDO_PRECOND_*                                      */
    int ionic;         /* 0 = Mitchell-Schaeffer (one gate per vertex)       */
    int n_threads;     /* host threads for set-up; 0 = library default       */
    int scheme;        /* BIDO_SCHEME_*: time discretisation                 */
    int inner_p1;      /* BIDO_P1_*: the inner solve P_1 ~ S_1 (Sec. 5.3)    */
    int inner_pk;      /* BIDO_PK_*: the inner solve P_K ~ K_m (Sec. 5.3)    */
    int amg_columns;   /* column indices of the multigrid levels, the
                          coupling blocks and the blocked Lambda (all in a
                          banded order when the inner solves are not
                          factored): 0 = 16-bit offsets from a per-row
                          base wherever every row of a matrix spans fewer
                          than 65536 columns (the default), 1 = always
                          32-bit; the result is the same                  */
    int guess_states;  /* initial guess of a step's solve: 0 = X0 = (U^n,
                          V^n); k = 1..16 (default 8) = the projection of
                          the solution onto the span of the states the
                          last k consecutive steps of this context started
                          from (X^n included), orthogonal in the Lambda
                          inner product: X0 = W c, (W^T Lambda W) c = W^T Y.
                          A change of dt restarts the span.  Only the
                          iteration count moves.                        */
} bido_params;

/* Inner solves inside the block-LU preconditioner (Def. 2).  Sec. 5.3 lets
 * P_1 and P_K be any preconditioners of the elliptic block S_1 and of the
 * parabolic block K_m.  CHOLESKY: the multifrontal Cholesky factor in
 * nested-dissection order with the hierarchical top (the default; the
 * paper's choice).  AMG: a symmetric V-cycle of smoothed-aggregation
 * algebraic multigrid (Chebyshev smoothing, dense coarsest solve), set up
 * without any factorisation (linear in the non-zeros), with FP32 level
 * values and vectors in mixed precision (FP64 accumulation, input and
 * output); its block takes the reverse Cuthill-McKee
 * order instead of nested dissection (one order for u and v when the heart
 * is the whole mesh).  CHEBYSHEV (P_K only): Chebyshev-accelerated Jacobi steps on
 * K_m (see bido_set_pk).  A block that is not CHOLESKY is never factored,
 * so the factor-only calls (plans, autotuning, the allocation-free inner
 * solve) refuse it with BIDO_ERR_STATE, and so does a fused batch.       */
#define BIDO_P1_CHOLESKY 0
#define BIDO_P1_AMG      1

/* Time schemes.  EULER: the semi-implicit scheme of Sec. 3.2 (backward
 * Euler on the diffusion, reaction explicit).  CN: Crank-Nicolson on the
 * diffusion terms of the parabolic row with the reaction explicit (the
 * remark on the time discretisation after Prop. 3: only Step 1 and K
 * change): Lambda and K_m take 2 gamma instead of gamma, and Step 1 becomes
 * Y_2 = M_H (2 gamma V^n - 2 chi (I_ion - I_st)) - S_i (V^n + Pi U^n), so a
 * step reads U^n as well as V^n (both from the state arrays).  STRANG:
 * Strang operator splitting (named by the same remark): a reaction
 * half-step of dt/2 (c dV/dt = I_st - I_ion, dw/dt = g, pointwise, Heun's
 * method) from (V^n, w^n), the Crank-Nicolson diffusion step without the
 * ionic term from (U^n, V*), and a second reaction half-step from the
 * diffusion output; second order in dt.  Lambda and K_m as for CN.        */
#define BIDO_SCHEME_EULER 0
#define BIDO_SCHEME_CN 1
#define BIDO_SCHEME_STRANG 2

typedef struct {
    int iterations;        /* PCG iterations of the (last) solve            */
    int converged;         /* 1 if the tolerance was met                    */
    double rel_residual;   /* final |Lambda X - Y| / |Y|                    */
    double ms;             /* wall time of the call on the stream [ms]       */
    int fallbacks;         /* learned-correction fallbacks to the plain one */
    double range_removed;  /* |component of Y_1 along 1| removed (solve)    */
    int64_t total_iterations; /* summed over the steps of bido_run          */
} bido_stats;

typedef struct {
    int64_t n_nodes, n_heart, n_elems;
    int64_t nnz_lambda;          /* stored entries of Lambda                  */
    int64_t bytes_lambda;        /* bytes one Lambda product moves: the blocked
                                    form (one column and the S_1, S_i values
                                    per position, 20 bytes, or 18 with 16-bit
                                    column offsets and a 4-byte base per row)
                                    when the heart is the whole mesh, else the
                                    CSR (12 bytes per stored entry)          */
    int64_t bytes_p1, bytes_pk;  /* bytes of the P_1 / P_K factors as stored
                                    (the active precision); for a multigrid
                                    block, the bytes one V-cycle reads and
                                    writes                                   */
    int64_t dense_bytes_p1, dense_bytes_pk; /* same factors uncompressed      */
    int levels_p1, levels_pk;    /* nested-dissection tree heights (multigrid
                                    levels for a multigrid block)           */
    int64_t lowrank_blocks;      /* low-rank blocks (rank > 0) stored in the
                                    hierarchical tops of P_1 and P_K        */
    double setup_seconds;        /* host set-up time of bido_create           */
    int ground_index;            /* internal index of the grounded u node    */
    int launches_per_sweep_p1;   /* kernel launches of one triangular sweep   */
    int launches_per_sweep_pk;
} bido_info;

/* Last error message of the calling thread ("" if none).                  */
const char* bido_last_error(void);

/* Fill *p with the defaults (chi 200, cm 1, dt 0.1, eps 1e-3, eta 2,
 * tol 1e-10, leaf 64, max_iter 200, FP64, plain, MS, semi-implicit Euler,
 * Cholesky inner solves, 16-bit multigrid columns where they fit,
 * projected initial guesses over 8 states).                              */
void bido_default_params(bido_params* p);

/* Assemble S_1, S_i, S_m and the lumped M, M_H from the mesh (Sec. 3.1,
 * Sec. 5.2), order the unknowns, build the hierarchical Cholesky factors of
 * the grounded S_1 and of K_m (Sec. 5.3) and upload everything to the
 * current HIP device.  `stream` (a hipStream_t, may be NULL for the null
 * stream) is the stream every later call enqueues on.  Returns
 * BIDO_ERR_NOT_SPD if a factorisation meets a non-positive pivot.       */
bido_status bido_create(const bido_mesh* mesh, const bido_tissue* tissue,
                        const bido_params* params, void* stream,
                        bido_ctx** out);

/* Frees the context.  A context still in a batch first leaves it (its own
 * stream and vectors back); that batch then returns BIDO_ERR_STATE from
 * bido_batch_run and must still be destroyed.                            */
void bido_destroy(bido_ctx* ctx);

bido_status bido_get_info(const bido_ctx* ctx, bido_info* info);

/* Heart vertices (global ids, ascending) in the order used for v and w.
 * The array is library-owned host memory valid until bido_destroy.       */
bido_status bido_heart_nodes(const bido_ctx* ctx, const int64_t** ids,
                             int64_t* n_h);

/* One time step (Steps 1-3).  v (dev, N_H), w (dev, N_H gates) and u (dev,
 * N) are updated in place; n is the step index (stimulus window).  The
 * solve starts from X0 = (U^n, V^n) and stops at the context's tol.
 * dt must equal params.dt (gamma is built into K_m), else
 * BIDO_ERR_DT_MISMATCH.  Synchronises the stream once.                  */
bido_status bido_step(bido_ctx* ctx, double* v, double* w, double* u,
                      double dt, int64_t n, bido_stats* st);

/* n_steps consecutive steps starting at index n0, same contract as
 * bido_step; st->total_iterations sums the steps.                        */
bido_status bido_run(bido_ctx* ctx, double* v, double* w, double* u,
                     double dt, int64_t n0, int64_t n_steps, bido_stats* st);

/* Step 2 alone: solve Lambda X = Y (Prop. 1).  rhs (dev, N + N_H) is
 * [Y_1 (global order); Y_2 (heart-local order)]; x (dev, same layout) holds
 * the initial guess on entry and the normalised solution on return.  If the
 * mean of Y_1 exceeds 1e-8 |Y| / sqrt(N) the call returns BIDO_ERR_RANGE
 * and leaves x untouched; otherwise that mean is removed and reported.
 * tol <= 0 selects the context's tol.  On BIDO_ERR_NOT_CONVERGED x holds
 * the last iterate (normalised).                                        */
bido_status bido_solve(bido_ctx* ctx, const double* rhs, double* x,
                       double tol, bido_stats* st);

/* Change the preconditioner precision (BIDO_PREC_*) of an existing context.
 * Mixed precision keeps FP32 copies of the factors and runs the outer
 * solve as flexible CG in FP64.                                         */
bido_status bido_set_precision(bido_ctx* ctx, int precision);

/* Change the time step (steps then pass this dt).  gamma = chi cm / dt
 * (2 gamma for Crank-Nicolson) enters only the v-v diagonal of Lambda and
 * K_m = gamma M_H + S_m (Sec. 3.2, Sec. 5.2); S_1 and its factor P_1 do not
 * depend on dt.  With the factored P_K (BIDO_PK_CHOLESKY) K_m is factored
 * again on the host in its elimination tree and uploaded, with the plan
 * options in use; with the Chebyshev P_K nothing is factored: the device
 * copies of Lambda's values, K_m and its inverse diagonal are replaced and
 * an estimated interval is estimated again (an explicit one is kept).  A
 * multigrid K_m (inner_pk = BIDO_PK_AMG, also while another P_K is active)
 * moves to the new gamma on the device, on the same aggregation and
 * transfer operators: every level's matrix plus (gamma' - gamma) times its
 * Galerkin mass part, new inverse diagonals, smoother copies and smoother
 * intervals (the set-up's Lanczos estimate), and the coarsest inverse by
 * Gauss-Jordan; no host work but the Lanczos scalars.  The
 * stimulus window keeps its times (its step range follows dt).  The
 * learned correction is set up again from scratch (its pairs, weights and
 * stencil were fitted to K_m at the old step; collect and train again) and
 * the preconditioner returns to BIDO_PRECOND_PLAIN.  Captured graphs are
 * rebuilt.  seconds (may be null): wall time of the call.  Errors:
 * BIDO_ERR_ARG for dt <= 0, BIDO_ERR_STATE inside a batch,
 * BIDO_ERR_NOT_SPD if the new K_m cannot be factored (the context keeps
 * its old step), BIDO_ERR_DEVICE for a failed upload (the context then
 * refuses every step with BIDO_ERR_DT_MISMATCH until a later call
 * succeeds).  Synchronises.                                              */
bido_status bido_set_dt(bido_ctx* ctx, double dt, double* seconds);

/* Override tolerance and iteration cap (tol <= 0 / max_iter <= 0 keep the
 * current values).                                                      */
bido_status bido_set_solver(bido_ctx* ctx, double tol, int max_iter);

/* Apply one inner solve on the device: which = 0 for P_1^-1 (grounded S_1,
 * internal u order, N entries), 1 for P_K^-1 (K_m, internal v order, N_H
 * entries).  b and x are device arrays in that internal order (the orders
 * are those of bido_host_index); synchronises the stream.  A check entry
 * point for the triangular sweeps; the solve path does not call it.      */
bido_status bido_inner_solve(bido_ctx* ctx, int which, const double* b, double* x);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the apply of
 * bido_inner_solve, same arguments, kernels and result (bit-identical),
 * with the sweeps' work arrays (intermediate vector, update workspace,
 * partial sums of split tiles, the top's vectors; the Chebyshev P_K's three
 * vectors) taken from a fixed device workspace of 2^23 doubles (64 MiB)
 * that every GPU the library runs on holds until the process ends, instead
 * of the context's buffers.  The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine); the context must exist.  *need
 * (may be null) gets the workspace doubles this apply uses.  Errors:
 * BIDO_ERR_ARG as bido_inner_solve; BIDO_ERR_RANGE when the apply needs more
 * than the fixed workspace (x untouched).  All calls on one GPU share its
 * workspace and it keeps the last call's contents, so calls that overlap on
 * one GPU (other streams, other threads) race; the call synchronises its
 * stream before returning.                                               */
bido_status bido_inner_solve_noalloc(bido_ctx* ctx, int which, const double* b, double* x, int64_t* need);

/* --- alternative P_K (Sec. 5.3: P_1 and P_K are free choices) ----------- *
 * P_K ~ K_m = gamma M_H + S_m (Sec. 5.2) inside P_Lambda (Def. 2) is either
 * the hierarchical Cholesky factor of K_m (BIDO_PK_CHOLESKY, the default)
 * or `steps` steps of the Chebyshev acceleration of the Jacobi iteration on
 * K_m from z_0 = 0 (BIDO_PK_CHEBYSHEV): with D = diag K_m and the interval
 * [lo, hi] holding the spectrum of D^-1 K_m, the error of each eigencomponent
 * lambda is multiplied by T_steps((hi + lo - 2 lambda) / (hi - lo)) /
 * T_steps((hi + lo) / (hi - lo)).  The apply is symmetric positive definite
 * whenever the spectrum lies below lo + hi, so plain CG stays valid; it
 * runs in FP64 in both precisions and costs one product with K_m per step
 * after the first.  lo = hi = 0 estimates the interval on the host
 * (BIDO_PK_LANCZOS_STEPS Lanczos steps on D^-1/2 K_m D^-1/2, the top Ritz
 * value raised by 5 %, clamped to the rigorous bounds min gamma m_i / K_ii
 * and Gershgorin).  The first Chebyshev call uploads K_m (12 bytes per
 * entry) and three N_H work vectors.  Errors: BIDO_ERR_ARG for a bad kind,
 * steps outside [1, BIDO_PK_MAX_STEPS] or an interval other than
 * 0 < lo < hi (or both 0); BIDO_ERR_STATE inside a batch.  Synchronises the
 * stream; captured step graphs are rebuilt.  A fused batch takes the
 * choice of its slices (all must agree on the kind and the step count;
 * each keeps its own interval) and runs the steps as segmented launches
 * over the union.                                                        */
#define BIDO_PK_CHOLESKY  0
#define BIDO_PK_CHEBYSHEV 1
#define BIDO_PK_AMG       2
#define BIDO_PK_MAX_STEPS 64
#define BIDO_PK_LANCZOS_STEPS 20
bido_status bido_set_pk(bido_ctx* ctx, int kind, int steps, double lo, double hi);
/* The current choice: kind, steps and interval (0 for the factor).        */
bido_status bido_get_pk(const bido_ctx* ctx, int* kind, int* steps, double* lo, double* hi);

/* --- recordings of a run (Sec. 6: activation maps and ECG) -------------- *
 * The paper's test cases map the activation time of each point (the time at
 * which the transmembrane potential crosses a fixed level during the
 * depolarisation) and record the potential u at body-surface electrodes at
 * every time step.  bido_record starts (or restarts) such a recording for
 * the following steps of the context (bido_step, bido_run, batches):
 *  - v_act: activation level in the units of v (mV above rest); NaN records
 *    no activation times.  The activation time of heart vertex i is the
 *    first t at which v_i reaches v_act, linearly interpolated between
 *    t_n = n dt and t_n + dt over the step n that crosses it (t_n if v_i
 *    was already at or above v_act before that step); fused into the
 *    write-back of V^{n+1}.
 *  - xyz: host, n_probes x dim probe points (copied); each must lie in the
 *    mesh (BIDO_ERR_ARG otherwise).  After every step the P1 interpolant of
 *    the normalised u at each probe is stored as one row, for the first
 *    max_steps steps (later steps are not recorded).
 * Device memory: 8 N_H + 8 n_probes max_steps bytes plus the weights.
 * Errors: BIDO_ERR_ARG for bad sizes or an infinite v_act, BIDO_ERR_STATE
 * for a context in a batch (start the recording before creating it).     */
bido_status bido_record(bido_ctx* ctx, double v_act, int n_probes, const double* xyz, int64_t max_steps);
/* Copy the recording to host memory: act (N_H, heart-local order; -1 for a
 * vertex not reached; BIDO_ERR_STATE if none are recorded), probes (rows x
 * n_probes, row-major) and the number of rows.  Any pointer may be null.
 * Synchronises the context's stream.                                      */
bido_status bido_record_read(bido_ctx* ctx, double* act, double* probes, int64_t* n_rows);

/* --- learned correction of the monodomain preconditioner (flexible CG) -- *
 * One two-layer message-passing network on the heart vertices (the S_m
 * pattern as graph, hidden width 32, BF16 weights and activations, FP32
 * accumulation), used in one of two ways:
 *  - stencil (BIDO_LEARN_STENCIL / BIDO_PRECOND_LEARNED): fed the static
 *    vertex features only, it gives embeddings h and the symmetric sparse
 *    correction C_ij = dbar (sum_a w3_a h_ia h_ja + b3 [i==j]) on the S_m
 *    pattern; trained so that (K_m + C) z*_k ~ t_k on pairs where
 *    z*_k = V* - V_k is the exact Schur-complement solve of t_k that a
 *    converged plain solve reveals; K_m + C is then factored (Sec. 5.3) and
 *    replaces K_m in P_K (Sec. 5.2).  If K_m + C is not SPD the plain
 *    factor stays.
 *  - additive (BIDO_LEARN_ADDITIVE / BIDO_PRECOND_LEARNED_ADDITIVE): fed
 *    t / rms(t) as an extra channel, its output delta(t) is added to
 *    P_K^-1 t; trained on targets (V* - V_k) - Z2_k.  An apply that is not a
 *    descent direction is redone without it (bido_stats.fallbacks).
 * Pairs come from plain solves (bido_learn_collect).                       */
/* Losses are per sample.  Stencil: |C^ zh - bh|^2 with zh = z* / rms(z*),
 * bh = (t - K_m z*) / (dbar rms(z*)), C^ = C / dbar.  Additive: r^T W r,
 * r the error of the predicted correction in units of the RMS target and
 * W = K_m scaled to unit mean diagonal.                                   */
typedef struct {
    int samples, train_samples, epochs;
    double loss_zero;       /* mean loss of the zero correction (training)   */
    double loss_zero_val;   /* the same on the validation samples            */
    double loss_first;      /* mean training loss before training            */
    double loss_last;       /* mean training loss after training             */
    double loss_val;        /* mean validation loss after training           */
    double seconds;
    int spd;                /* stencil: K_m + C factored (1) or not (0)       */
    double refactor_seconds;
    int best_epoch;         /* stencil: the epoch whose weights are kept (the
                               lowest validation loss, or training loss when
                               n_val = 0; 0: the weights before training)   */
} bido_train_stats;

/* BIDO_PRECOND_* for later solves; BIDO_PRECOND_LEARNED needs a trained
 * stencil (BIDO_ERR_STATE otherwise).                                      */
bido_status bido_set_precond(bido_ctx* ctx, int precond);

/* Forget the states of the previous steps that span the projected initial
 * guess (bido_params.guess_states): the next step starts a new span from
 * its own state.  For callers that restart a run from another state, and
 * for comparing runs from equal starting points.  Enqueues nothing.       */
bido_status bido_reset_guess(bido_ctx* ctx);

/* Run n_steps plain steps (as bido_run) recording training pairs, up to
 * max_samples in total (device memory: 16 N_H + 16 bytes per sample).            */
bido_status bido_learn_collect(bido_ctx* ctx, double* v, double* w, double* u, double dt,
                               int64_t n0, int64_t n_steps, int max_samples, bido_stats* st);
bido_status bido_learn_samples(const bido_ctx* ctx, int* n_samples);

/* Train for `kind` (BIDO_LEARN_*): Adam on the FP32 master weights over the
 * first (samples - n_val) pairs, mini-batches of `batch`, shuffled by
 * `seed`; the last n_val pairs are held out for the validation loss.  The
 * stencil keeps the weights of the epoch with the lowest validation loss
 * (training loss when n_val = 0), the weights before training included.  */
bido_status bido_learn_train(bido_ctx* ctx, int kind, int epochs, int batch, float lr, uint64_t seed,
                             int n_val, bido_train_stats* st);

/* FP32 master weights (3169 floats, layout W1s W1n b1 W2s W2n b2 w3 b3):
 * dir 0 copies them to buf, dir 1 loads buf (and resets Adam and the output
 * unit to 1).                                                             */
bido_status bido_weights_io(bido_ctx* ctx, float* buf, int n, int dir);

/* Check entry points (not used by the solve path).  gnn_eval: out = delta(t)
 * for a device vector t in heart-local order.  gnn_loss_grad: for device
 * inputs t/rms(t) and target/rms(t) (FP32, heart-local; rms(t) =
 * |t|_2 / sqrt(N_H)) the loss r^T W r (r = o - y, W as above) and its
 * gradient (host outputs), with the output unit 1.                        */
bido_status bido_gnn_eval(bido_ctx* ctx, const double* t, double* out);
bido_status bido_gnn_loss_grad(bido_ctx* ctx, const float* that, const float* y, double* loss,
                               float* grad);
/* stencil_check: with the current weights, for device FP32 vectors zh, bh in
 * heart-local order: r = C^ zh - bh (device FP32, heart-local; may be NULL),
 * the loss |r|^2 and its gradient (host; grad may be NULL).               */
bido_status bido_stencil_check(bido_ctx* ctx, const float* zh, const float* bh, float* r, double* loss,
                               float* grad);

/* Execution plan of an inner solve's triangular sweeps (the device layout
 * of the Cholesky factors of Sec. 5.3; results do not depend on it beyond
 * rounding).  The nodes of the elimination tree below a subtree cut height
 * are swept by one workgroup per subtree, the levels above it by one launch
 * per tree height (forward items of 64 rows x fwd_cols columns, backward
 * items of up to 64 columns x a row range, split tiles summed by a combine
 * launch), and the nodes from the top cut up by one product with the
 * (dense or hierarchical) inverse of their Schur complement.  Fields <= 0
 * (top_h, sub_h, bwd_wide, level_items < 0) take the defaults.           */
typedef struct {
    int top_h;          /* first tree height of the top; -1: cost model;
                           tree height + 1: no top                        */
    int fwd_cols;       /* columns per forward level item (0: 128)        */
    int bwd_rows;       /* rows per backward level item (0: rule below)   */
    int bwd_wide;       /* 1024-thread backward items over whole column
                           tiles (1), 256-thread items over row ranges (0);
                           -1: 1                                          */
    int level_items;    /* without bwd_rows, a level of tall tiles is split
                           into row ranges until it has about this many
                           wide items (-1: 512; 0 keeps tiles whole)      */
    int sub_h;          /* cap of the subtree cut heights (-1: none)      */
    int sub_want;       /* subtrees wanted per tree (0: 256)              */
    int sub_total;      /* subtrees shared over a fused batch's forest
                           (0: 512 there, sub_want per tree elsewhere)    */
    int bwd_group_max;  /* backward subtree heights with at most this many
                           nodes use wave groups (0: 2 in 2D, 4 in 3D)    */
    int spmv_group;     /* lanes per row of the sparse products of the
                           context: 4, 8, 16 or 32 (0: 4 in 2D, 16 in 3D) */
} bido_plan;
void bido_default_plan(bido_plan* plan);
/* Rebuild the device plan of factor `which` (BIDO_FACTOR_P1 = 0,
 * BIDO_FACTOR_PK = 1) with these options, and set the context's spmv_group
 * (when non-zero).  Synchronises; captured graphs are rebuilt.  Errors:
 * BIDO_ERR_ARG (bad which or spmv_group; the old plan is kept),
 * BIDO_ERR_STATE for a context in a batch.  bido_get_plan reads the options
 * of the plan in use (defaults resolved as built).                        */
bido_status bido_set_plan(bido_ctx* ctx, int which, const bido_plan* plan);
bido_status bido_get_plan(const bido_ctx* ctx, int which, bido_plan* plan);

/* Autotuning of the inner-solve plans: for P_1 and P_K, candidate plans
 * (the first height of the top one or two levels either side of the cost
 * model's choice, then forward column chunks of 64/128/256 and backward row
 * ranges of 256/1024 or the default) are built, their triangular solves are
 * timed on the device (`reps` back-to-back solves, <= 0: 10) and the fastest
 * plan is kept.  Results do not change beyond rounding.  Synchronises the
 * stream; not for a context in a batch (BIDO_ERR_STATE).                  */
typedef struct {
    int candidates;          /* plans built and timed                         */
    double seconds;          /* host time of the whole tuning                 */
    double us_before[2];     /* P_1, P_K solve time with the initial plans    */
    double us_after[2];      /* ... with the chosen plans                     */
    int top_h[2];            /* chosen first height of the top                */
    int fwd_cols[2];         /* chosen forward column chunk                   */
    int bwd_rows[2];         /* chosen backward row range (0: default)        */
} bido_tune_report;
bido_status bido_autotune(bido_ctx* ctx, int reps, bido_tune_report* report);

/* HIP graphs: bido_step / bido_run / bido_batch_run can replay one captured
 * graph per PCG iteration (preconditioner apply, direction update, SpMV,
 * PCG update, copy of the scalars) instead of launching its kernels one by
 * one; graphs are captured on first use and again after a change of
 * precision or preconditioner.  on = 1: always, 0: never, -1 (default):
 * only while the context belongs to a batch (where the many small launches
 * of its slices make them pay; a single large context runs faster eager).
 * Steps run on a stream of the context ordered after and before the
 * caller's stream.  Profiling, sample collection and the additive learned
 * mode run eagerly.  Results are the same bit for bit either way.        */
bido_status bido_set_graphs(bido_ctx* ctx, int on);

/* --- batched execution of independent slices ---------------------------- *
 * A batch runs bido_run on many contexts at once (Sec. 3.2 for each slice,
 * each with its own PCG scalars and stopping test).  The contexts keep their
 * settings (precision, preconditioner); while they belong to the batch their
 * launches go to the batch's own streams (n_streams of them, <= 0: up to 4;
 * default priority), packed by size, and the host waits once per PCG phase
 * for all slices.  The contexts must live on the current device, may not be
 * listed twice or belong to another batch (BIDO_ERR_STATE), and must not be
 * used on their own until bido_batch_destroy gives them back.  `stream` is
 * the caller's stream (a hipStream_t): bido_batch_run waits for it and makes it wait for the
 * batch.  The additive learned mode is refused (BIDO_ERR_STATE).          */
typedef struct bido_batch bido_batch;
bido_status bido_batch_create(bido_ctx* const* ctxs, int n_ctx, int n_streams, void* stream,
                              bido_batch** out);
/* v[i], w[i], u[i]: device state of slice i as for bido_run.  per_ctx (host
 * array of n_ctx, may be NULL): the last step's statistics of each slice with
 * its summed iterations; total: the largest per-step iteration count
 * (iterations), the sum over slices and steps (total_iterations), the worst
 * final residual, wall time.  Returns the first error of any slice.       */
bido_status bido_batch_run(bido_batch* b, double* const* v, double* const* w, double* const* u, double dt,
                           int64_t n0, int64_t n_steps, bido_stats* per_ctx, bido_stats* total);
void bido_batch_destroy(bido_batch* b);

/* Fused batch (same run and destroy calls).  The slices' vectors, Lambda,
 * S_i Pi, Pi^T S_i and their P1 and PK factors are laid side by side in one
 * union (slice s at the sum of the earlier slices' N + N_H, u rows first),
 * so that each phase of the PCG iteration of Sec. 3.2 is one launch for all
 * slices: segmented vector kernels keep alpha, beta and r.z per slice, the
 * stopping test is per slice and runs on the device at the end of every
 * iteration (the next iteration's kernels read its flags), so the host
 * waits once per chunk of iterations (one less than the previous step's
 * count, then one at a time), not once per iteration; a slice that has met
 * the test is frozen (alpha = beta = 0) while the others iterate; the inner
 * solves sweep the forest of
 * all slices' elimination trees level by level, each tree with the top cut
 * of its own plan.  Steps 1 and 3 and the normalisation stay per slice.
 * Each slice runs the plain preconditioner or the learned stencil
 * (BIDO_PRECOND_LEARNED with a trained stencil and the factored P_K: its
 * factor of K_m + C takes K_m's place in the slice's tree; the union then
 * takes the flexible direction update, as the slice alone does); the
 * additive network form is refused.  Needs one precision, one P_K choice
 * (bido_set_pk) and factored P_1 and K_m for all slices, and refuses
 * contexts already in a batch (BIDO_ERR_STATE).  While in the batch a
 * slice's preconditioner, precision and learned state are fixed
 * (bido_set_precond, bido_learn_collect and bido_learn_train return
 * BIDO_ERR_STATE).  Set-up merges the host factors and uploads a second
 * copy of them (the contexts keep theirs); results agree with the slices
 * run alone up to rounding order.  The contexts' U/V work vectors alias
 * the union while in the batch.                                          */
bido_status bido_batch_create_fused(bido_ctx* const* ctxs, int n_ctx, void* stream, bido_batch** out);
/* Fused batch only: replay captured graphs of the PCG iterations (on != 0,
 * the default) or launch every kernel eagerly (BIDO_ERR_STATE for a batch
 * of streams, whose contexts follow bido_set_graphs).                    */
bido_status bido_batch_set_graphs(bido_batch* b, int on);
/* fused: 1 for a fused batch; n_union: its union length (sum of N + N_H);
 * setup_seconds: host and upload time of bido_batch_create_fused.  Any
 * output may be NULL.                                                    */
bido_status bido_batch_info(const bido_batch* b, int* fused, int64_t* n_union, double* setup_seconds);
/* Fused batch counters since its creation: steps, PCG iterations launched
 * (over all steps; the union iterates until its last slice stops), host
 * waits inside the iterations, kernel launches of the captured iteration
 * graphs (0 when graphs are off).  Any output may be NULL; BIDO_ERR_STATE
 * for a batch of streams.                                                */
bido_status bido_batch_counters(const bido_batch* b, int64_t* steps, int64_t* iterations, int64_t* host_waits,
                                int64_t* kernels);

/* Per-kernel profile: launches, summed event-timed duration [ms] and the
 * algorithmic bytes those launches must move (inputs read once, outputs
 * written once), aggregated by kernel class.                            */
typedef struct {
    char name[24];
    int64_t launches;
    double ms;
    double bytes;
} bido_kprof;

/* enable != 0 brackets every later launch on the context's stream with a
 * pair of HIP events (adds a little launch overhead); resets the records. */
bido_status bido_profile(bido_ctx* ctx, int enable);

/* Synchronise, aggregate the records since the last read or enable into
 * out[0..cap) (one entry per kernel class seen), set *n to the number of
 * classes and clear the records.                                         */
bido_status bido_profile_read(bido_ctx* ctx, bido_kprof* out, int cap, int* n);

/* The same for a fused batch (BIDO_ERR_STATE for a batch on streams, whose
 * contexts are profiled one by one): the union's triangular sweeps, tops
 * and Chebyshev steps are bracketed, the segmented vector kernels are not;
 * while profiling the batch launches eagerly instead of replaying graphs. */
bido_status bido_batch_profile(bido_batch* b, int enable);
bido_status bido_batch_profile_read(bido_batch* b, bido_kprof* out, int cap, int* n);

#ifdef __cplusplus
}
#endif
#endif /* BIDO_H */
