/*
 * bido_host.h - host-only inspection entry points of libbido.
 *
 * These run the host set-up of bido_create (assembly of Sec. 3.1, the
 * nested-dissection orderings, the hierarchical Cholesky factors of the
 * grounded S_1 and of K_m, Sec. 5.3) without touching a GPU, and expose
 * its results for checks.  They are not part of the solve path: bido_step,
 * bido_run and bido_solve never call them.
 *
 * Ownership: every returned pointer is owned by the bido_host object and
 * stays valid until bido_host_free.  Errors are reported as in bido.h.
 */
#ifndef BIDO_HOST_H
#define BIDO_HOST_H

#include "bido.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bido_host bido_host;

#define BIDO_MAT_S1     0  /* S_1, caller's global numbering, N x N          */
#define BIDO_MAT_SI     1  /* S_i, heart-local numbering, N_H x N_H           */
#define BIDO_MAT_SM     2  /* S_m, heart-local numbering                      */
#define BIDO_MAT_LAMBDA 3  /* Lambda in the internal order (u then v)         */
#define BIDO_MAT_GNN_AGG 4 /* neighbour weights of the learned correction,
                              heart-local: |S_m,ij| / sum_k!=i |S_m,ik|, j != i */
#define BIDO_MAT_KM     5  /* K_m = gamma M_H + S_m, internal v order         */

#define BIDO_VEC_M      0  /* lumped M, global numbering                      */
#define BIDO_VEC_MH     1  /* lumped M_H, heart-local numbering               */
#define BIDO_VEC_GNN_STATIC 2 /* static vertex features of the learned
                                 correction, N_H x 15 row-major, heart-local  */

#define BIDO_IDX_UPOS   0  /* global id -> internal u index                    */
#define BIDO_IDX_VPOS   1  /* heart-local index -> internal v index            */
#define BIDO_IDX_HEART  2  /* heart-local index -> global id                   */

#define BIDO_FACTOR_P1  0  /* factor of the grounded S_1 (internal u order)   */
#define BIDO_FACTOR_PK  1  /* factor of K_m (internal v order)                */

/* Last error message of the host entry points on the calling thread.    */
const char* bido_host_last_error(void);

bido_status bido_host_setup(const bido_mesh* mesh, const bido_tissue* tissue,
                            const bido_params* params, bido_host** out);
void bido_host_free(bido_host* h);

/* CSR view: row pointers (n+1, int64), columns (int32), values (double). */
bido_status bido_host_csr(const bido_host* h, int which, int64_t* n, int64_t* nnz,
                          const int64_t** ptr, const int32_t** col, const double** val);
bido_status bido_host_vec(const bido_host* h, int which, int64_t* n, const double** data);

/* Spectral interval of the Chebyshev P_K (bido_set_pk with lo = hi = 0):
 * out[0..6) = the interval used (lo, hi), the extreme Ritz values of
 * `lanczos_steps` Lanczos steps on D^-1/2 K_m D^-1/2, and the rigorous
 * bounds (min gamma m_i / K_ii, Gershgorin).                              */
bido_status bido_host_pk_interval(const bido_host* h, int lanczos_steps, double* out);

/* Host emulation of the Chebyshev P_K apply (the device recurrence and its
 * coefficients, in FP64 on the CPU; a check hook): x = P_K^-1 b for `steps`
 * steps on [lo, hi], b and x in the internal v order (N_H entries).       */
bido_status bido_host_pk_emulate(const bido_host* h, int steps, double lo, double hi, const double* b, double* x);

/* Probe location of bido_record: for each of n points (host, n x dim) the
 * dim + 1 vertex ids (caller's numbering) of an element holding it and the
 * barycentric weights there (ids, wts: n x (dim + 1)).  BIDO_ERR_ARG if a
 * point lies outside the mesh.                                           */
bido_status bido_host_locate(const bido_host* h, int n, const double* pts, int64_t* ids, double* wts);

/* The host part of bido_set_dt: gamma, the v-v diagonal of Lambda, K_m and
 * (refactor != 0) the factor of K_m at the new dt.                        */
bido_status bido_host_set_dt(bido_host* h, double dt, int refactor);
bido_status bido_host_index(const bido_host* h, int which, int64_t* n, const int64_t** data);

/* Sizes of a factor: panel entries (the lower triangles of L_tt^-1 and the
 * blocks L_Bt L_tt^-1 of every tree node, held exactly), tree height,
 * largest separator.  The hierarchical compression at eps_h applies to the
 * top of the execution plan (bido_host_factor_top).                       */
bido_status bido_host_factor_stats(const bido_host* h, int which, int64_t* entries, int* height,
                                   int* max_sep);

/* Per tree node (post-order): nI, nB, height, depth, parent, as 5 int32
 * per node into out[0..5*cap).  *n_nodes gets the count.                 */
bido_status bido_host_factor_nodes(const bido_host* h, int which, int64_t* n_nodes, int32_t* out,
                                   int64_t cap);

/* Apply the factor on the host: x = (L L^T)^-1 b in the factor's internal
 * order (for P_1 the grounded entry of b is ignored and x there is 0).     */
bido_status bido_host_factor_apply(const bido_host* h, int which, const double* b, double* x);

/* Run the device execution plan of a factor (the work items the GPU sweep
 * kernels process, in launch order) through a sequential CPU emulation of
 * those kernels with bounds-checked accesses; x as bido_host_factor_apply. */
bido_status bido_host_factor_emulate(const bido_host* h, int which, const double* b, double* x);

/* Shape of that plan: subtree cut height, subtrees, level launches per
 * sweep above the cut, forward and backward work items, and the backward
 * column tiles split over several row-range items (summed by a combine
 * launch).                                                               */
bido_status bido_host_factor_plan(const bido_host* h, int which, int* hc, int* n_sub, int* n_levels,
                                  int64_t* n_fwd_items, int64_t* n_bwd_items, int64_t* n_bwd_split);

/* Lambda in blocked form (Sec. 3.2 system with Pi = I: the heart is the
 * whole mesh and u and v share one internal order).  Row k of the u rows
 * and row k of the v rows share one position list: columns col[ptr[k] ..
 * ptr[k+1]) with the value pairs val[2q] = S_1[k, c], val[2q+1] =
 * S_i[k, c], and gm[k] = gamma m_k, so that
 *   (Lambda x)_u[k] = sum S_1 x_u[c] + S_i x_v[c],
 *   (Lambda x)_v[k] = sum S_i (x_u[c] + x_v[c]) + gm[k] x_v[k].
 * The device's Lambda product reads this form when it exists.  Arrays are
 * owned by the set-up.  BIDO_ERR_STATE when there is none (torso rows, or
 * the two orders differ).                                                */
bido_status bido_host_lambda_blocked(const bido_host* h, int64_t* n, int64_t* npos, const int64_t** ptr,
                                     const int32_t** col, const double** val, const double** gm);

/* Multigrid hierarchy of a block set up with inner_p1 / inner_pk = AMG
 * (which = BIDO_FACTOR_P1 / BIDO_FACTOR_PK; BIDO_ERR_STATE if it has none).
 * info: levels, size of the coarsest level, operator complexity (sum of the
 * levels' non-zeros over the fine matrix's), host seconds of its set-up,
 * Chebyshev steps per smoothing on the finest level.  level: CSR view of
 * level `level`'s matrix (what = 0) or prolongation (what = 1; not on the
 * coarsest level), owned by the hierarchy.  smoother: D^-1 of the level (0
 * at the grounded vertex), the interval [lo, hi] of the smoother polynomial
 * and the level's Chebyshev steps per smoothing (1 on the coarser levels by
 * default: the damped Jacobi sweep).  apply: one host V-cycle x = B b (a
 * check hook; internal order).                                           */
bido_status bido_host_amg_info(const bido_host* h, int which, int* levels, int64_t* n_coarse,
                               double* op_complexity, double* seconds, int* smooth_steps);
bido_status bido_host_amg_level(const bido_host* h, int which, int level, int what, int64_t* n, int64_t* nnz,
                                const int64_t** ptr, const int32_t** col, const double** val);
bido_status bido_host_amg_smoother(const bido_host* h, int which, int level, const double** dinv, double* lo,
                                   double* hi, int* steps);
bido_status bido_host_amg_apply(const bido_host* h, int which, const double* b, double* x);

/* Plan options (bido_plan, bido.h) of the later bido_host_factor_emulate,
 * _plan and _top queries of factor `which` (default: bido_default_plan).  */
bido_status bido_host_set_plan(bido_host* h, int which, const bido_plan* plan);

/* Test hook for batches of independent slices: a host object whose factors
 * are the forests of the slices' factors (the factors of the block-diagonal
 * union), slice s at offset O_s = sum_{t<s} (N_t + N_H,t): P_1 on
 * [O_s, O_s + N_s), P_K on [O_s + N_s, O_s + N_s + N_H,s), vectors of
 * sum_s (N_s + N_H,s) entries.  Only the bido_host_factor_* entry points
 * apply to it; free it with bido_host_free.  A tree whose slice's own plan
 * already holds a hierarchical top of the same cut (any earlier
 * bido_host_factor_* call on that slice with eps_h > 0) takes it over
 * instead of inverting again, so the slices' objects must outlive this one.*/
bido_status bido_host_merge(const bido_host* const* hs, int n, bido_host** out);

/* Dense top of that plan: the tree nodes of height >= top_h are solved as
 * one product with the explicit inverse of their Schur complement (the
 * Cholesky factor of Sec. 5.3 restricted to the top separators, inverted
 * once at set-up); n_top vertices, `seconds` of host time to invert.
 * top_h = tree height + 1 means no dense top.  The cut comes from a cost
 * model; the plan option top_h (bido_host_set_plan) forces it (raised as
 * far as the bound of the top size requires).  With eps_h > 0 the inverse is held in
 * hierarchical low-rank form (the top vertices in geometric bisection
 * order, off-diagonal blocks truncated by rank-revealing QR at relative
 * accuracy eps_h, Sec. 5.3): stored_entries counts its values, max_rank its
 * largest block rank (-1 when dense), n_lowrank its blocks of rank > 0. */
bido_status bido_host_factor_top(const bido_host* h, int which, int* top_h, int64_t* n_top, double* seconds,
                                 int64_t* stored_entries, int* max_rank, int64_t* n_lowrank);

#ifdef __cplusplus
}
#endif
#endif /* BIDO_HOST_H */
