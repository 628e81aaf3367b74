/*
 * msp_stages.h -- per-step entry points of libmsp.  Each runs exactly one step
 * of the hot path on the context's current matrix / preconditioner so that it
 * can be checked and timed on its own.  Same conventions as msp.h (device
 * pointers unless "host", synchronous on return, negative = error).
 * All of them return MSP_ERR_STATE before a successful msp_setup.
 */
#ifndef MSP_STAGES_H
#define MSP_STAGES_H

#include "msp.h"

#ifdef __cplusplus
extern "C" {
#endif

/* y = A x, the block SpMV of every FGMRES iteration (Sec. 5), FP64.
 * x, y: double[n*b], must not alias. */
int msp_stage_spmv(msp_ctx *ctx, const double *x, double *y);

/* z = B v, one application of the two-stage preconditioner of eq. (MSP) /
 * Alg. 3.1 (pressure stage then BILU stage, initial w = 0), in the context's
 * preconditioner precision.  v, z: double[n*b], must not alias. */
int msp_stage_precond(msp_ctx *ctx, const double *v, double *z);

/* e = V-cycle(f) on the decoupled pressure matrix (level 0 of the UA-AMG
 * hierarchy, Sec. 5) with the PGS-MC smoother of Alg. 4.3.  f, e: double[n]
 * in natural cell order (converted to the preconditioner precision inside). */
int msp_stage_vcycle(msp_ctx *ctx, const double *f, double *e);

/* One sweep of the configured AMG smoother on level `level`
 * (0 <= level < n_levels-1): multi-color Gauss-Seidel (Alg. 4.3), colors
 * 1..g if forward != 0, else g..1; or one weighted point-Jacobi sweep
 * (forward ignored).  f: double[n_level] read; x: double[n_level] updated in
 * place; natural order of that level. */
int msp_stage_smooth(msp_ctx *ctx, int level, const double *f, double *x, int forward);

/* The R stage of eq. MSP on its own: z = (LU)^{-1} r with the block ILU(0)
 * factors, or z_c = A_cc^{-1} r_c with block Jacobi.  r, z: double[n*b]. */
int msp_stage_bilu(msp_ctx *ctx, const double *r, double *z);

/* Shape of AMG level `level` (host outputs, any may be NULL): rows, stored
 * entries, number of PGS-MC groups (0 on the coarsest), rows of the next
 * level (0 on the coarsest). */
int msp_stage_level_info(msp_ctx *ctx, int level, int *n, long long *nnz, int *ncolors,
                         int *n_next);

/* Copy AMG level `level` to HOST arrays in natural order (any may be NULL):
 * row_ptr int32[n+1], col_ind int32[nnz] (ascending per row), val
 * double[nnz] (FP64 setup values), color int32[n] (1..g; not on the
 * coarsest), agg int32[n] (row of the next level; not on the coarsest). */
int msp_stage_get_level(msp_ctx *ctx, int level, int *row_ptr, int *col_ind, double *val,
                        int *color, int *agg);

/* FP32 copy of level `level`'s values (HOST float[nnz], natural order);
 * MSP_ERR_STATE unless precond_fp32. */
int msp_stage_get_level_f32(msp_ctx *ctx, int level, float *val);

/* Decoupling weights w_c (row p of the inverse diagonal block), HOST
 * double[n*b], cell-major. */
int msp_stage_get_omega(msp_ctx *ctx, double *omega);

/* Block ILU(0) factors in natural BSR order of the pattern used at the last
 * regeneration: F double[nnzb*b*b] (strictly lower blocks L, unit diagonal
 * implied; upper blocks U; diagonal slots hold the factored pivot block) and
 * Dinv double[n*b*b] (inverted pivot blocks); HOST pointers, either may be
 * NULL.  With block Jacobi as R, F is left untouched and Dinv receives the
 * inverted diagonal blocks A_cc^{-1}. */
int msp_stage_get_bilu(msp_ctx *ctx, double *F, double *Dinv);

/* FP32 copies of the BILU factors (HOST, same layout; block Jacobi: Dinv
 * only); precond_fp32 only. */
int msp_stage_get_bilu_f32(msp_ctx *ctx, float *F, float *Dinv);

/* Setup data of the concentration stage (n_stage = 1, b >= 2), FP64, HOST
 * pointers (either may be NULL): Dn double[n*(b-1)*b], rows N (the unknowns
 * other than p, ascending) of D_c^{-1} per cell; Ann double[nnzb*(b-1)^2],
 * (D_c^{-1} A_cd)[N, N] per stored block in BSR order (identity on the
 * diagonal blocks).  MSP_ERR_STATE if the stage is off. */
int msp_stage_get_nstage(msp_ctx *ctx, double *Dn, double *Ann);

/* Stage ids for msp_stage_repeat. */
#define MSP_STAGE_SPMV 0    /* out = A in (double[n*b]) */
#define MSP_STAGE_GS0 1     /* one forward PGS-MC sweep on AMG level 0 (all colors) on the
                               library's level-0 work vectors; in/out unused */
#define MSP_STAGE_PRECOND 2 /* out = B in (double[n*b]) */
#define MSP_STAGE_BILU 3    /* block ILU(0) forward + backward solve on the library's
                               work vector; in/out unused */
#define MSP_STAGE_VCYCLE 4  /* level-0 V-cycle on the library's work vectors; in/out unused */
#define MSP_STAGE_COARSE 5  /* coarsest-level solve on the library's work vectors */
#define MSP_STAGE_TRI_SWEEP 6 /* the largest step of the triangular-inverse sweeps of
                                 the coarsest-level solver, W's last block column: C = -A B
                                 with A (J P) x k and B k x P, P = 128 the block size of
                                 its block LU, J its last block and k the depth of U's band
                                 there (FP64 matrix cores), on scratch operands; in/out
                                 unused */

/* Enqueue `reps` (>= 1) back-to-back executions of one stage on the context's
 * stream with no host synchronisation between them, then synchronise.  Meant
 * for timing with events recorded on the same stream around the call.
 * in/out: device double arrays as listed above (may be NULL where unused).
 * Errors: MSP_ERR_ARG (unknown stage, reps < 1, missing array),
 * MSP_ERR_STATE. */
int msp_stage_repeat(msp_ctx *ctx, int stage, int reps, const double *in, double *out);

/* Per-part timing of msp_solve with HIP events on the context's stream, for
 * measuring the kernels of the FGMRES iteration (Sec. 5) over a real solve
 * rather than in isolation.  on != 0 makes every later msp_solve record four
 * events per Arnoldi step (before the preconditioner apply, before the SpMV
 * w = A z, before the Gram-Schmidt step, after it); each is read after the
 * step's own host synchronisation, so no extra wait is added.  on = 0 stops
 * recording.  Errors: MSP_ERR_ARG (ctx NULL), MSP_ERR_HIP. */
int msp_stage_set_timing(msp_ctx *ctx, int on);

/* Sums over the Arnoldi steps of the last msp_solve with timing on (HOST
 * outputs): ms[0] SpMV, ms[1] preconditioner apply (the captured graph, or
 * the eager launches), ms[2] Gram-Schmidt step (dot products, reductions,
 * updates, norm); calls[i] the number of steps summed.  Zero when timing was
 * off.  Errors: MSP_ERR_ARG (a NULL pointer). */
int msp_stage_get_timing(msp_ctx *ctx, double *ms, int *calls);

#ifdef __cplusplus
}
#endif

#endif /* MSP_STAGES_H */
