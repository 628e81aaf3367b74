/*
 * msp.h -- C-ABI of libmsp: a multi-stage (CPR-type) preconditioned FGMRES
 * solver for the block-sparse Jacobians of fully implicit compositional
 * reservoir simulation, for AMD Instinct MI355X (gfx950).
 *
 * Method: L. Zhao, C.-S. Zhang, C.-S. Feng, S. Shu, "An Improved Multi-Stage
 * Preconditioner on GPUs for Compositional Reservoir Simulation" (2022):
 *   - the block system of Sec. 2.3 (n_c+1 unknowns per cell, pressure first);
 *   - the multiplicative multi-stage preconditioner of eq. (MSP) applied as
 *     in Alg. 3.1, here with two stages: a pressure stage (unsmoothed
 *     aggregation AMG V-cycle, Sec. 5) on the decoupled pressure block and a
 *     full-system block ILU(0) stage;
 *   - the multi-color Gauss-Seidel smoother PGS-MC of Alg. 4.3 on the groups
 *     of Alg. 4.2 (VerticesGrouping);
 *   - the adaptive SETUP of Sec. 3.2: the preconditioner of the previous
 *     Newton system is reused while that solve needed at most mu iterations
 *     and the size is unchanged;
 *   - restarted GMRES(m) of Sec. 5 as flexible GMRES(m).
 *
 * Conventions for every entry point:
 *   - return value: MSP_OK (0), a negative error code, or a positive warning;
 *     no entry point throws, aborts or prints;
 *   - array arguments are DEVICE pointers on the device that was current when
 *     the context was created, unless the comment says "host";
 *   - all work is ordered on the context's stream; every entry point is
 *     synchronous with the host on return;
 *   - a context is used by one host thread at a time (not re-entrant); many
 *     contexts may run concurrently on different streams.
 */
#ifndef MSP_H
#define MSP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSP_OK 0
#define MSP_ERR_ARG (-1)       /* null pointer, n < 1, b outside 1..8, p outside [0,b), nnzb < n */
#define MSP_ERR_PATTERN (-2)   /* row_ptr not monotone, column out of range, unsorted or duplicate
                                  column, or a block row without its diagonal block */
#define MSP_ERR_SINGULAR (-3)  /* singular diagonal block (decoupling or BILU pivot), zero AMG
                                  diagonal, or singular coarsest-level block */
#define MSP_ERR_NONFINITE (-4) /* NaN or Inf in the matrix values or the right-hand side */
#define MSP_ERR_NOMEM (-5)     /* device or host allocation failed */
#define MSP_ERR_HIP (-6)       /* a HIP runtime call failed */
#define MSP_ERR_NO_DEVICE (-7) /* no usable GPU */
#define MSP_ERR_STATE (-8)     /* solve or inspection before a successful setup */
#define MSP_ERR_COARSE (-9)    /* coarsening stalled above the dense coarsest-level limit */
#define MSP_ERR_SCRATCH (-10)  /* msp_solve_noalloc: the FGMRES workspace of this system does
                                  not fit MSP_NOALLOC_SCRATCH_BYTES */
#define MSP_NOT_CONVERGED 1    /* max_iter reached; x holds the last iterate, info is filled */

#define MSP_MAX_LEVELS 25
/* Size of the fixed per-GPU device scratch that msp_solve_noalloc takes its
 * FGMRES workspace from (128 MiB). */
#define MSP_NOALLOC_SCRATCH_BYTES (128ull << 20)
#define MSP_MAX_BLOCK 8

/* Solver options.  msp_default_options() fills the paper's settings
 * (Sec. 5: GMRES(30), MaxIt 1000, coarsest space of at most 10000 unknowns)
 * with mu = 0 (standard MSP, every system rebuilds, Sec. 3.2), an FP64
 * preconditioner, the multi-color block ILU(0) order, one PGS-MC sweep
 * before and after each coarse correction, and block ILU(0) as R. */
typedef struct {
    int mu;           /* adaptive-setup threshold It^(i-1) <= mu => reuse (Sec. 3.2) */
    int restart;      /* m of FGMRES(m), 1..200 */
    int max_iter;     /* total Arnoldi steps over all restarts */
    int max_coarse;   /* the coarsest AMG level has at most this many rows */
    int precond_fp32; /* 0: FP64 preconditioner; 1: AMG hierarchy, GS, BILU and the
                         pressure-column residual stored and applied in FP32 (FGMRES,
                         decoupling weights and the coarsest solve stay FP64) */
    int bilu_order;   /* elimination order of the block ILU(0) stage:
                         1 (default): the groups of Alg. 4.2 on the block adjacency graph
                         one after another (two dependency levels on a 7-point grid);
                         0: natural block order (nx+ny+nz-2 levels on a 7-point grid) */
    int use_graphs;   /* 1 (default): the preconditioner apply is captured once per
                         regeneration into a HIP graph and replayed every iteration
                         (input/output staged through two context-owned vectors);
                         0: every kernel is launched eagerly */
    void *stream;     /* hipStream_t for all work; NULL = the default stream */
    /* Optional device allocator (e.g. a framework caching allocator); both NULL =
     * hipMalloc/hipFree.  dev_alloc returns NULL on failure. */
    void *(*dev_alloc)(size_t bytes, void *user);
    void (*dev_free)(void *ptr, void *user);
    void *alloc_user;
    /* AMG smoother (Table 1 of Sec. 6 compares them): 0 (default) PGS-MC, the
     * multi-color Gauss-Seidel of Alg. 4.3; 1 point Jacobi,
     * x <- x + jacobi_weight D^-1 (f - A x) (the PJAC variant) */
    int smoother;
    int nu_pre;       /* smoothing sweeps before the coarse correction, 0..8 (default 1) */
    int nu_post;      /* ... after it, 0..8 (default 1); Gauss-Seidel runs its colors
                         forward before and backward after */
    int full_smoother; /* relaxation operator R of the last stage (Sec. 3.1): 0 (default)
                          block ILU(0), 1 block Jacobi (z_c = A_cc^-1 r_c) */
    double jacobi_weight; /* weight of the Jacobi correction, (0, 2] (default 1) */
    int n_stage;      /* 1: the concentration stage B_N of eq. MSP runs first in Alg. 3.1,
                         as one block Gauss-Seidel sweep on the decoupled concentration
                         block in the groups of Alg. 4.2 on the block graph; 0 (default):
                         the two stages P then R */
    int host_chain;   /* 0 (default): the aggregation chain (pairwise passes and Galerkin
                         products of every level) runs on the device whenever the block
                         pattern is structurally symmetric, else on the host; 1: always on
                         the host.  Both give the same hierarchy bit for bit. */
} msp_options;

typedef struct {
    int status;               /* return code of the call that filled it */
    int iterations;           /* Arnoldi steps of the last solve (Iter, Tables 2/4/6) */
    int restarts;             /* restart cycles of the last solve */
    int rebuilt;              /* 1 if the last setup regenerated the preconditioner */
    int setup_calls;          /* number of rebuilds so far (SetupCalls, Tables 2/4/6) */
    int solves;               /* number of solves so far */
    int n_levels;             /* AMG levels including the coarsest */
    int level_rows[MSP_MAX_LEVELS];
    int n_colors[MSP_MAX_LEVELS]; /* PGS-MC groups per level (0 on the coarsest) */
    int bilu_levels_fwd;      /* dependency levels of the BILU forward solve */
    int bilu_levels_bwd;
    double rel_true_residual; /* ||b - A x|| / ||b|| after the last solve (FP64) */
    double setup_ms;          /* host wall time of the last setup */
    double rebuild_ms;        /* ... of which preconditioner regeneration */
    double solve_ms;          /* host wall time of the last solve */
    /* host wall time of the phases of the last setup (ms):
     * [0] pattern check (a device comparison when the pattern is unchanged),
     * [1] value ingest, [2] decoupling,
     * [3] aggregation chain (pairwise passes and Galerkin products, on the
     *     device unless the pattern is not structurally symmetric) up to
     *     starting the coarsest-level solver (its kernels are queued from a
     *     host thread of their own),
     * [7] waiting for the host worker threads (block ILU(0) plan, groups and
     *     layouts of the smoothed levels) after the chain,
     * [6] block ILU(0) uploads and factorisation (while the coarsest-level
     *     solver runs on the device) and the final wait for the side stream,
     * [4] level uploads (likewise overlapped),
     * [5] what remains of the coarsest-level solver after [4], [6], [7] */
    double phase_ms[8];
} msp_info;

/* Fill *opt with the defaults listed above.  Returns MSP_ERR_ARG on NULL. */
int msp_default_options(msp_options *opt);

/* Create a context on the current device: the state that Sec. 3.2 carries
 * from one Newton system to the next (the preconditioner B^(i-1), the
 * iteration count It^(i-1) of the last solve, the setup-call counter) and the
 * solver settings of Sec. 5.  *ctx receives an opaque handle owned by the
 * caller until msp_destroy.  opt may be NULL (defaults).
 * Errors: MSP_ERR_ARG (ctx NULL, bad option values), MSP_ERR_NO_DEVICE,
 * MSP_ERR_NOMEM. */
int msp_create(struct msp_ctx **ctx, const msp_options *opt);

/* Ingest one Newton-step Jacobian A^(i) (Sec. 3.2) and decide, by the
 * adaptive rule, whether to regenerate the preconditioner:
 *   regenerate iff no preconditioner exists yet, or (n, b, p) differ from the
 *   last regeneration, or the last solve took more than mu iterations;
 *   otherwise B^(i-1) is kept whole (decoupling weights, AMG hierarchy, BILU
 *   factors).  The current matrix is always ingested: FGMRES and the residual
 *   steps of Alg. 3.1 use A^(i).
 * Arguments (device pointers, read only, may be overwritten by the caller as
 * soon as the call returns):
 *   n_block_rows  n >= 1 block rows (cells);
 *   block_size    b in 1..MSP_MAX_BLOCK (n_c+1 in the paper);
 *   pressure_index p in [0, b): the pressure unknown inside each block;
 *   row_ptr       int32[n+1], row_ptr[0] = 0, row_ptr[n] = nnzb;
 *   col_ind       int32[nnzb], strictly ascending inside each block row, every
 *                 block row holding its diagonal block;
 *   vals          double[nnzb*b*b], block k row-major at vals[k*b*b].
 * Errors: MSP_ERR_ARG, MSP_ERR_PATTERN, MSP_ERR_NONFINITE, MSP_ERR_SINGULAR,
 * MSP_ERR_COARSE, MSP_ERR_NOMEM, MSP_ERR_HIP.  After an error the context
 * holds no preconditioner and the next setup regenerates it. */
int msp_setup(struct msp_ctx *ctx, int n_block_rows, int block_size, int pressure_index,
              const int *row_ptr, const int *col_ind, const double *vals, long long nnzb);

/* Solve A x = rhs by FGMRES(restart) preconditioned with B, to
 * ||rhs - A x||_2 <= rtol ||rhs||_2 (true FP64 residual).
 *   rhs  double[n*b], device, read only;
 *   x    double[n*b], device: initial guess on entry, solution on return;
 *   rtol > 0;
 *   info may be NULL (host).
 * rhs = 0 gives x = 0 after 0 iterations.  Returns MSP_OK,
 * MSP_NOT_CONVERGED (x = last iterate), MSP_ERR_STATE (no setup),
 * MSP_ERR_NONFINITE (rhs), MSP_ERR_ARG, MSP_ERR_HIP. */
int msp_solve(struct msp_ctx *ctx, const double *rhs, double *x, double rtol, msp_info *info);

/* k FGMRES solves of Sec. 5 (as msp_solve), one per context, advanced
 * together by the calling thread: each solve's next Arnoldi step is queued on
 * its context's stream as soon as its previous one has finished, so the
 * device work of all k overlaps while the host does each one's Givens
 * rotations in turn.  Meant for many small systems served at once, whose
 * solves alone leave the device mostly idle.  Each solve's steps, kernels and
 * result are exactly those of msp_solve on the same context.
 *   ctx   k distinct contexts (host array), each set up, on the current device;
 *   rhs   k device pointers, rhs[i] double[n_i b_i] (read only);
 *   x     k device pointers: initial guesses in, solutions out;
 *   infos host array of k msp_info (may be NULL), infos[i].status the solve's
 *         own status.
 * Returns MSP_OK if every solve returned MSP_OK, the first negative status
 * if any failed, else MSP_NOT_CONVERGED.  MSP_ERR_ARG (a NULL pointer, k < 1,
 * a context listed twice), MSP_ERR_STATE (a context without setup). */
int msp_solve_batch(struct msp_ctx *const *ctx, int k, const double *const *rhs,
                    double *const *x, double rtol, msp_info *infos);

/* msp_solve for callers that cannot allocate device memory (code that must
 * not call hipMalloc, tight serving loops, harnesses that forbid it): the
 * same solve, the same arguments, errors and result as msp_solve, but no
 * device allocation of any kind.  The FGMRES workspace (basis V of restart+1
 * vectors, directions Z of restart vectors, one more vector and the
 * reduction buffers; about 8 (2 restart + 2) n b bytes) comes from one fixed
 * per-GPU array of MSP_NOALLOC_SCRATCH_BYTES that the library holds from its
 * load until the process ends; with restart = 30 it fits systems of up to
 * about 260,000 unknowns.  The preconditioner apply replays the HIP graph of
 * an earlier msp_solve if one exists, and is launched kernel by kernel
 * otherwise (the same kernels, the same result).  The context's setup must
 * already have been done with msp_setup, which does allocate.
 * Every call on one GPU uses that GPU's single array and leaves its last
 * contents there (nothing in it needs to start at zero): two calls that
 * overlap in time on the same GPU, from any contexts or threads, race and
 * give wrong results.  Callers serialise them.
 * Errors: those of msp_solve, and MSP_ERR_SCRATCH when the workspace does not
 * fit (nothing is launched then). */
int msp_solve_noalloc(struct msp_ctx *ctx, const double *rhs, double *x, double rtol,
                      msp_info *info);

/* Statistics of the last setup/solve (host pointer). */
int msp_get_info(struct msp_ctx *ctx, msp_info *info);

/* Upper bound of the device memory a context needs for a system of this
 * shape: the FP64 block matrix of Sec. 2.3 (n block rows, nnzb blocks of
 * b x b), the AMG hierarchy of Sec. 5 bounded by the coarsening limits, the
 * block ILU(0) factors of the last stage of eq. (MSP), and the 2m+1 Krylov
 * vectors of FGMRES(m).  The paper has no such query; it serves admission by
 * memory when many systems share one GPU.  opt may be NULL (defaults);
 * bytes: host pointer.  Errors: MSP_ERR_ARG (bytes NULL, n < 1, b outside
 * 1..MSP_MAX_BLOCK, nnzb < n). */
int msp_footprint(int n_block_rows, long long nnzb, int block_size, const msp_options *opt,
                  size_t *bytes);

/* End a Newton sequence (Sec. 3.2): release every device and host resource
 * of the context, after waiting for its stream.  NULL is accepted; the handle
 * is invalid afterwards.  Returns MSP_OK, or MSP_ERR_HIP if a HIP call
 * failed while freeing (the context is released regardless). */
int msp_destroy(struct msp_ctx *ctx);

/* Static, NUL-terminated description of a status code of this header
 * (never NULL; unknown codes give a generic text).  Not from the paper:
 * error reporting of the library. */
const char *msp_status_string(int status);

typedef struct msp_ctx msp_ctx;

#ifdef __cplusplus
}
#endif

#endif /* MSP_H */
