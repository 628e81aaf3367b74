// Launchers of the libmsp HIP kernels (gfx950, wave64).  Every launcher
// enqueues on `st` and returns hipSuccess or the launch error.  Matrices in
// the sliced-ELL layout: slices of 64 rows; slice s = {row0, rows, width, off}
// (off in slot-lanes, a multiple of 64); entry e of slot k of lane l lives at
// val[((off/64) + k) * 64 * E + e * 64 + l], column index at col[off + k*64 + l].
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace msp {

struct SellView {
    const int4 *slices = nullptr;  // {row0, rows, width, off}
    const int *col = nullptr;
    int slice_begin = 0, slice_end = 0;
    // lanes per row of the scalar sweep and residual kernels: 1 (one thread
    // per row) or kRowLanes (a row's entries spread over that many lanes,
    // for short-latency sweeps on the small coarse levels)
    int lanes = 1;
};
constexpr int kRowLanes = 8;

// ---- ingest / layout ----------------------------------------------------
// Copy BSR blocks (row-major, b*b) into the sliced layout: dst entry (q, e) =
// vals[src[q]*b*b + e] (0 where src < 0).  Sets *bad to 1 if a value is not
// finite.  If dst32 != nullptr also writes the FP32 pressure column
// (E = b: entry r = (float)block[r][p]).
hipError_t launch_ingest_bsr(int b, int p, long long slot_lanes, const int *src,
                             const double *vals, double *dst, float *dst32_pcol, int *bad,
                             hipStream_t st);
// Generic block gather into a sliced layout of E = b*b entries, converting
// to float when dst32 != nullptr (RNE) else copying to dst64.
hipError_t launch_gather_blocks(int b, long long slot_lanes, const int *src, const double *blocks,
                                double *dst64, float *dst32, hipStream_t st);
// Scalar level in position space from its natural-order CSR (rp, ci, val)
// and the position maps perm (natural -> position) / iperm: slot k of the
// row at position t (lane t - row0 of its slice) holds the k-th stored
// off-diagonal entry of row iperm[t] in CSR order -- col = perm[j], src = its
// CSR index, value converted to the level's precision (RNE for float) --
// padding slots col = src = -1 and value 0; diag[t] = the row's diagonal
// value (0 if not stored).  Same arrays as the host sliced layout of the
// entries, built where the matrix already is.
hipError_t launch_level_fill(bool fp32, int nslices, const int4 *slices, const int *rp,
                             const int *ci, const double *val, const int *perm, const int *iperm,
                             int *col, int *src, void *vals, void *diag, hipStream_t st);
// Triangular part of the block pattern in a sliced layout: the rows of
// `rows` (level order), slot k of the row at r holding its k-th stored entry
// with pos[j] < pos[i] (lower) or pos[j] > pos[i] (upper) in elimination
// order -- col = pos[j] (the solves index their vectors by elimination
// position), src = its BSR index; padding col = src = -1.
hipError_t launch_tri_fill(int nslices, const int4 *slices, const int *rows, const int *rp,
                           const int *ci, const int *pos, bool lower, int *col, int *src,
                           hipStream_t st);
hipError_t launch_check_finite(const double *x, long long n, int *bad, hipStream_t st);
// Sets *bad to 1 if a[i] != b[i] for some i < n.
hipError_t launch_diff_i32(const int *a, const int *b, long long n, int *bad, hipStream_t st);
hipError_t launch_round_f32(const double *x, float *y, long long n, hipStream_t st);

// ---- decoupling (ABF) ----------------------------------------------------
// omega[c*b..] = row p of D_c^{-1}; ap[k] = sum_r omega_c[r] * A_k[r][p] for
// the blocks of row c.  Fixed evaluation order without contraction.
hipError_t launch_decouple(int b, int p, int n, const int *rp, const int *diag_pos,
                           const double *vals, double *omega, double *ap, int *bad,
                           hipStream_t st);

// ---- block ILU(0) factorisation ----------------------------------------
// One dependency level of the block ILU(0) factorisation.  Row i takes its
// stored lower entries (k, pos[k] < pos[i]) in elimination order, and for
// each: F_ik <- F_ik Dinv_k, then F_ij -= F_ik F_kj for every column j stored
// in both rows with pos[j] > pos[k], in ascending j (a merge of the two
// sorted rows); finally Dinv_i = F_ii^{-1}.  rp/ci: the block pattern (rows
// sorted by column), pos: elimination position of each block row.
struct BiluTasks {
    const int *rows = nullptr;  // block rows of this level
    int nrows = 0;
    const int *rp = nullptr, *ci = nullptr, *pos = nullptr;
    const int *diag_pos = nullptr;
};
hipError_t launch_bilu_factor_level(int b, const BiluTasks &t, double *F, double *Dinv, int *bad,
                                    hipStream_t st);

// ---- SpMV -----------------------------------------------------------------
// y[row] = A x (or sub - A x when sub != nullptr), FP64, natural rows.
hipError_t launch_spmv(int b, const SellView &A, const double *val, const double *x,
                       const double *sub, double *y, hipStream_t st);

// ---- preconditioner pieces (T = float or double) ------------------------
// Input and output vectors of a preconditioner apply, read by its kernels at
// run time, so that one captured graph of the apply serves every pair of
// Krylov vectors.  A kernel given io != nullptr takes io->v (io->z) instead
// of its pointer argument.
struct ApplyIo {
    const double *v;
    double *z;
};
hipError_t launch_set_io(ApplyIo *io, const double *v, double *z, hipStream_t st);
template <typename T>
hipError_t launch_decouple_restrict(int b, int n, const int *iperm0, const double *omega,
                                    const double *v, const ApplyIo *io, T *g, hipStream_t st);
template <typename T>
hipError_t launch_gs_first(const SellView &seg0, int npos, const T *diag, const T *f, T *x,
                           int seg0_begin, int seg0_end, hipStream_t st);
template <typename T>
hipError_t launch_gs_color(const SellView &seg, const T *val, const T *diag, const T *f, T *x,
                           hipStream_t st);
template <typename T>
hipError_t launch_residual(const SellView &all, const T *val, const T *diag, const T *f,
                           const T *x, T *r, hipStream_t st);
template <typename T>
hipError_t launch_restrict(int nc, const int *mem_ptr, const int *mem, const T *r, T *fc,
                           hipStream_t st);
// launch_restrict, then the first color [p0, p1) of the coarse level's forward
// sweep from x = 0 (xc = fc / diag_c there, 0 elsewhere), in one launch.
template <typename T>
hipError_t launch_restrict_first(int nc, const int *mem_ptr, const int *mem, const T *r, T *fc,
                                 int p0, int p1, const T *diag_c, T *xc, hipStream_t st);
template <typename T>
hipError_t launch_prolong(int n, const int *agg_pos, const T *xc, T *x, hipStream_t st);
// The restriction and prolongation maps of a level (n fine positions, nc
// coarse rows) from their coarse-natural-order forms and the coarse level's
// permutation cperm (natural -> position): agg_pos[t] = cperm[natc[t]], and
// the member list of coarse row J (fine positions, mem_nat[mptr_nat[J] ..
// mptr_nat[J+1])) copied to mem from mptr_pos[cperm[J]] on.
hipError_t launch_link(int n, int nc, const int *natc, const int *mptr_nat, const int *mem_nat,
                       const int *cperm, const int *mptr_pos, int *agg_pos, int *mem,
                       hipStream_t st);
// Coarsest-level solve x = A^-1 f = W (Y f) with the factors of
// dense_inverse (row-major, leading dimension ld even, block size P even):
// t = Y f (FP64 work vector of n entries), then x = W t.
template <typename T>
hipError_t launch_coarse_solve(int n, int ld, int P, const double *Y, const double *W,
                               const T *f, double *t, T *x, hipStream_t st);
// weighted point-Jacobi smoothing: x = w D^-1 f (first sweep from zero) and
// x += w D^-1 r; launch_zero clears a level vector (kernel, graph-safe)
template <typename T>
hipError_t launch_jacobi_first(int n, T w, const T *diag, const T *f, T *x, hipStream_t st);
template <typename T>
hipError_t launch_jacobi_update(int n, T w, const T *diag, const T *r, T *x, hipStream_t st);
template <typename T>
hipError_t launch_zero(int n, T *x, hipStream_t st);
// block Jacobi R stage: Dinv_c = A_cc^-1 (FP64, *bad set on a singular block)
// and y_c <- Dinv_c y_c
hipError_t launch_block_inverse(int b, int n, const int *diag_pos, const double *vals,
                                double *Dinv, int *bad, hipStream_t st);
template <typename T>
hipError_t launch_block_jacobi(int b, int n, const T *Dinv, T *y, hipStream_t st);

template <typename T>
hipError_t launch_unpermute(int n, const int *perm0, const T *epos, T *enat, hipStream_t st);
// r_c[k] = v_c[k] - sum_d A_cd[k][p] e_d; pcol64: FP64 A (E = b*b, entry k*b+p);
// pcol32: FP32 pressure columns (E = b).
// rperm (or nullptr): r is written in that block order, r[rperm[c]] (the
// elimination order of the block ILU(0) solves).
template <typename T>
hipError_t launch_pcol_residual(int b, int p, const SellView &A, const double *val64,
                                const float *pcol32, const double *v, const ApplyIo *io,
                                const T *e, const int *rperm, T *r, hipStream_t st);
// The block ILU(0) solves of one dependency level, in place on y (z), a
// block vector in elimination order: rows[r] is the elimination position of
// the r-th row of the level order, the layouts' columns are positions too.
template <typename T>
hipError_t launch_bilu_fwd(int b, const SellView &L, const int *rows, const T *Lval, T *y,
                           hipStream_t st);
template <typename T>
hipError_t launch_bilu_bwd(int b, const SellView &U, const int *rows, const T *Uval,
                           const T *Dval, T *z, hipStream_t st);
// z_c = zz[zperm[c]] (zperm may be nullptr: natural order) + e_c at the
// pressure entry (+ w1_c if w1 != nullptr).
template <typename T>
hipError_t launch_finish(int b, int p, int n, const T *zz, const int *zperm, const T *e,
                         const double *w1, double *z, const ApplyIo *io, hipStream_t st);
// Block vectors between natural and another block order pos (natural c at
// pos[c]): dst[pos[c]] = (T)src[c] when src != nullptr, else
// dst64[c] = (double)srcT[pos[c]].
template <typename T>
hipError_t launch_perm_blocks(int n, int b, const int *pos, const double *src, T *dst,
                              double *dst64, const T *srcT, hipStream_t st);
// N stage (concentration block, block Gauss-Seidel): setup of Dn = rows N of
// D_c^-1 (n x (b-1) x b) and Ann = (D_c^-1 A_cd)[N, N] per stored block
// (nnzb x (b-1)^2, identity on the diagonal blocks), FP64; the right-hand side
// gN = Dn v; one group of the sweep; w1 = Pi_N y.  All no-ops for b = 1.
hipError_t launch_decouple_n(int b, int p, int n, const int *rp, const int *ci,
                             const int *diag_pos, const double *vals, double *Dn, double *Ann,
                             int *bad, hipStream_t st);
template <typename T>
hipError_t launch_n_rhs(int b, int n, const T *Dn, const double *v, T *gN, hipStream_t st);
template <typename T>
hipError_t launch_bgs_group(int b, int ncell, const int *cells, const int *rp, const int *ci,
                            const T *Ann, const T *gN, T *y, hipStream_t st);
template <typename T>
hipError_t launch_expand_n(int b, int p, int n, const T *y, double *w1, hipStream_t st);
template <typename T>
hipError_t launch_to_double(long long n, const T *x, double *y, hipStream_t st);
template <typename T>
hipError_t launch_from_double(long long n, const double *x, T *y, hipStream_t st);

// ---- Krylov (FP64) --------------------------------------------------------
constexpr int kDotBlocks = 1024;
// partial[blk * nv + i] = sum over the block's chunk of V_i . w  (V_i = V + i*ldv)
hipError_t launch_dot_multi(long long N, int nv, const double *V, long long ldv, const double *w,
                            double *partial, hipStream_t st);
// out[i] = sum_blk partial[blk*nv + i] (+ out[i] if accumulate)
hipError_t launch_reduce_partials(int nv, const double *partial, double *out, int accumulate,
                                  hipStream_t st);
// w -= sum_i h[i] V_i
hipError_t launch_axpy_multi(long long N, int nv, const double *V, long long ldv,
                             const double *h, double *w, hipStream_t st);
// One pass of the Gram-Schmidt step over nv <= kFusedGsMax basis vectors,
// each V entry read once: mode 0 the partials of V_i . w (as
// launch_dot_multi), mode 1 w -= sum_i h[i] V_i then the partials of V_i . w,
// mode 2 the same update then the partials of w . w (one value per block).
constexpr int kFusedGsMax = 32;
hipError_t launch_gs_pass(int mode, long long N, int nv, const double *V, long long ldv,
                          const double *h, double *w, double *partial, hipStream_t st);
// y = x / s
hipError_t launch_scale(long long N, const double *x, double s, double *y, hipStream_t st);
// x += sum_i y[i] Z_i
hipError_t launch_update_x(long long N, int k, const double *Z, long long ldz, const double *y,
                           double *x, hipStream_t st);
hipError_t launch_fill(long long N, double v, double *x, hipStream_t st);

// ---- dense coarsest level ---------------------------------------------------
hipError_t launch_dense_scatter(int n, int ld, const int *rp, const int *ci, const double *val,
                                double *M, hipStream_t st);
// C = alpha A B + beta C, row-major FP64 (matrix-core tiles).
hipError_t launch_dgemm(int Mr, int Nc, int Kd, const double *A, int lda, const double *B, int ldb,
                        double *C, int ldc, double alpha, double beta, hipStream_t st);
// Direct solver of the n x n row-major matrix M (leading dimension ld), in
// the form A^-1 = W Y.  A block LU factorisation over kLuBlock-wide blocks,
// A = L U with L unit block-lower triangular, makes no row interchanges
// across blocks; each pivot block is inverted by k_gj_diag, with partial
// pivoting inside the block (*bad is set on a zero pivot).  Then W = U^-1
// (block upper triangular) overwrites M, with zeros below its diagonal
// blocks, and Y = L^-1 (block unit lower triangular: identity diagonal
// blocks, zeros above) fills Y (n x n, leading dimension ld).
//
// With `la` the work runs on three streams that wait for la->ev_start (the
// caller records it on its stream before the call).  la->aux runs the
// critical chain of each step: L's block column, the next pivot block
// (formed apart from the step's Schur update) and its inverse.  la->main
// puts each pivot inverse on the diagonal and runs the Schur updates.
// la->third computes W's block column s and Y's block row s + 1 as soon as
// LU step s has produced them (W by columns, Y by rows in the row-block copy
// of L).  The solver is complete once la->ev_done, recorded on la->main at
// the end, has fired; the caller makes its stream wait for it.  aux is meant
// to own a few compute units of its own, so the latency-bound chain never
// waits for slots behind the GEMMs of the other two.  Without `la`
// everything runs in order on st.
//
// rows_end/cols_end (host arrays, one entry per block step s, or null for
// the full matrix) bound the fill: with rows_end[s] = 1 + the last row whose
// first stored column lies before the end of block s (cols_end likewise by
// columns), L and U have no entries outside rows [0, rows_end[s]) of block
// column s and columns [0, cols_end[s]) of block row s, and the
// factorisation never touches them.  lband must hold
// dense_inverse_lband(n, rows_end) doubles (L by block columns, then by
// block rows) and work dense_inverse_work(n) doubles.
constexpr int kLuBlock = 128;
struct GjLookAhead {
    hipStream_t main, aux, third;
    hipEvent_t ev_start, ev_done, ev_block[2], ev_inv[2], ev_l, ev_y;
};
size_t dense_inverse_work(int n);
size_t dense_inverse_lband(int n, const int *rows_end);
// Depth of the W product of the last block column J (the largest step of
// the sweeps): J P minus the first row of U's band in that column.
int dense_inverse_sweep_k(int n, const int *cols_end);
hipError_t dense_inverse(int n, int ld, double *M, double *Y, double *lband, double *work, int *bad,
                         hipStream_t st, const GjLookAhead *la, const int *rows_end,
                         const int *cols_end);

}  // namespace msp
