// HIP kernels of libmsp for gfx950 (CDNA4, wave64).
//
// Layout conventions are in msp_kernels.h.  Sparse kernels map one thread to
// one row of a 64-row slice, so every value load of a wave is a contiguous,
// 512-byte (FP64) or 256-byte (FP32) access; column indices are read the same
// way.  Reductions use a fixed tree, so results are identical run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "msp_kernels.h"

namespace msp {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ bool finite_d(double v) { return __builtin_isfinite(v); }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Work-groups are dispatched to the 8 XCDs round-robin (work-group b to XCD
// b mod 8), and each XCD has its own L2.  xcd_block maps the dispatch order
// to a logical index so that every XCD works on one contiguous range of
// logical work-groups: neighbouring slices, which gather the same x entries,
// then share an L2.  It is a bijection on [0, nb): XCD x receives
// q + (x < r) work-groups (q = nb / 8, r = nb mod 8), at logical indices
// x q + min(x, r) onwards.
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

inline unsigned blocks_for(long long work, int per_block = kThreads)
{
    long long b = (work + per_block - 1) / per_block;
    return (unsigned)(b < 1 ? 1 : b);
}

inline unsigned slice_blocks(const SellView &v)
{
    int ns = v.slice_end - v.slice_begin;
    return ns > 0 ? (unsigned)((ns + 3) / 4) : 0u;
}

// ---------------------------------------------------------------------------
// ingest / layout
// ---------------------------------------------------------------------------
template <int B>
__global__ __launch_bounds__(kThreads) void k_ingest(int p, long long slot_lanes,
                                                     const int *__restrict__ src,
                                                     const double *__restrict__ vals,
                                                     double *__restrict__ dst,
                                                     float *__restrict__ dst32, int *bad)
{
    constexpr int E = B * B;
    long long q = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (q >= slot_lanes) return;
    const int s = src[q];
    const long long sb = q >> 6;
    const int lane = (int)(q & 63);
    double *d = dst + sb * 64 * E + lane;
    bool fin = true;
    double v[E];
    if (s >= 0) {
        const double *blk = vals + (long long)s * E;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            v[e] = blk[e];
            fin = fin && finite_d(v[e]);
        }
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = 0.0;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) d[(long long)e * 64] = v[e];
    if (dst32) {
        float *d32 = dst32 + sb * 64 * B + lane;
#pragma unroll
        for (int r = 0; r < B; ++r) {
            double a = 0.0;
#pragma unroll
            for (int c = 0; c < B; ++c)
                if (c == p) a = v[r * B + c];
            d32[r * 64] = (float)a;
        }
    }
    if (!fin) atomicOr(bad, 1);
}

template <int B>
__global__ __launch_bounds__(kThreads) void k_gather_blocks(long long slot_lanes,
                                                            const int *__restrict__ src,
                                                            const double *__restrict__ blocks,
                                                            double *__restrict__ dst64,
                                                            float *__restrict__ dst32)
{
    constexpr int E = B * B;
    long long q = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (q >= slot_lanes) return;
    const int s = src[q];
    const long long base = (q >> 6) * 64 * E + (q & 63);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        double v = s >= 0 ? blocks[(long long)s * E + e] : 0.0;
        if (dst32)
            dst32[base + (long long)e * 64] = (float)v;
        else
            dst64[base + (long long)e * 64] = v;
    }
}

// one thread per (slice, lane); lanes past the slice's rows pad every slot
template <typename T>
__global__ __launch_bounds__(kThreads) void k_level_fill(int nslices,
                                                        const int4 *__restrict__ slices,
                                                        const int *__restrict__ rp,
                                                        const int *__restrict__ ci,
                                                        const double *__restrict__ val,
                                                        const int *__restrict__ perm,
                                                        const int *__restrict__ iperm,
                                                        int *__restrict__ col,
                                                        int *__restrict__ src,
                                                        T *__restrict__ vals,
                                                        T *__restrict__ diag)
{
    const long long g = (long long)blockIdx.x * kThreads + threadIdx.x;
    const int s = (int)(g >> 6), lane = (int)(g & 63);
    if (s >= nslices) return;
    const int4 d = slices[s];  // row0, rows, width, slot-lane offset
    int m = 0;
    if (lane < d.y) {
        const int t = d.x + lane;
        const int i = iperm[t];
        T dv = 0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            const int j = ci[k];
            if (j == i) {
                dv = (T)val[k];
            } else {
                const long long q = (long long)d.w + (long long)m * 64 + lane;
                col[q] = perm[j];
                src[q] = k;
                vals[q] = (T)val[k];
                ++m;
            }
        }
        diag[t] = dv;
    }
    for (; m < d.z; ++m) {
        const long long q = (long long)d.w + (long long)m * 64 + lane;
        col[q] = -1;
        src[q] = -1;
        vals[q] = 0;
    }
}

__global__ __launch_bounds__(kThreads) void k_diff_i32(const int *__restrict__ a,
                                                       const int *__restrict__ b, long long n,
                                                       int *bad)
{
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i < n && a[i] != b[i]) atomicOr(bad, 1);
}

__global__ __launch_bounds__(kThreads) void k_check_finite(const double *__restrict__ x,
                                                           long long n, int *bad)
{
    long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i < n && !finite_d(x[i])) atomicOr(bad, 1);
}

__global__ __launch_bounds__(kThreads) void k_round_f32(const double *__restrict__ x,
                                                        float *__restrict__ y, long long n)
{
    long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}

// ---------------------------------------------------------------------------
// decoupling: solve D_c^T w = e_p by Gaussian elimination with partial
// pivoting (first largest pivot), then A_P[c,d] = sum_r w[r] A_cd[r][p].
// The evaluation order is fixed and contraction is off, so the pressure
// matrix rounds exactly as the same formula evaluated sequentially.
// ---------------------------------------------------------------------------
template <int B>
__global__ __launch_bounds__(kThreads) void k_decouple(int p, int n, const int *__restrict__ rp,
                                                       const int *__restrict__ diag_pos,
                                                       const double *__restrict__ vals,
                                                       double *__restrict__ omega,
                                                       double *__restrict__ ap, int *bad)
{
#pragma clang fp contract(off)
    int c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= n) return;
    const double *D = vals + (long long)diag_pos[c] * B * B;
    double T[B][B], y[B], w[B];
#pragma unroll
    for (int r = 0; r < B; ++r)
#pragma unroll
        for (int s = 0; s < B; ++s) T[r][s] = D[s * B + r];
#pragma unroll
    for (int r = 0; r < B; ++r) y[r] = (r == p) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < B; ++k) {
        int piv = k;
        double best = fabs(T[k][k]);
#pragma unroll
        for (int r = k + 1; r < B; ++r) {
            double a = fabs(T[r][k]);
            if (a > best) { best = a; piv = r; }
        }
        if (best == 0.0) {
            atomicOr(bad, 1);
            return;
        }
        // swap rows k and piv (select-based, no dynamic register indexing)
#pragma unroll
        for (int r = k + 1; r < B; ++r) {
            if (r == piv) {
#pragma unroll
                for (int s = 0; s < B; ++s) {
                    double t = T[k][s];
                    T[k][s] = T[r][s];
                    T[r][s] = t;
                }
                double t = y[k];
                y[k] = y[r];
                y[r] = t;
            }
        }
#pragma unroll
        for (int r = k + 1; r < B; ++r) {
            double m = T[r][k] / T[k][k];
#pragma unroll
            for (int s = k + 1; s < B; ++s) T[r][s] = T[r][s] - m * T[k][s];
            y[r] = y[r] - m * y[k];
        }
    }
#pragma unroll
    for (int r = B - 1; r >= 0; --r) {
        double acc = y[r];
#pragma unroll
        for (int s = r + 1; s < B; ++s) acc = acc - T[r][s] * w[s];
        w[r] = acc / T[r][r];
    }
#pragma unroll
    for (int r = 0; r < B; ++r) omega[(long long)c * B + r] = w[r];
    for (int k = rp[c]; k < rp[c + 1]; ++k) {
        const double *blk = vals + (long long)k * B * B;
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < B; ++r) acc = acc + w[r] * blk[r * B + p];
        ap[k] = acc;
    }
}

// ---------------------------------------------------------------------------
// block ILU(0) factorisation, one dependency level per launch, one thread per
// block row: F_ik <- F_ik Dinv_k, F_ij <- F_ij - F_ik F_kj, Dinv_i = F_ii^-1.
// ---------------------------------------------------------------------------
template <int B>
__device__ bool invert_block(const double (&M)[B * B], double (&X)[B * B])
{
    double A[B][B];
    int perm[B];
#pragma unroll
    for (int r = 0; r < B; ++r) {
        perm[r] = r;
#pragma unroll
        for (int s = 0; s < B; ++s) A[r][s] = M[r * B + s];
    }
    bool ok = true;
#pragma unroll
    for (int k = 0; k < B; ++k) {
        int piv = k;
        double best = fabs(A[k][k]);
#pragma unroll
        for (int r = k + 1; r < B; ++r) {
            double a = fabs(A[r][k]);
            if (a > best) { best = a; piv = r; }
        }
        if (best == 0.0) ok = false;
#pragma unroll
        for (int r = k + 1; r < B; ++r) {
            if (r == piv) {
#pragma unroll
                for (int s = 0; s < B; ++s) {
                    double t = A[k][s];
                    A[k][s] = A[r][s];
                    A[r][s] = t;
                }
                int t = perm[k];
                perm[k] = perm[r];
                perm[r] = t;
            }
        }
        double inv = 1.0 / A[k][k];
#pragma unroll
        for (int r = k + 1; r < B; ++r) {
            A[r][k] = A[r][k] * inv;
#pragma unroll
            for (int s = k + 1; s < B; ++s) A[r][s] -= A[r][k] * A[k][s];
        }
    }
#pragma unroll
    for (int e = 0; e < B; ++e) {
        double y[B];
#pragma unroll
        for (int r = 0; r < B; ++r) {
            double acc = (perm[r] == e) ? 1.0 : 0.0;
#pragma unroll
            for (int s = 0; s < r; ++s) acc -= A[r][s] * y[s];
            y[r] = acc;
        }
#pragma unroll
        for (int r = B - 1; r >= 0; --r) {
            double acc = y[r];
#pragma unroll
            for (int s = r + 1; s < B; ++s) acc -= A[r][s] * y[s];
            y[r] = acc / A[r][r];
        }
#pragma unroll
        for (int r = 0; r < B; ++r) X[r * B + e] = y[r];
    }
    return ok;
}

// Block-Jacobi full-system smoother (the alternative R stage): Dinv_c =
// A_cc^-1 by the same partial-pivoting inversion as the block ILU(0) pivots,
// and y_c <- Dinv_c y_c in place.
template <int B>
__global__ __launch_bounds__(kThreads) void k_block_inverse(int n, const int *__restrict__ diag_pos,
                                                            const double *__restrict__ vals,
                                                            double *__restrict__ Dinv, int *bad)
{
    constexpr int E = B * B;
    const int c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= n) return;
    double M[E], X[E];
    const double *src = vals + (long long)diag_pos[c] * E;
#pragma unroll
    for (int e = 0; e < E; ++e) M[e] = src[e];
    if (!invert_block<B>(M, X)) atomicOr(bad, 1);
#pragma unroll
    for (int e = 0; e < E; ++e) Dinv[(long long)c * E + e] = X[e];
}

template <int B, typename T>
__global__ __launch_bounds__(kThreads) void k_block_jacobi(int n, const T *__restrict__ Dinv,
                                                           T *__restrict__ y)
{
    constexpr int E = B * B;
    const int c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= n) return;
    T v[B];
#pragma unroll
    for (int s = 0; s < B; ++s) v[s] = y[(long long)c * B + s];
    const T *D = Dinv + (long long)c * E;
#pragma unroll
    for (int a = 0; a < B; ++a) {
        T acc = 0;
#pragma unroll
        for (int s = 0; s < B; ++s) acc += D[a * B + s] * v[s];
        y[(long long)c * B + a] = acc;
    }
}

template <int B>
__global__ __launch_bounds__(64) void k_bilu_factor(BiluTasks t, double *__restrict__ F,
                                                    double *__restrict__ Dinv, int *bad)
{
    constexpr int E = B * B;
    int idx = blockIdx.x * 64 + threadIdx.x;
    if (idx >= t.nrows) return;
    const int i = t.rows[idx];
    const int r0 = t.rp[i], r1 = t.rp[i + 1], pi = t.pos[i];
    int last = -1;  // elimination position of the last lower entry taken
    for (;;) {
        // the next stored lower entry in elimination order
        int kk = -1, pk = pi;
        for (int q = r0; q < r1; ++q) {
            const int pj = t.pos[t.ci[q]];
            if (pj > last && pj < pk) {
                pk = pj;
                kk = q;
            }
        }
        if (kk < 0) break;
        last = pk;
        const int k = t.ci[kk];
        double L[E], P[E];
#pragma unroll
        for (int e = 0; e < E; ++e) L[e] = F[(long long)kk * E + e];
        const double *Dk = Dinv + (long long)k * E;
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int s = 0; s < B; ++s) {
                double acc = 0.0;
#pragma unroll
                for (int u = 0; u < B; ++u) acc += L[r * B + u] * Dk[u * B + s];
                P[r * B + s] = acc;
            }
#pragma unroll
        for (int e = 0; e < E; ++e) F[(long long)kk * E + e] = P[e];
        // columns stored in both rows i and k, eliminated after k
        int x = r0, y = t.rp[k];
        const int ye = t.rp[k + 1];
        while (x < r1 && y < ye) {
            const int jx = t.ci[x], jy = t.ci[y];
            if (jx < jy) {
                ++x;
                continue;
            }
            if (jy < jx) {
                ++y;
                continue;
            }
            if (t.pos[jx] > pk) {
                const double *Fkj = F + (long long)y * E;
                double *Fij = F + (long long)x * E;
                double K[E];
#pragma unroll
                for (int e = 0; e < E; ++e) K[e] = Fkj[e];
#pragma unroll
                for (int r = 0; r < B; ++r) {
                    double row[B];
#pragma unroll
                    for (int s = 0; s < B; ++s) row[s] = Fij[r * B + s];
#pragma unroll
                    for (int s = 0; s < B; ++s) {
                        double acc = 0.0;
#pragma unroll
                        for (int u = 0; u < B; ++u) acc += P[r * B + u] * K[u * B + s];
                        row[s] -= acc;
                    }
#pragma unroll
                    for (int s = 0; s < B; ++s) Fij[r * B + s] = row[s];
                }
            }
            ++x;
            ++y;
        }
    }
    double M[E], X[E];
    const long long dp = t.diag_pos[i];
#pragma unroll
    for (int e = 0; e < E; ++e) M[e] = F[dp * E + e];
    if (!invert_block<B>(M, X)) atomicOr(bad, 1);
#pragma unroll
    for (int e = 0; e < E; ++e) Dinv[(long long)i * E + e] = X[e];
}

// one thread per (slice, lane): the row's triangular entries by selection in
// elimination order (rows are short), then padding up to the slice width
__global__ __launch_bounds__(kThreads) void k_tri_fill(int nslices, const int4 *__restrict__ slices,
                                                      const int *__restrict__ rows,
                                                      const int *__restrict__ rp,
                                                      const int *__restrict__ ci,
                                                      const int *__restrict__ pos, int lower,
                                                      int *__restrict__ col,
                                                      int *__restrict__ src)
{
    const long long g = (long long)blockIdx.x * kThreads + threadIdx.x;
    const int s = (int)(g >> 6), lane = (int)(g & 63);
    if (s >= nslices) return;
    const int4 d = slices[s];  // first row, rows, width, slot-lane offset
    int m = 0;
    if (lane < d.y) {
        const int i = rows[d.x + lane];
        const int r0 = rp[i], r1 = rp[i + 1], pi = pos[i];
        // lower: positions in (last, pi); upper: positions above last = pi
        int last = lower ? -1 : pi;
        const int lim = lower ? pi : 0x7fffffff;
        for (;;) {
            int qb = -1, pb = lim;
            for (int q = r0; q < r1; ++q) {
                const int pj = pos[ci[q]];
                if (pj > last && pj < pb) {
                    pb = pj;
                    qb = q;
                }
            }
            if (qb < 0) break;
            last = pb;
            const long long o = (long long)d.w + (long long)m * 64 + lane;
            col[o] = pb;  // the solves run on vectors in elimination order
            src[o] = qb;
            ++m;
        }
    }
    for (; m < d.z; ++m) {
        const long long o = (long long)d.w + (long long)m * 64 + lane;
        col[o] = -1;
        src[o] = -1;
    }
}

// ---------------------------------------------------------------------------
// block SpMV (FP64), one thread per block row of a 64-row slice.  The matrix
// values and column indices are read once per SpMV, so they are loaded
// non-temporally (they do not displace the x entries that neighbouring rows
// gather again).  A padding slot (column -1, value 0) reads the row's own x
// block and adds nothing: no branch per entry, so the loads of consecutive
// entries issue back to back.
// ---------------------------------------------------------------------------
template <int B>
__global__ __launch_bounds__(kThreads) void k_spmv(const int4 *__restrict__ slices,
                                                   const int *__restrict__ col, int s0, int s1,
                                                   const double *__restrict__ val,
                                                   const double *__restrict__ x,
                                                   const double *__restrict__ sub,
                                                   double *__restrict__ y)
{
    constexpr int E = B * B;
    const int s = s0 + xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (s >= s1) return;
    const int lane = threadIdx.x & 63;
    const int4 d = slices[s];
    if (lane >= d.y) return;
    const long long row = d.x + lane;
    double acc[B];
#pragma unroll
    for (int r = 0; r < B; ++r) acc[r] = 0.0;
    const int *cb = col + d.w + lane;
    const double *vb = val + (long long)(d.w >> 6) * 64 * E + lane;
    for (int k = 0; k < d.z; ++k) {
        const int c = __builtin_nontemporal_load(cb + k * 64);
        const long long cs = c >= 0 ? c : row;
        double xv[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const double t = x[cs * B + u];
            xv[u] = c >= 0 ? t : 0.0;
        }
        const double *v = vb + (long long)k * 64 * E;
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int u = 0; u < B; ++u)
                acc[r] += __builtin_nontemporal_load(v + (r * B + u) * 64) * xv[u];
    }
#pragma unroll
    for (int r = 0; r < B; ++r)
        y[row * B + r] = sub ? sub[row * B + r] - acc[r] : acc[r];
}

// ---------------------------------------------------------------------------
// preconditioner kernels
// ---------------------------------------------------------------------------
template <int B, typename T>
__global__ __launch_bounds__(kThreads) void k_decouple_restrict(int n,
                                                                const int *__restrict__ iperm0,
                                                                const double *__restrict__ omega,
                                                                const double *v,
                                                                const ApplyIo *io,
                                                                T *__restrict__ g)
{
    int t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= n) return;
    if (io) v = io->v;
    const long long c = iperm0[t];
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < B; ++k) acc += omega[c * B + k] * v[c * B + k];
    g[t] = (T)acc;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_gs_first(int npos, int p0, int p1,
                                                       const T *__restrict__ diag,
                                                       const T *__restrict__ f,
                                                       T *__restrict__ x)
{
    int t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= npos) return;
    x[t] = (t >= p0 && t < p1) ? f[t] / diag[t] : T(0);
}

// sum0 + sum over the stored entries k < width of one sliced-ELL row (lane
// stride 64) of val[k] x[col[k]], in k order, padding (col < 0) skipped.  The
// entries go in batches of 8: the column and value loads of a batch issue
// together, then its gathers of x, so a row costs two memory round trips per
// batch instead of two per entry.
template <typename T>
__device__ inline T sell_row_dot(const int *__restrict__ cb, const T *__restrict__ vb, int width,
                                 const T *x, T sum0 = 0)
{
    T sum = sum0;
    for (int k0 = 0; k0 < width; k0 += 8) {
        int c[8];
        T v[8], xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const bool in = k0 + u < width;
            c[u] = in ? __builtin_nontemporal_load(cb + (k0 + u) * 64) : -1;
            v[u] = in ? __builtin_nontemporal_load(vb + (k0 + u) * 64) : T(0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) xv[u] = c[u] >= 0 ? x[c[u]] : T(0);
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (c[u] >= 0) sum += v[u] * xv[u];
    }
    return sum;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_gs_color(const int4 *__restrict__ slices,
                                                       const int *__restrict__ col, int s0,
                                                       int s1, const T *__restrict__ val,
                                                       const T *__restrict__ diag,
                                                       const T *__restrict__ f, T *x)
{
    const int s = s0 + xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (s >= s1) return;
    const int lane = threadIdx.x & 63;
    const int4 d = slices[s];
    if (lane >= d.y) return;
    const int row = d.x + lane;
    const T fr = f[row], dr = diag[row];
    const T sum = sell_row_dot<T>(col + d.w + lane, val + d.w + lane, d.z, x);
    x[row] = (fr - sum) / dr;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_residual(const int4 *__restrict__ slices,
                                                       const int *__restrict__ col, int s0,
                                                       int s1, const T *__restrict__ val,
                                                       const T *__restrict__ diag,
                                                       const T *__restrict__ f,
                                                       const T *__restrict__ x,
                                                       T *__restrict__ r)
{
    const int s = s0 + xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (s >= s1) return;
    const int lane = threadIdx.x & 63;
    const int4 d = slices[s];
    if (lane >= d.y) return;
    const int row = d.x + lane;
    const T fr = f[row];
    const T sum = sell_row_dot<T>(col + d.w + lane, val + d.w + lane, d.z, x, diag[row] * x[row]);
    r[row] = fr - sum;
}

// The same sweep and residual with each row's stored entries spread over L
// lanes (entry k on lane k mod L) and summed across them with a fixed
// butterfly.  A wave holds 64 / L rows, so a slice takes L waves.  Lane
// (j, t) = (entry phase, row) sits at j * (64 / L) + t: lanes of one phase
// read consecutive rows of a slot, which are contiguous in the layout.
template <typename T, int L, bool RESIDUAL>
__device__ inline void sweep_row_lanes(const int4 *__restrict__ slices,
                                       const int *__restrict__ col, int s0, int s1,
                                       const T *__restrict__ val, const T *__restrict__ diag,
                                       const T *__restrict__ f, T *x, T *__restrict__ r)
{
    constexpr int RPW = 64 / L;  // rows per wave
    const int gw = xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    const int s = s0 + gw / L;
    if (s >= s1) return;  // uniform over the wave
    const int lane = threadIdx.x & 63, t = lane % RPW, j = lane / RPW;
    const int4 d = slices[s];
    const int local = (gw % L) * RPW + t;
    const bool live = local < d.y;
    const int row = d.x + local;
    T fr = 0, dr = 1, xr = 0;
    if (live && j == 0) {
        fr = f[row];
        dr = diag[row];
        if (RESIDUAL) xr = x[row];
    }
    T sum = 0;
    if (live) {
        const int *cb = col + d.w + local;
        const T *vb = val + d.w + local;
        for (int k0 = j; k0 < d.z; k0 += 8 * L) {
            int c[8];
            T v[8], xv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = k0 + u * L;
                const bool in = k < d.z;
                c[u] = in ? __builtin_nontemporal_load(cb + k * 64) : -1;
                v[u] = in ? __builtin_nontemporal_load(vb + k * 64) : T(0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) xv[u] = c[u] >= 0 ? x[c[u]] : T(0);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (c[u] >= 0) sum += v[u] * xv[u];
        }
    }
#pragma unroll
    for (int o = RPW; o < 64; o <<= 1) sum += __shfl_xor(sum, o, 64);
    if (live && j == 0) {
        if (RESIDUAL)
            r[row] = fr - (dr * xr + sum);
        else
            x[row] = (fr - sum) / dr;
    }
}

template <typename T, int L>
__global__ __launch_bounds__(kThreads) void k_gs_color_lanes(
    const int4 *__restrict__ slices, const int *__restrict__ col, int s0, int s1,
    const T *__restrict__ val, const T *__restrict__ diag, const T *__restrict__ f, T *x)
{
    sweep_row_lanes<T, L, false>(slices, col, s0, s1, val, diag, f, x, nullptr);
}

template <typename T, int L>
__global__ __launch_bounds__(kThreads) void k_residual_lanes(
    const int4 *__restrict__ slices, const int *__restrict__ col, int s0, int s1,
    const T *__restrict__ val, const T *__restrict__ diag, const T *__restrict__ f,
    const T *__restrict__ x, T *__restrict__ r)
{
    sweep_row_lanes<T, L, true>(slices, col, s0, s1, val, diag, f, const_cast<T *>(x), r);
}

// Weighted point-Jacobi smoothing (the PJAC ablation of Sec. 6): the first
// sweep from x = 0 is x = w D^-1 f; a later sweep is x += w D^-1 r with
// r = f - A x from k_residual (all rows read the old x).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_jacobi_first(int n, T w, const T *__restrict__ diag,
                                                           const T *__restrict__ f,
                                                           T *__restrict__ x)
{
    int t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= n) return;
    x[t] = w * (f[t] / diag[t]);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_jacobi_update(int n, T w,
                                                            const T *__restrict__ diag,
                                                            const T *__restrict__ r,
                                                            T *__restrict__ x)
{
    int t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= n) return;
    x[t] = x[t] + w * (r[t] / diag[t]);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_zero(int n, T *__restrict__ x)
{
    int t = blockIdx.x * kThreads + threadIdx.x;
    if (t < n) x[t] = T(0);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_restrict(int nc, const int *__restrict__ mem_ptr,
                                                       const int *__restrict__ mem,
                                                       const T *__restrict__ r,
                                                       T *__restrict__ fc)
{
    int J = blockIdx.x * kThreads + threadIdx.x;
    if (J >= nc) return;
    T s = 0;
    for (int m = mem_ptr[J]; m < mem_ptr[J + 1]; ++m) s += r[mem[m]];
    fc[J] = s;
}

// k_restrict, then the first color of the coarse level's forward sweep from
// x = 0 (k_gs_first): the same two results, in one pass.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_restrict_first(int nc, const int *__restrict__ mem_ptr,
                                                             const int *__restrict__ mem,
                                                             const T *__restrict__ r,
                                                             T *__restrict__ fc, int p0, int p1,
                                                             const T *__restrict__ diag_c,
                                                             T *__restrict__ xc)
{
    int J = blockIdx.x * kThreads + threadIdx.x;
    if (J >= nc) return;
    T s = 0;
    for (int m = mem_ptr[J]; m < mem_ptr[J + 1]; ++m) s += r[mem[m]];
    fc[J] = s;
    xc[J] = (J >= p0 && J < p1) ? s / diag_c[J] : T(0);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_prolong(int n, const int *__restrict__ agg_pos,
                                                      const T *__restrict__ xc,
                                                      T *__restrict__ x)
{
    int t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= n) return;
    x[t] += xc[agg_pos[t]];
}

// Maps between a level and the next coarser one in position space, from the
// same maps in the coarse level's natural order: thread t < n sets
// agg_pos[t] = cperm[natc[t]]; thread J < nc moves coarse row J's member list
// (mem_nat[mptr_nat[J] .. mptr_nat[J+1])) to mem[mptr_pos[cperm[J]] ..].
__global__ __launch_bounds__(kThreads) void k_link(int n, int nc, const int *__restrict__ natc,
                                                   const int *__restrict__ mptr_nat,
                                                   const int *__restrict__ mem_nat,
                                                   const int *__restrict__ cperm,
                                                   const int *__restrict__ mptr_pos,
                                                   int *__restrict__ agg_pos,
                                                   int *__restrict__ mem)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) agg_pos[i] = cperm[natc[i]];
    if (i < nc) {
        const int a = mptr_nat[i], b = mptr_nat[i + 1];
        const int d = mptr_pos[cperm[i]] - a;
        for (int k = a; k < b; ++k) mem[d + k] = mem_nat[k];
    }
}

// x = Ainv f on the coarsest level, FP64 arithmetic, one wave per row; rows
// are 16-byte aligned (ld even) so each lane streams pairs of doubles.
// One triangle of the coarsest-level solve x = W (Y f), row-major FP64
// factors of leading dimension ld (even) and block size P (even).  With
// LOWER, out_i = in_i + sum over j < bs(i) of Y_ij in_j, where bs(i) is the
// first row of i's block (Y is block unit lower triangular); otherwise
// out_i = sum over j >= bs(i) of W_ij in_j (W is block upper triangular).
// One wavefront per row, 16-byte loads from bs(i) (a multiple of P) on.
template <bool LOWER, typename TI, typename TO>
__global__ __launch_bounds__(kThreads) void k_coarse_tri(int n, int ld, int P,
                                                         const double *__restrict__ F,
                                                         const TI *__restrict__ in,
                                                         TO *__restrict__ out)
{
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= n) return;
    const int lane = threadIdx.x & 63;
    const int bs = row - row % P;
    const int lo = LOWER ? 0 : bs, hi = LOWER ? bs : n;
    const double2 *a = reinterpret_cast<const double2 *>(F + (long long)row * ld);
    double acc = 0.0;
#pragma unroll 4
    for (int j2 = (lo >> 1) + lane; j2 < (hi >> 1); j2 += 64) {
        const double2 v = a[j2];
        acc += v.x * (double)in[2 * j2] + v.y * (double)in[2 * j2 + 1];
    }
    if ((hi & 1) && lane == 0) acc += F[(long long)row * ld + hi - 1] * (double)in[hi - 1];
    acc = wave_sum(acc);
    if (lane == 0) out[row] = (TO)(LOWER ? acc + (double)in[row] : acc);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_unpermute(int n, const int *__restrict__ perm0,
                                                        const T *__restrict__ epos,
                                                        T *__restrict__ enat)
{
    int c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= n) return;
    enat[c] = epos[perm0[c]];
}

template <int B, typename T, bool F32>
__global__ __launch_bounds__(kThreads) void k_pcol_residual(
    int p, const int4 *__restrict__ slices, const int *__restrict__ col, int s0, int s1,
    const double *__restrict__ val64, const float *__restrict__ pcol32,
    const double *v, const ApplyIo *io, const T *__restrict__ e, const int *__restrict__ rperm,
    T *__restrict__ r)
{
    constexpr int E = B * B;
    if (io) v = io->v;
    const int s = s0 + xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (s >= s1) return;
    const int lane = threadIdx.x & 63;
    const int4 d = slices[s];
    if (lane >= d.y) return;
    const long long row = d.x + lane;
    T acc[B];
#pragma unroll
    for (int k = 0; k < B; ++k) acc[k] = 0;
    const int *cb = col + d.w + lane;
    for (int k0 = 0; k0 < d.z; k0 += 8) {  // column indices, then e, in batches of 8
        int cc[8];
        T ev[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            cc[u] = k0 + u < d.z ? __builtin_nontemporal_load(cb + (k0 + u) * 64) : -1;
#pragma unroll
        for (int u = 0; u < 8; ++u) ev[u] = cc[u] >= 0 ? e[cc[u]] : T(0);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (cc[u] < 0) continue;
            const T ec = ev[u];
            const long long sb = (long long)(d.w >> 6) + k0 + u;
#pragma unroll
            for (int q = 0; q < B; ++q) {
                T a;
                if (F32)
                    a = (T)__builtin_nontemporal_load(pcol32 + sb * 64 * B + q * 64 + lane);
                else
                    a = (T)__builtin_nontemporal_load(val64 + sb * 64 * E + (q * B + p) * 64 + lane);
                acc[q] += a * ec;
            }
        }
    }
    const long long ro = rperm ? rperm[row] : row;
#pragma unroll
    for (int q = 0; q < B; ++q) r[ro * B + q] = (T)v[row * B + q] - acc[q];
}

// Block ILU(0) triangular solves, one dependency level per launch, one
// thread per block row of a 64-row slice.  As in k_spmv: the factor values
// and column indices are read once per solve (non-temporal loads), padding
// slots read the row's own block and add nothing, and slices are assigned to
// XCDs in contiguous ranges.
template <int B, typename T>
__global__ __launch_bounds__(kThreads) void k_bilu_fwd(const int4 *__restrict__ slices,
                                                       const int *__restrict__ col, int s0,
                                                       int s1, const int *__restrict__ rows,
                                                       const T *__restrict__ Lval, T *y)
{
    constexpr int E = B * B;
    const int s = s0 + xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (s >= s1) return;
    const int lane = threadIdx.x & 63;
    const int4 d = slices[s];
    if (lane >= d.y) return;
    const long long i = rows[d.x + lane];
    T acc[B];
#pragma unroll
    for (int r = 0; r < B; ++r) acc[r] = 0;
    const int *cb = col + d.w + lane;
    const T *vb = Lval + (long long)(d.w >> 6) * 64 * E + lane;
    for (int k = 0; k < d.z; ++k) {
        const int c = __builtin_nontemporal_load(cb + k * 64);
        const long long cs = c >= 0 ? c : i;
        T yk[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const T t = y[cs * B + u];
            yk[u] = c >= 0 ? t : T(0);
        }
        const T *v = vb + (long long)k * 64 * E;
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int u = 0; u < B; ++u)
                acc[r] += __builtin_nontemporal_load(v + (r * B + u) * 64) * yk[u];
    }
#pragma unroll
    for (int r = 0; r < B; ++r) y[i * B + r] = y[i * B + r] - acc[r];
}

template <int B, typename T>
__global__ __launch_bounds__(kThreads) void k_bilu_bwd(const int4 *__restrict__ slices,
                                                       const int *__restrict__ col, int s0,
                                                       int s1, const int *__restrict__ rows,
                                                       const T *__restrict__ Uval,
                                                       const T *__restrict__ Dval, T *z)
{
    constexpr int E = B * B;
    const int s = s0 + xcd_block(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
    if (s >= s1) return;
    const int lane = threadIdx.x & 63;
    const int4 d = slices[s];
    if (lane >= d.y) return;
    const long long i = rows[d.x + lane];
    T t[B];
#pragma unroll
    for (int r = 0; r < B; ++r) t[r] = z[i * B + r];
    const int *cb = col + d.w + lane;
    const T *vb = Uval + (long long)(d.w >> 6) * 64 * E + lane;
    for (int k = 0; k < d.z; ++k) {
        const int c = __builtin_nontemporal_load(cb + k * 64);
        const long long cs = c >= 0 ? c : i;
        T zk[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const T w = z[cs * B + u];
            zk[u] = c >= 0 ? w : T(0);
        }
        const T *v = vb + (long long)k * 64 * E;
#pragma unroll
        for (int r = 0; r < B; ++r) {
            T a = 0;
#pragma unroll
            for (int u = 0; u < B; ++u) a += __builtin_nontemporal_load(v + (r * B + u) * 64) * zk[u];
            t[r] -= a;
        }
    }
    const T *D = Dval + (long long)s * 64 * E + lane;
#pragma unroll
    for (int r = 0; r < B; ++r) {
        T a = 0;
#pragma unroll
        for (int u = 0; u < B; ++u) a += __builtin_nontemporal_load(D + (r * B + u) * 64) * t[u];
        z[i * B + r] = a;
    }
}

template <int B, typename T>
__global__ __launch_bounds__(kThreads) void k_finish(int p, int n, const T *__restrict__ zz,
                                                     const int *__restrict__ zperm,
                                                     const T *__restrict__ e,
                                                     const double *__restrict__ w1,
                                                     double *z, const ApplyIo *io)
{
    long long q = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (q >= (long long)n * B) return;
    if (io) z = io->z;
    const int k = (int)(q % B);
    const long long c = q / B;
    const long long qz = zperm ? (long long)zperm[c] * B + k : q;
    const double v = (double)zz[qz] + (k == p ? (double)e[c] : 0.0);
    z[q] = w1 ? v + w1[q] : v;
}

// ---------------------------------------------------------------------------
// N stage (the concentration stage B_N of eq. MSP): one block Gauss-Seidel
// sweep on the decoupled concentration block.  With D_c = A_cc its diagonal
// blocks are the identity; the off-diagonal blocks are (D_c^-1 A_cd)[N, N]
// and the right-hand side is (D_c^-1 v_c)[N], N = unknowns other than p.
// ---------------------------------------------------------------------------
template <int B>
__global__ __launch_bounds__(kThreads) void k_decouple_n(int n, int p, const int *__restrict__ rp,
                                                         const int *__restrict__ ci,
                                                         const int *__restrict__ diag_pos,
                                                         const double *__restrict__ vals,
                                                         double *__restrict__ Dn,
                                                         double *__restrict__ Ann, int *bad)
{
    constexpr int E = B * B, M = B - 1;
    const int c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= n) return;
    double Dm[E], Di[E];
    const double *dblk = vals + (long long)diag_pos[c] * E;
#pragma unroll
    for (int e = 0; e < E; ++e) Dm[e] = dblk[e];
    if (!invert_block<B>(Dm, Di)) atomicOr(bad, 1);
#pragma unroll
    for (int a = 0, ra = 0; a < B; ++a) {
        if (a == p) continue;
#pragma unroll
        for (int s = 0; s < B; ++s) Dn[((long long)c * M + ra) * B + s] = Di[a * B + s];
        ++ra;
    }
    for (int q = rp[c]; q < rp[c + 1]; ++q) {
        double *out = Ann + (long long)q * M * M;
        const double *blk = vals + (long long)q * E;
        const bool dg = ci[q] == c;
        for (int a = 0, ra = 0; a < B; ++a) {
            if (a == p) continue;
            for (int t = 0, rt = 0; t < B; ++t) {
                if (t == p) continue;
                double acc = 0.0;
#pragma unroll
                for (int u = 0; u < B; ++u) acc = acc + Di[a * B + u] * blk[u * B + t];
                out[ra * M + rt] = dg ? (ra == rt ? 1.0 : 0.0) : acc;
                ++rt;
            }
            ++ra;
        }
    }
}

// gN_c = Dn_c v_c (rows N of D_c^-1 times v_c), in the preconditioner precision
template <int B, typename T>
__global__ __launch_bounds__(kThreads) void k_n_rhs(int n, const T *__restrict__ Dn,
                                                    const double *__restrict__ v,
                                                    T *__restrict__ gN)
{
    constexpr int M = B - 1;
    const int c = blockIdx.x * kThreads + threadIdx.x;
    if (c >= n) return;
    T vc[B];
#pragma unroll
    for (int s = 0; s < B; ++s) vc[s] = (T)v[(long long)c * B + s];
#pragma unroll
    for (int a = 0; a < M; ++a) {
        T acc = 0;
#pragma unroll
        for (int s = 0; s < B; ++s) acc = acc + Dn[((long long)c * M + a) * B + s] * vc[s];
        gN[(long long)c * M + a] = acc;
    }
}

// one group of the sweep: y_c = gN_c - sum_{d != c} Ann_cd y_d for the cells
// of the group (independent: no stored block joins two cells of one group)
template <int B, typename T>
__global__ __launch_bounds__(kThreads) void k_bgs_group(int ncell, const int *__restrict__ cells,
                                                        const int *__restrict__ rp,
                                                        const int *__restrict__ ci,
                                                        const T *__restrict__ Ann,
                                                        const T *__restrict__ gN, T *y)
{
    constexpr int M = B - 1, M1 = M > 0 ? M : 1;
    const int idx = blockIdx.x * kThreads + threadIdx.x;
    if (idx >= ncell) return;
    const int c = cells[idx];
    T acc[M1];
#pragma unroll
    for (int a = 0; a < M; ++a) acc[a] = gN[(long long)c * M + a];
    for (int q = rp[c]; q < rp[c + 1]; ++q) {
        const int d = ci[q];
        if (d == c) continue;
        T yd[M1];
#pragma unroll
        for (int t = 0; t < M; ++t) yd[t] = y[(long long)d * M + t];
        const T *blk = Ann + (long long)q * M * M;
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int t = 0; t < M; ++t) acc[a] = acc[a] - blk[a * M + t] * yd[t];
    }
#pragma unroll
    for (int a = 0; a < M; ++a) y[(long long)c * M + a] = acc[a];
}

// w1 = Pi_N y (FP64, zero at the pressure unknowns)
template <int B, typename T>
__global__ __launch_bounds__(kThreads) void k_expand_n(int n, int p, const T *__restrict__ y,
                                                       double *__restrict__ w1)
{
    long long q = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (q >= (long long)n * B) return;
    const int k = (int)(q % B);
    const long long c = q / B;
    w1[q] = (k == p) ? 0.0 : (double)y[c * (B - 1) + (k < p ? k : k - 1)];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_to_double(long long n, const T *__restrict__ x,
                                                        double *__restrict__ y)
{
    long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) y[i] = (double)x[i];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_from_double(long long n,
                                                          const double *__restrict__ x,
                                                          T *__restrict__ y)
{
    long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) y[i] = (T)x[i];
}

// ---------------------------------------------------------------------------
// Krylov vector kernels (FP64).  The dot products use a fixed grid and a fixed
// reduction tree: identical results on every run.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_dot_multi(long long N, int nv,
                                                        const double *__restrict__ V,
                                                        long long ldv,
                                                        const double *__restrict__ w,
                                                        double *__restrict__ partial)
{
    __shared__ double red[4][8];
    const long long chunk = ((N + gridDim.x - 1) / gridDim.x + 63) & ~63LL;
    const long long b0 = (long long)blockIdx.x * chunk;
    const long long b1 = b0 + chunk < N ? b0 + chunk : N;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i0 = 0; i0 < nv; i0 += 8) {
        double acc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = 0.0;
        const int nu = nv - i0 < 8 ? nv - i0 : 8;
        for (long long q = b0 + threadIdx.x; q < b1; q += kThreads) {
            const double wq = w[q];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (u < nu) acc[u] += V[(long long)(i0 + u) * ldv + q] * wq;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            double v = wave_sum(acc[u]);
            if (lane == 0) red[wave][u] = v;
        }
        __syncthreads();
        if (threadIdx.x < nu)
            partial[(long long)blockIdx.x * nv + i0 + threadIdx.x] =
                (red[0][threadIdx.x] + red[1][threadIdx.x]) +
                (red[2][threadIdx.x] + red[3][threadIdx.x]);
        __syncthreads();
    }
}

// out[i] = sum over the nblk blocks of partial[b * nv + i]: one wave per
// vector i (lane l adds blocks l, l + 64, ... in order, then a fixed
// butterfly across the wave), so every sum has a fixed order.
constexpr int kReduceThreads = 1024;
__global__ __launch_bounds__(kReduceThreads) void k_reduce_partials(
    int nv, int nblk, const double *__restrict__ partial, double *__restrict__ out,
    int accumulate)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = wave; i < nv; i += kReduceThreads / 64) {
        double s = 0.0;
        for (int b = lane; b < nblk; b += 64) s += partial[(long long)b * nv + i];
        s = wave_sum(s);
        if (lane == 0) out[i] = accumulate ? out[i] + s : s;
    }
}

__global__ __launch_bounds__(kThreads) void k_axpy_multi(long long N, int nv,
                                                         const double *__restrict__ V,
                                                         long long ldv,
                                                         const double *__restrict__ h,
                                                         double *__restrict__ w)
{
    __shared__ double hs[256];
    for (int i = threadIdx.x; i < nv; i += kThreads) hs[i] = h[i];
    __syncthreads();
    for (long long q = (long long)blockIdx.x * kThreads + threadIdx.x; q < N;
         q += (long long)gridDim.x * kThreads) {
        double acc = 0.0;
        for (int i = 0; i < nv; ++i) acc += hs[i] * V[(long long)i * ldv + q];
        w[q] -= acc;
    }
}

// One pass of the Gram-Schmidt step over the nv = NV basis vectors V_i (the
// count is a template parameter, so a row's NV entries load together with no
// per-vector tests):
//   MODE 0: partial sums of V_i . w;
//   MODE 1: w -= V h, then partial sums of V_i . w (the updated w);
//   MODE 2: w -= V h, then partial sums of w . w.
// Each V entry is read once per pass.  Every block sums a fixed chunk of rows
// (each thread its rows in ascending order) and combines its four waves in a
// fixed tree, so the partials are the same on every run.
template <int NV, int MODE>
__global__ __launch_bounds__(kThreads) void k_gs_pass(long long N, const double *__restrict__ V,
                                                      long long ldv,
                                                      const double *__restrict__ h,
                                                      double *__restrict__ w,
                                                      double *__restrict__ partial)
{
    constexpr int NOUT = MODE == 2 ? 1 : NV;
    __shared__ double hs[NV];
    __shared__ double red[4][NOUT];
    if (MODE != 0) {
        for (int i = threadIdx.x; i < NV; i += kThreads) hs[i] = h[i];
        __syncthreads();
    }
    const long long chunk = ((N + gridDim.x - 1) / gridDim.x + 63) & ~63LL;
    const long long b0 = (long long)blockIdx.x * chunk;
    const long long b1 = b0 + chunk < N ? b0 + chunk : N;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double acc[NOUT];
#pragma unroll
    for (int i = 0; i < NOUT; ++i) acc[i] = 0.0;
    for (long long q = b0 + threadIdx.x; q < b1; q += kThreads) {
        double v[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = V[(long long)i * ldv + q];
        double wq = w[q];
        if (MODE != 0) {
            double a = 0.0;
#pragma unroll
            for (int i = 0; i < NV; ++i) a += hs[i] * v[i];
            wq -= a;
            w[q] = wq;
        }
        if (MODE == 2) {
            acc[0] += wq * wq;
        } else {
#pragma unroll
            for (int i = 0; i < NOUT; ++i) acc[i] += v[i] * wq;
        }
    }
#pragma unroll
    for (int i = 0; i < NOUT; ++i) {
        const double t = wave_sum(acc[i]);
        if (lane == 0) red[wave][i] = t;
    }
    __syncthreads();
    if (threadIdx.x < NOUT)
        partial[(long long)blockIdx.x * NOUT + threadIdx.x] =
            (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

__global__ __launch_bounds__(kThreads) void k_scale(long long N, const double *__restrict__ x,
                                                    double s, double *__restrict__ y)
{
    for (long long q = (long long)blockIdx.x * kThreads + threadIdx.x; q < N;
         q += (long long)gridDim.x * kThreads)
        y[q] = x[q] / s;
}

__global__ __launch_bounds__(kThreads) void k_update_x(long long N, int k,
                                                       const double *__restrict__ Z,
                                                       long long ldz,
                                                       const double *__restrict__ y,
                                                       double *__restrict__ x)
{
    __shared__ double ys[256];
    for (int i = threadIdx.x; i < k; i += kThreads) ys[i] = y[i];
    __syncthreads();
    for (long long q = (long long)blockIdx.x * kThreads + threadIdx.x; q < N;
         q += (long long)gridDim.x * kThreads) {
        double acc = x[q];
        for (int i = 0; i < k; ++i) acc += ys[i] * Z[(long long)i * ldz + q];
        x[q] = acc;
    }
}

__global__ __launch_bounds__(kThreads) void k_fill(long long N, double v, double *__restrict__ x)
{
    for (long long q = (long long)blockIdx.x * kThreads + threadIdx.x; q < N;
         q += (long long)gridDim.x * kThreads)
        x[q] = v;
}

// ---------------------------------------------------------------------------
// dense coarsest level: scatter, pivot-block inverses, block LU and the
// triangular-inverse sweeps
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_dense_scatter(int n, int ld,
                                                            const int *__restrict__ rp,
                                                            const int *__restrict__ ci,
                                                            const double *__restrict__ val,
                                                            double *__restrict__ M)
{
    int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    for (int k = rp[i]; k < rp[i + 1]; ++k) M[(long long)i * ld + ci[k]] = val[k];
}

constexpr int kNB = 128;  // pivot block of k_gj_diag

// Largest 64-bit key over the wavefront: butterflies inside each row of 16
// lanes by DPP moves, then the four row maxima read as scalars.
template <int CTRL>
__device__ inline unsigned long long dpp_u64(unsigned long long x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)x, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(x >> 32), CTRL, 0xf, 0xf, true);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}
__device__ inline unsigned long long umax64(unsigned long long a, unsigned long long b)
{
    return a > b ? a : b;
}
__device__ inline unsigned long long readlane_u64(unsigned long long x, int l)
{
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), l);
    return ((unsigned long long)hi << 32) | lo;
}
__device__ inline unsigned long long wave_max_u64(unsigned long long k)
{
    k = umax64(k, dpp_u64<0xB1>(k));   // quad_perm [1,0,3,2]
    k = umax64(k, dpp_u64<0x4E>(k));   // quad_perm [2,3,0,1]
    k = umax64(k, dpp_u64<0x141>(k));  // row_half_mirror
    k = umax64(k, dpp_u64<0x140>(k));  // row_mirror
    return umax64(umax64(readlane_u64(k, 0), readlane_u64(k, 16)),
                  umax64(readlane_u64(k, 32), readlane_u64(k, 48)));
}
__device__ inline double readlane_f64(double x, int l)
{
    return __longlong_as_double((long long)readlane_u64((unsigned long long)__double_as_longlong(x), l));
}

// Pivot key of row r (< 128): |v| with its 8 lowest mantissa bits replaced by
// 255 - r, so the largest key is the largest magnitude (to 2^-44 relative)
// and the lowest row among equals; 0 marks a row already used.
__device__ inline unsigned long long pivot_key(double v, int r)
{
    const unsigned long long m = (unsigned long long)__double_as_longlong(fabs(v));
    return (m & ~255ull) | (unsigned long long)(255 - r);
}

constexpr int kDP = 16;  // column panel of the diagonal-block inverse

typedef double gjd4 __attribute__((ext_vector_type(4)));

// Inverse of the kb x kb diagonal block at (K, K) (kb <= 128, padded with the
// identity) by blocked Gauss-Jordan elimination with partial pivoting inside
// the block.  Pivoting is implicit: column k is eliminated with the unused row
// p_k of largest magnitude and no rows move.  The elimination runs in place:
// once column k is eliminated its slot holds column p_k of the growing
// inverse X, so at the end S[i][k] = X[i][p_k] and A^-1[q][p_k] = S[p_q][k].
// Per panel of 16 columns, wave 0 eliminates the panel alone (pivot search
// by DPP max over packed keys, pivot row by lane reads), tracking the panel's
// row transformation T = I + (Z - E_P) E_P^T; then all four waves apply it to
// the other columns as one rank-16 update S += (Z - E_P) S[P, :] on the FP64
// matrix cores and store Z in the panel's slots.  S lives in MFMA
// accumulator tiles of 16 x 16: wave w holds rows 32w .. 32w + 31 (tiles
// rt = 0, 1) of every column tile ct; element r of lane (li, lk) of tile
// (rt, ct) is S[32w + 16rt + lk + 4r][16ct + li].  Dblk has leading
// dimension kNB.
__global__ __launch_bounds__(256) void k_gj_diag(int ld, int K, int kb,
                                                 const double *__restrict__ M,
                                                 double *__restrict__ Dblk, int *bad)
{
    __shared__ double Pn[kNB][kDP + 1];   // panel columns
    __shared__ double Zm[kNB][kDP + 1];   // Z - E_P
    __shared__ double Rp[kDP][kNB];       // pivot rows of the panel
    __shared__ int rstep[kNB];            // panel step that chose row i, or -1
    __shared__ int prow[kNB];             // pivot row of column k
    __shared__ int invp[kNB];             // column whose pivot row is i
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int row0 = 32 * wave + lk;  // + 16 rt + 4 r
    gjd4 S[2][8];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 8; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = row0 + 16 * rt + 4 * r, j = 16 * ct + li;
                S[rt][ct][r] = (i < kb && j < kb) ? M[(long long)(K + i) * ld + K + j]
                                                  : (i == j ? 1.0 : 0.0);
            }
    if (tid < kNB) {
        prow[tid] = -1;
        invp[tid] = -1;
    }
    bool used0 = false, used1 = false;  // wave 0: rows lane and lane + 64
    for (int pnl = 0; pnl < kNB / kDP; ++pnl) {
        // the panel's column tile to LDS
#pragma unroll
        for (int ct = 0; ct < 8; ++ct)
            if (ct == pnl)
#pragma unroll
                for (int rt = 0; rt < 2; ++rt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) Pn[row0 + 16 * rt + 4 * r][li] = S[rt][ct][r];
        __syncthreads();
        if (wave == 0) {
            double P0[kDP], P1[kDP], Z0[kDP], Z1[kDP];
#pragma unroll
            for (int c = 0; c < kDP; ++c) {
                P0[c] = Pn[lane][c];
                P1[c] = Pn[lane + 64][c];
                Z0[c] = 0.0;
                Z1[c] = 0.0;
            }
            int step0 = -1, step1 = -1;
#pragma unroll
            for (int t = 0; t < kDP; ++t) {
                const unsigned long long k0 = used0 ? 0ull : pivot_key(P0[t], lane);
                const unsigned long long k1 = used1 ? 0ull : pivot_key(P1[t], lane + 64);
                const unsigned long long kmax = wave_max_u64(umax64(k0, k1));
                const int p = 255 - (int)(kmax & 255ull);
                const int owner = p & 63;
                const bool hi = p >= 64;
                double pr[kDP], pz[kDP];
#pragma unroll
                for (int c = 0; c < kDP; ++c) {
                    if (c >= t) pr[c] = readlane_f64(hi ? P1[c] : P0[c], owner);
                    if (c < t) pz[c] = readlane_f64(hi ? Z1[c] : Z0[c], owner);
                }
                const double piv = pr[t];
                if (lane == 0 && !(fabs(piv) > 0.0)) atomicOr(bad, 1);
                const double rp = 1.0 / piv;
#pragma unroll
                for (int c = 0; c < kDP; ++c) {
                    if (c > t) pr[c] *= rp;
                    if (c < t) pz[c] *= rp;
                }
                pz[t] = rp;
                // row lane
                if (lane == p) {
                    used0 = true;
                    step0 = t;
#pragma unroll
                    for (int c = 0; c < kDP; ++c) {
                        if (c > t) P0[c] = pr[c];
                        if (c <= t) Z0[c] = pz[c];
                    }
                } else {
                    const double f = P0[t];
#pragma unroll
                    for (int c = 0; c < kDP; ++c) {
                        if (c > t) P0[c] -= f * pr[c];
                        if (c <= t) Z0[c] -= f * pz[c];
                    }
                }
                // row lane + 64
                if (lane + 64 == p) {
                    used1 = true;
                    step1 = t;
#pragma unroll
                    for (int c = 0; c < kDP; ++c) {
                        if (c > t) P1[c] = pr[c];
                        if (c <= t) Z1[c] = pz[c];
                    }
                } else {
                    const double f = P1[t];
#pragma unroll
                    for (int c = 0; c < kDP; ++c) {
                        if (c > t) P1[c] -= f * pr[c];
                        if (c <= t) Z1[c] -= f * pz[c];
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < kDP; ++c) {
                Zm[lane][c] = Z0[c] - (step0 == c ? 1.0 : 0.0);
                Zm[lane + 64][c] = Z1[c] - (step1 == c ? 1.0 : 0.0);
            }
            rstep[lane] = step0;
            rstep[lane + 64] = step1;
            if (step0 >= 0) prow[kDP * pnl + step0] = lane;
            if (step1 >= 0) prow[kDP * pnl + step1] = lane + 64;
        }
        __syncthreads();
        // pivot rows (before this panel's transformation) to LDS
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = rstep[row0 + 16 * rt + 4 * r];
                if (t >= 0)
#pragma unroll
                    for (int ct = 0; ct < 8; ++ct) Rp[t][16 * ct + li] = S[rt][ct][r];
            }
        __syncthreads();
        // S += (Z - E_P) S[P, :] outside the panel; the panel tile takes Z
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            double av[kDP / 4];
#pragma unroll
            for (int kk = 0; kk < kDP / 4; ++kk) av[kk] = Zm[32 * wave + 16 * rt + li][4 * kk + lk];
#pragma unroll
            for (int ct = 0; ct < 8; ++ct) {
                if (ct == pnl) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = row0 + 16 * rt + 4 * r;
                        S[rt][ct][r] = Zm[i][li] + (rstep[i] == li ? 1.0 : 0.0);
                    }
                } else {
#pragma unroll
                    for (int kk = 0; kk < kDP / 4; ++kk)
                        S[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                            av[kk], Rp[4 * kk + lk][16 * ct + li], S[rt][ct], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    if (tid < kNB && prow[tid] >= 0) invp[prow[tid]] = tid;
    __syncthreads();
    // S[i][c] = X[i][p_c] = A^-1[invp(i)][p_c]
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q = invp[row0 + 16 * rt + 4 * r];
#pragma unroll
            for (int ct = 0; ct < 8; ++ct) {
                const int col = prow[16 * ct + li];
                if (q >= 0 && q < kb && col >= 0 && col < kb) Dblk[q * kNB + col] = S[rt][ct][r];
            }
        }
    for (int idx = tid; idx < kNB * kNB; idx += 256) {
        const int r = idx / kNB, c = idx % kNB;
        if (r >= kb || c >= kb) Dblk[idx] = 0.0;
    }
}

// B[r][c] = A[r][c] for r, c < kb (B with ld ldb)
__global__ __launch_bounds__(kThreads) void k_copy_block(int kb, const double *__restrict__ A,
                                                         int lda, double *__restrict__ B,
                                                         int ldb)
{
    long long q = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (q >= (long long)kb * kb) return;
    const int r = (int)(q / kb), c = (int)(q % kb);
    B[(long long)r * ldb + c] = A[(long long)r * lda + c];
}

// C = alpha * A B + beta * C (row-major, FP64) on the matrix cores.  A
// work-group owns a TM x TN tile of C, its WM x WN waves a (TM/WM) x (TN/WN)
// block each, made of 16x16 v_mfma_f64_16x16x4 blocks.  A and B are staged
// through LDS in k-chunks of 16, double buffered: the next chunk is fetched
// into registers while the current one is multiplied.
// Lane layout of the 16x16x4 FP64 MFMA: A[i][k] in lane i + 16k, B[k][j] in
// lane j + 16k, D[i][j] in lane j + 16(i%4), element i/4 (the output rows of
// one lane are interleaved by 4, unlike the FP32 variant).
typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int kGK = 16;

// Tile (ti, tj) of work-group `wg` (1-D grid) so that each XCD gets a compact
// region: the grid's work-groups go round-robin to the 8 XCDs, so XCD x runs
// a contiguous segment of a column-band order (bands of ceil(Tx/8) tile
// columns, row-major inside a band), and the A row-blocks and B column-blocks
// its concurrent tiles share stay in its L2.
__device__ inline void xcd_tile(int wg, int Ty, int Tx, int &ti, int &tj)
{
    constexpr int kXcd = 8;
    const int N = Ty * Tx;
    const int q = N / kXcd, r = N % kXcd;
    const int x = wg % kXcd, k = wg / kXcd;
    const int g = x * q + (x < r ? x : r) + k;  // position in the band order
    const int W = (Tx + kXcd - 1) / kXcd;
    const int band = g / (W * Ty);
    const int c0 = band * W;
    const int w = Tx - c0 < W ? Tx - c0 : W;
    const int gl = g - band * W * Ty;
    ti = gl / w;
    tj = c0 + gl % w;
}

// One TM x TN tile at (i0, j0).  FULL: the tile lies inside C and Kd is a
// multiple of the k-chunk, so no load or store needs a bounds check (the
// loads of a chunk and the C reads of the epilogue then issue back to back).
template <int TM, int TN, int WM, int WN, bool FULL>
__device__ inline void dgemm_body(int i0, int j0, int Mr, int Nc, int Kd,
                                  const double *__restrict__ A, int lda,
                                  const double *__restrict__ B, int ldb, double *__restrict__ C,
                                  int ldc, double alpha, double beta,
                                  double (*__restrict__ As)[TM][kGK + 1],
                                  double (*__restrict__ Bs)[kGK][TN + 1])
{
    constexpr int T = 64 * WM * WN;         // threads
    constexpr int FM = TM / WM / 16, FN = TN / WN / 16;
    constexpr int AR = T / kGK;             // A rows fetched per pass
    constexpr int BK = T / TN;              // B k-rows fetched per pass
    static_assert(TM % AR == 0 && kGK % BK == 0, "fetch mapping");
    constexpr int AU = TM / AR, BU = kGK / BK;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wr = (wave / WN) * (TM / WM), wc = (wave % WN) * (TN / WN);
    const int li = lane & 15, lk = lane >> 4;
    dbl4 acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
    // per-thread fetch slots: A rows r0 + AR u (column ac), B k-rows bk0 + BK u
    // (column bj)
    const int ac = tid % kGK, r0 = tid / kGK, bk0 = tid / TN;
    const int bj = j0 + tid % TN;
    const bool bj_ok = bj < Nc;
    const double *pa = A + (long long)(i0 + r0) * lda + ac;
    const double *pb = B + (bj_ok ? bj : 0);
    const int arows = Mr - i0 - r0;  // row r0 + AR u valid iff AR u < arows
    double ra[AU], rb[BU];
    auto fetch = [&](int k0) {
        if (FULL) {
#pragma unroll
            for (int u = 0; u < AU; ++u) ra[u] = pa[(long long)(AR * u) * lda + k0];
#pragma unroll
            for (int u = 0; u < BU; ++u) rb[u] = pb[(long long)(k0 + bk0 + BK * u) * ldb];
            return;
        }
        const bool ak_ok = k0 + ac < Kd;
#pragma unroll
        for (int u = 0; u < AU; ++u)
            ra[u] = (AR * u < arows && ak_ok) ? pa[(long long)(AR * u) * lda + k0] : 0.0;
#pragma unroll
        for (int u = 0; u < BU; ++u) {
            const int kk = k0 + bk0 + BK * u;
            rb[u] = (bj_ok && kk < Kd) ? pb[(long long)kk * ldb] : 0.0;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int u = 0; u < AU; ++u) As[buf][r0 + AR * u][ac] = ra[u];
#pragma unroll
        for (int u = 0; u < BU; ++u) Bs[buf][bk0 + BK * u][tid % TN] = rb[u];
    };
    const int nchunk = (Kd + kGK - 1) / kGK;
    fetch(0);
    stash(0);
    __syncthreads();
    for (int ch = 0; ch < nchunk; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nchunk) fetch((ch + 1) * kGK);
#pragma unroll
        for (int kk = 0; kk < kGK; kk += 4) {
            double av[FM], bv[FN];
#pragma unroll
            for (int a = 0; a < FM; ++a) av[a] = As[buf][wr + a * 16 + li][kk + lk];
#pragma unroll
            for (int b = 0; b < FN; ++b) bv[b] = Bs[buf][kk + lk][wc + b * 16 + li];
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
                for (int b = 0; b < FN; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        if (ch + 1 < nchunk) stash(buf ^ 1);
        __syncthreads();
    }
    if (FULL) {
        // the C reads of one 16-row block go out together, then their writes
        constexpr int FH = 1;
#pragma unroll
        for (int h = 0; h < FM; h += FH) {
            double cv[FH][4][FN];
            if (beta != 0.0) {
#pragma unroll
                for (int a = 0; a < FH; ++a)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int b = 0; b < FN; ++b)
                            cv[a][r][b] = C[(long long)(i0 + wr + (h + a) * 16 + lk + 4 * r) * ldc +
                                            j0 + wc + b * 16 + li];
            }
#pragma unroll
            for (int a = 0; a < FH; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int b = 0; b < FN; ++b) {
                        const double v = alpha * acc[h + a][b][r];
                        C[(long long)(i0 + wr + (h + a) * 16 + lk + 4 * r) * ldc + j0 + wc + b * 16 +
                          li] = (beta != 0.0) ? v + beta * cv[a][r][b] : v;
                    }
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + wr + a * 16 + lk + 4 * r;
            if (i >= Mr) continue;
            double *crow = C + (long long)i * ldc + j0 + wc + li;
#pragma unroll
            for (int b = 0; b < FN; ++b) {
                if (j0 + wc + b * 16 + li >= Nc) continue;
                double *c = crow + b * 16;
                const double v = alpha * acc[a][b][r];
                *c = (beta != 0.0) ? v + beta * *c : v;
            }
        }
}


template <int TM, int TN, int WM, int WN>
__device__ inline void dgemm_tile(int Mr, int Nc, int Kd, const double *__restrict__ A, int lda,
                                  const double *__restrict__ B, int ldb, double *__restrict__ C,
                                  int ldc, double alpha, double beta)
{
    __shared__ double As[2][TM][kGK + 1];
    __shared__ double Bs[2][kGK][TN + 1];
    int ti, tj;
    xcd_tile(blockIdx.x, (Mr + TM - 1) / TM, (Nc + TN - 1) / TN, ti, tj);
    const int i0 = ti * TM, j0 = tj * TN;
    if (i0 + TM <= Mr && j0 + TN <= Nc && Kd % kGK == 0)
        dgemm_body<TM, TN, WM, WN, true>(i0, j0, Mr, Nc, Kd, A, lda, B, ldb, C, ldc, alpha, beta,
                                         As, Bs);
    else
        dgemm_body<TM, TN, WM, WN, false>(i0, j0, Mr, Nc, Kd, A, lda, B, ldb, C, ldc, alpha, beta,
                                          As, Bs);
}

// Large products: 128x128 tiles, 8 waves of 64x32; two work-groups per CU (68
// KB of LDS each, <= 128 registers per lane) so one work-group's C
// read-modify-write overlaps the other's matrix-core work.
constexpr int kGT = 128, kGThreads = 512;
__global__ __launch_bounds__(kGThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_dgemm(
    int Mr, int Nc, int Kd, const double *__restrict__ A, int lda, const double *__restrict__ B,
    int ldb, double *__restrict__ C, int ldc, double alpha, double beta)
{
    dgemm_tile<kGT, kGT, 2, 4>(Mr, Nc, Kd, A, lda, B, ldb, C, ldc, alpha, beta);
}

// Small products (too few 128x128 tiles to fill the chip): 64x64 tiles, 4
// waves of 32x32, so four times as many work-groups share the work.
constexpr int kGTs = 64, kGThreadsS = 256;
constexpr long long kDgemmBigTiles = 512;  // two 128x128 tiles per compute unit
__global__ __launch_bounds__(kGThreadsS) void k_dgemm_s(int Mr, int Nc, int Kd,
                                                      const double *__restrict__ A, int lda,
                                                      const double *__restrict__ B, int ldb,
                                                      double *__restrict__ C, int ldc,
                                                      double alpha, double beta)
{
    dgemm_tile<kGTs, kGTs, 2, 2>(Mr, Nc, Kd, A, lda, B, ldb, C, ldc, alpha, beta);
}

}  // namespace

// ===========================================================================
// launchers
// ===========================================================================
#define MSP_SWITCH_B(b, CALL)              \
    switch (b) {                           \
    case 1: { constexpr int B = 1; CALL; } break; \
    case 2: { constexpr int B = 2; CALL; } break; \
    case 3: { constexpr int B = 3; CALL; } break; \
    case 4: { constexpr int B = 4; CALL; } break; \
    case 5: { constexpr int B = 5; CALL; } break; \
    case 6: { constexpr int B = 6; CALL; } break; \
    case 7: { constexpr int B = 7; CALL; } break; \
    case 8: { constexpr int B = 8; CALL; } break; \
    default: return hipErrorInvalidValue;  \
    }

hipError_t launch_ingest_bsr(int b, int p, long long slot_lanes, const int *src,
                             const double *vals, double *dst, float *dst32_pcol, int *bad,
                             hipStream_t st)
{
    if (slot_lanes <= 0) return hipSuccess;
    MSP_SWITCH_B(b, (k_ingest<B><<<blocks_for(slot_lanes), kThreads, 0, st>>>(
                        p, slot_lanes, src, vals, dst, dst32_pcol, bad)));
    return hipGetLastError();
}

hipError_t launch_gather_blocks(int b, long long slot_lanes, const int *src, const double *blocks,
                                double *dst64, float *dst32, hipStream_t st)
{
    if (slot_lanes <= 0) return hipSuccess;
    MSP_SWITCH_B(b, (k_gather_blocks<B><<<blocks_for(slot_lanes), kThreads, 0, st>>>(
                        slot_lanes, src, blocks, dst64, dst32)));
    return hipGetLastError();
}

hipError_t launch_level_fill(bool fp32, int nslices, const int4 *slices, const int *rp,
                             const int *ci, const double *val, const int *perm, const int *iperm,
                             int *col, int *src, void *vals, void *diag, hipStream_t st)
{
    if (nslices <= 0) return hipSuccess;
    const unsigned nb = blocks_for((long long)nslices * 64);
    if (fp32)
        k_level_fill<float><<<nb, kThreads, 0, st>>>(nslices, slices, rp, ci, val, perm, iperm,
                                                     col, src, (float *)vals, (float *)diag);
    else
        k_level_fill<double><<<nb, kThreads, 0, st>>>(nslices, slices, rp, ci, val, perm, iperm,
                                                      col, src, (double *)vals, (double *)diag);
    return hipGetLastError();
}

hipError_t launch_tri_fill(int nslices, const int4 *slices, const int *rows, const int *rp,
                           const int *ci, const int *pos, bool lower, int *col, int *src,
                           hipStream_t st)
{
    if (nslices <= 0) return hipSuccess;
    k_tri_fill<<<blocks_for((long long)nslices * 64), kThreads, 0, st>>>(
        nslices, slices, rows, rp, ci, pos, lower ? 1 : 0, col, src);
    return hipGetLastError();
}

hipError_t launch_diff_i32(const int *a, const int *b, long long n, int *bad, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    k_diff_i32<<<blocks_for(n), kThreads, 0, st>>>(a, b, n, bad);
    return hipGetLastError();
}

hipError_t launch_check_finite(const double *x, long long n, int *bad, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    k_check_finite<<<blocks_for(n), kThreads, 0, st>>>(x, n, bad);
    return hipGetLastError();
}

hipError_t launch_round_f32(const double *x, float *y, long long n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    k_round_f32<<<blocks_for(n), kThreads, 0, st>>>(x, y, n);
    return hipGetLastError();
}

hipError_t launch_decouple(int b, int p, int n, const int *rp, const int *diag_pos,
                           const double *vals, double *omega, double *ap, int *bad,
                           hipStream_t st)
{
    MSP_SWITCH_B(b, (k_decouple<B><<<blocks_for(n), kThreads, 0, st>>>(p, n, rp, diag_pos, vals,
                                                                      omega, ap, bad)));
    return hipGetLastError();
}

hipError_t launch_bilu_factor_level(int b, const BiluTasks &t, double *F, double *Dinv, int *bad,
                                    hipStream_t st)
{
    if (t.nrows <= 0) return hipSuccess;
    MSP_SWITCH_B(b, (k_bilu_factor<B><<<blocks_for(t.nrows, 64), 64, 0, st>>>(t, F, Dinv, bad)));
    return hipGetLastError();
}

hipError_t launch_spmv(int b, const SellView &A, const double *val, const double *x,
                       const double *sub, double *y, hipStream_t st)
{
    unsigned nb = slice_blocks(A);
    if (!nb) return hipSuccess;
    MSP_SWITCH_B(b, (k_spmv<B><<<nb, kThreads, 0, st>>>(A.slices, A.col, A.slice_begin,
                                                        A.slice_end, val, x, sub, y)));
    return hipGetLastError();
}

__global__ void k_set_io(ApplyIo *io, const double *v, double *z)
{
    io->v = v;
    io->z = z;
}

hipError_t launch_set_io(ApplyIo *io, const double *v, double *z, hipStream_t st)
{
    k_set_io<<<1, 1, 0, st>>>(io, v, z);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_decouple_restrict(int b, int n, const int *iperm0, const double *omega,
                                    const double *v, const ApplyIo *io, T *g, hipStream_t st)
{
    MSP_SWITCH_B(b, (k_decouple_restrict<B, T><<<blocks_for(n), kThreads, 0, st>>>(
                        n, iperm0, omega, v, io, g)));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gs_first(const SellView &, int npos, const T *diag, const T *f, T *x,
                           int p0, int p1, hipStream_t st)
{
    k_gs_first<T><<<blocks_for(npos), kThreads, 0, st>>>(npos, p0, p1, diag, f, x);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gs_color(const SellView &seg, const T *val, const T *diag, const T *f, T *x,
                           hipStream_t st)
{
    unsigned nb = slice_blocks(seg);
    if (!nb) return hipSuccess;
    if (seg.lanes == kRowLanes) {
        const int ns = seg.slice_end - seg.slice_begin;
        k_gs_color_lanes<T, kRowLanes><<<(ns * kRowLanes + 3) / 4, kThreads, 0, st>>>(
            seg.slices, seg.col, seg.slice_begin, seg.slice_end, val, diag, f, x);
    } else {
        k_gs_color<T><<<nb, kThreads, 0, st>>>(seg.slices, seg.col, seg.slice_begin,
                                               seg.slice_end, val, diag, f, x);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_residual(const SellView &all, const T *val, const T *diag, const T *f,
                           const T *x, T *r, hipStream_t st)
{
    unsigned nb = slice_blocks(all);
    if (!nb) return hipSuccess;
    if (all.lanes == kRowLanes) {
        const int ns = all.slice_end - all.slice_begin;
        k_residual_lanes<T, kRowLanes><<<(ns * kRowLanes + 3) / 4, kThreads, 0, st>>>(
            all.slices, all.col, all.slice_begin, all.slice_end, val, diag, f, x, r);
    } else {
        k_residual<T><<<nb, kThreads, 0, st>>>(all.slices, all.col, all.slice_begin,
                                               all.slice_end, val, diag, f, x, r);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(int nc, const int *mem_ptr, const int *mem, const T *r, T *fc,
                           hipStream_t st)
{
    k_restrict<T><<<blocks_for(nc), kThreads, 0, st>>>(nc, mem_ptr, mem, r, fc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_first(int nc, const int *mem_ptr, const int *mem, const T *r, T *fc,
                                 int p0, int p1, const T *diag_c, T *xc, hipStream_t st)
{
    k_restrict_first<T><<<blocks_for(nc), kThreads, 0, st>>>(nc, mem_ptr, mem, r, fc, p0, p1,
                                                              diag_c, xc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(int n, const int *agg_pos, const T *xc, T *x, hipStream_t st)
{
    k_prolong<T><<<blocks_for(n), kThreads, 0, st>>>(n, agg_pos, xc, x);
    return hipGetLastError();
}

hipError_t launch_link(int n, int nc, const int *natc, const int *mptr_nat, const int *mem_nat,
                       const int *cperm, const int *mptr_pos, int *agg_pos, int *mem,
                       hipStream_t st)
{
    const int m = std::max(n, nc);
    if (m <= 0) return hipSuccess;
    k_link<<<blocks_for(m), kThreads, 0, st>>>(n, nc, natc, mptr_nat, mem_nat, cperm, mptr_pos,
                                               agg_pos, mem);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_jacobi_first(int n, T w, const T *diag, const T *f, T *x, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    k_jacobi_first<T><<<blocks_for(n), kThreads, 0, st>>>(n, w, diag, f, x);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_jacobi_update(int n, T w, const T *diag, const T *r, T *x, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    k_jacobi_update<T><<<blocks_for(n), kThreads, 0, st>>>(n, w, diag, r, x);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_zero(int n, T *x, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    k_zero<T><<<blocks_for(n), kThreads, 0, st>>>(n, x);
    return hipGetLastError();
}

hipError_t launch_block_inverse(int b, int n, const int *diag_pos, const double *vals,
                                double *Dinv, int *bad, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    MSP_SWITCH_B(b, (k_block_inverse<B><<<blocks_for(n), kThreads, 0, st>>>(n, diag_pos, vals,
                                                                           Dinv, bad)));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_block_jacobi(int b, int n, const T *Dinv, T *y, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    MSP_SWITCH_B(b, (k_block_jacobi<B, T><<<blocks_for(n), kThreads, 0, st>>>(n, Dinv, y)));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_solve(int n, int ld, int P, const double *Y, const double *W,
                               const T *f, double *t, T *x, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    const unsigned g = (unsigned)((n + 3) / 4);
    k_coarse_tri<true, T, double><<<g, kThreads, 0, st>>>(n, ld, P, Y, f, t);
    k_coarse_tri<false, double, T><<<g, kThreads, 0, st>>>(n, ld, P, W, t, x);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_unpermute(int n, const int *perm0, const T *epos, T *enat, hipStream_t st)
{
    k_unpermute<T><<<blocks_for(n), kThreads, 0, st>>>(n, perm0, epos, enat);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pcol_residual(int b, int p, const SellView &A, const double *val64,
                                const float *pcol32, const double *v, const ApplyIo *io,
                                const T *e, const int *rperm, T *r, hipStream_t st)
{
    unsigned nb = slice_blocks(A);
    if (!nb) return hipSuccess;
    if (pcol32) {
        MSP_SWITCH_B(b, (k_pcol_residual<B, T, true><<<nb, kThreads, 0, st>>>(
                            p, A.slices, A.col, A.slice_begin, A.slice_end, val64, pcol32, v, io,
                            e, rperm, r)));
    } else {
        MSP_SWITCH_B(b, (k_pcol_residual<B, T, false><<<nb, kThreads, 0, st>>>(
                            p, A.slices, A.col, A.slice_begin, A.slice_end, val64, pcol32, v, io,
                            e, rperm, r)));
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_bilu_fwd(int b, const SellView &L, const int *rows, const T *Lval, T *y,
                           hipStream_t st)
{
    unsigned nb = slice_blocks(L);
    if (!nb) return hipSuccess;
    MSP_SWITCH_B(b, (k_bilu_fwd<B, T><<<nb, kThreads, 0, st>>>(L.slices, L.col, L.slice_begin,
                                                               L.slice_end, rows, Lval, y)));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_bilu_bwd(int b, const SellView &U, const int *rows, const T *Uval,
                           const T *Dval, T *z, hipStream_t st)
{
    unsigned nb = slice_blocks(U);
    if (!nb) return hipSuccess;
    MSP_SWITCH_B(b, (k_bilu_bwd<B, T><<<nb, kThreads, 0, st>>>(U.slices, U.col, U.slice_begin,
                                                               U.slice_end, rows, Uval, Dval,
                                                               z)));
    return hipGetLastError();
}

// dst_T[pos[c]*b + k] = (T)src[c*b + k] (src != nullptr), or
// dst64[c*b + k] = (double)srcT[pos[c]*b + k]
template <typename T>
__global__ __launch_bounds__(kThreads) void k_perm_blocks(int n, int b, const int *__restrict__ pos,
                                                          const double *__restrict__ src,
                                                          T *__restrict__ dst, double *__restrict__ dst64,
                                                          const T *__restrict__ srcT)
{
    const long long q = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (q >= (long long)n * b) return;
    const long long c = q / b, k = q % b, qp = (long long)pos[c] * b + k;
    if (src)
        dst[qp] = (T)src[q];
    else
        dst64[q] = (double)srcT[qp];
}

template <typename T>
hipError_t launch_perm_blocks(int n, int b, const int *pos, const double *src, T *dst,
                              double *dst64, const T *srcT, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    k_perm_blocks<T><<<blocks_for((long long)n * b), kThreads, 0, st>>>(n, b, pos, src, dst, dst64,
                                                                       srcT);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_finish(int b, int p, int n, const T *zz, const int *zperm, const T *e,
                         const double *w1, double *z, const ApplyIo *io, hipStream_t st)
{
    MSP_SWITCH_B(b, (k_finish<B, T><<<blocks_for((long long)n * B), kThreads, 0, st>>>(
                        p, n, zz, zperm, e, w1, z, io)));
    return hipGetLastError();
}

hipError_t launch_decouple_n(int b, int p, int n, const int *rp, const int *ci,
                             const int *diag_pos, const double *vals, double *Dn, double *Ann,
                             int *bad, hipStream_t st)
{
    if (b < 2 || n <= 0) return hipSuccess;
    MSP_SWITCH_B(b, (k_decouple_n<B><<<blocks_for(n), kThreads, 0, st>>>(n, p, rp, ci, diag_pos,
                                                                        vals, Dn, Ann, bad)));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_n_rhs(int b, int n, const T *Dn, const double *v, T *gN, hipStream_t st)
{
    if (b < 2 || n <= 0) return hipSuccess;
    MSP_SWITCH_B(b, (k_n_rhs<B, T><<<blocks_for(n), kThreads, 0, st>>>(n, Dn, v, gN)));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_bgs_group(int b, int ncell, const int *cells, const int *rp, const int *ci,
                            const T *Ann, const T *gN, T *y, hipStream_t st)
{
    if (b < 2 || ncell <= 0) return hipSuccess;
    MSP_SWITCH_B(b, (k_bgs_group<B, T><<<blocks_for(ncell), kThreads, 0, st>>>(ncell, cells, rp,
                                                                              ci, Ann, gN, y)));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_expand_n(int b, int p, int n, const T *y, double *w1, hipStream_t st)
{
    if (b < 2 || n <= 0) return hipSuccess;
    MSP_SWITCH_B(b, (k_expand_n<B, T><<<blocks_for((long long)n * B), kThreads, 0, st>>>(n, p, y,
                                                                                        w1)));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_to_double(long long n, const T *x, double *y, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    k_to_double<T><<<blocks_for(n), kThreads, 0, st>>>(n, x, y);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_from_double(long long n, const double *x, T *y, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    k_from_double<T><<<blocks_for(n), kThreads, 0, st>>>(n, x, y);
    return hipGetLastError();
}

#define MSP_INSTANTIATE(T)                                                                     \
    template hipError_t launch_decouple_restrict<T>(int, int, const int *, const double *,     \
                                                    const double *, const ApplyIo *, T *,      \
                                                    hipStream_t);                              \
    template hipError_t launch_gs_first<T>(const SellView &, int, const T *, const T *, T *,   \
                                           int, int, hipStream_t);                             \
    template hipError_t launch_gs_color<T>(const SellView &, const T *, const T *, const T *,  \
                                           T *, hipStream_t);                                  \
    template hipError_t launch_residual<T>(const SellView &, const T *, const T *, const T *,  \
                                           const T *, T *, hipStream_t);                       \
    template hipError_t launch_restrict<T>(int, const int *, const int *, const T *, T *,      \
                                           hipStream_t);                                       \
    template hipError_t launch_restrict_first<T>(int, const int *, const int *, const T *, T *, \
                                                 int, int, const T *, T *, hipStream_t);       \
    template hipError_t launch_prolong<T>(int, const int *, const T *, T *, hipStream_t);      \
    template hipError_t launch_jacobi_first<T>(int, T, const T *, const T *, T *, hipStream_t); \
    template hipError_t launch_jacobi_update<T>(int, T, const T *, const T *, T *, hipStream_t); \
    template hipError_t launch_zero<T>(int, T *, hipStream_t);                                 \
    template hipError_t launch_block_jacobi<T>(int, int, const T *, T *, hipStream_t);         \
    template hipError_t launch_coarse_solve<T>(int, int, int, const double *, const double *, \
                                               const T *, double *, T *, hipStream_t);         \
    template hipError_t launch_unpermute<T>(int, const int *, const T *, T *, hipStream_t);    \
    template hipError_t launch_pcol_residual<T>(int, int, const SellView &, const double *,    \
                                                const float *, const double *,                 \
                                                const ApplyIo *, const T *, const int *, T *,  \
                                                hipStream_t);                                  \
    template hipError_t launch_bilu_fwd<T>(int, const SellView &, const int *, const T *, T *, \
                                           hipStream_t);                                       \
    template hipError_t launch_bilu_bwd<T>(int, const SellView &, const int *, const T *,      \
                                           const T *, T *, hipStream_t);                       \
    template hipError_t launch_finish<T>(int, int, int, const T *, const int *, const T *,     \
                                         const double *, double *, const ApplyIo *,            \
                                         hipStream_t);                                         \
    template hipError_t launch_n_rhs<T>(int, int, const T *, const double *, T *, hipStream_t); \
    template hipError_t launch_bgs_group<T>(int, int, const int *, const int *, const int *,   \
                                            const T *, const T *, T *, hipStream_t);           \
    template hipError_t launch_expand_n<T>(int, int, int, const T *, double *, hipStream_t);   \
    template hipError_t launch_to_double<T>(long long, const T *, double *, hipStream_t);      \
    template hipError_t launch_from_double<T>(long long, const double *, T *, hipStream_t);    \
    template hipError_t launch_perm_blocks<T>(int, int, const int *, const double *, T *,      \
                                              double *, const T *, hipStream_t);

MSP_INSTANTIATE(float)
MSP_INSTANTIATE(double)

hipError_t launch_dot_multi(long long N, int nv, const double *V, long long ldv, const double *w,
                            double *partial, hipStream_t st)
{
    k_dot_multi<<<kDotBlocks, kThreads, 0, st>>>(N, nv, V, ldv, w, partial);
    return hipGetLastError();
}

hipError_t launch_reduce_partials(int nv, const double *partial, double *out, int accumulate,
                                  hipStream_t st)
{
    k_reduce_partials<<<1, kReduceThreads, 0, st>>>(nv, kDotBlocks, partial, out, accumulate);
    return hipGetLastError();
}

static unsigned stream_blocks(long long N)
{
    long long b = (N + kThreads - 1) / kThreads;
    if (b > 4096) b = 4096;
    return (unsigned)(b < 1 ? 1 : b);
}

hipError_t launch_axpy_multi(long long N, int nv, const double *V, long long ldv,
                             const double *h, double *w, hipStream_t st)
{
    k_axpy_multi<<<stream_blocks(N), kThreads, 0, st>>>(N, nv, V, ldv, h, w);
    return hipGetLastError();
}

template <int MODE>
static hipError_t gs_pass(long long N, int nv, const double *V, long long ldv, const double *h,
                          double *w, double *partial, hipStream_t st)
{
    switch (nv) {
#define MSP_GS_CASE(K)                                                                    \
    case K:                                                                               \
        k_gs_pass<K, MODE><<<kDotBlocks, kThreads, 0, st>>>(N, V, ldv, h, w, partial);    \
        break;
        MSP_GS_CASE(1) MSP_GS_CASE(2) MSP_GS_CASE(3) MSP_GS_CASE(4) MSP_GS_CASE(5)
        MSP_GS_CASE(6) MSP_GS_CASE(7) MSP_GS_CASE(8) MSP_GS_CASE(9) MSP_GS_CASE(10)
        MSP_GS_CASE(11) MSP_GS_CASE(12) MSP_GS_CASE(13) MSP_GS_CASE(14) MSP_GS_CASE(15)
        MSP_GS_CASE(16) MSP_GS_CASE(17) MSP_GS_CASE(18) MSP_GS_CASE(19) MSP_GS_CASE(20)
        MSP_GS_CASE(21) MSP_GS_CASE(22) MSP_GS_CASE(23) MSP_GS_CASE(24) MSP_GS_CASE(25)
        MSP_GS_CASE(26) MSP_GS_CASE(27) MSP_GS_CASE(28) MSP_GS_CASE(29) MSP_GS_CASE(30)
        MSP_GS_CASE(31) MSP_GS_CASE(32)
#undef MSP_GS_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_gs_pass(int mode, long long N, int nv, const double *V, long long ldv,
                          const double *h, double *w, double *partial, hipStream_t st)
{
    if (nv < 1 || nv > kFusedGsMax) return hipErrorInvalidValue;
    if (mode == 0) return gs_pass<0>(N, nv, V, ldv, h, w, partial, st);
    if (mode == 1) return gs_pass<1>(N, nv, V, ldv, h, w, partial, st);
    if (mode == 2) return gs_pass<2>(N, nv, V, ldv, h, w, partial, st);
    return hipErrorInvalidValue;
}

hipError_t launch_scale(long long N, const double *x, double s, double *y, hipStream_t st)
{
    k_scale<<<stream_blocks(N), kThreads, 0, st>>>(N, x, s, y);
    return hipGetLastError();
}

hipError_t launch_update_x(long long N, int k, const double *Z, long long ldz, const double *y,
                           double *x, hipStream_t st)
{
    k_update_x<<<stream_blocks(N), kThreads, 0, st>>>(N, k, Z, ldz, y, x);
    return hipGetLastError();
}

hipError_t launch_fill(long long N, double v, double *x, hipStream_t st)
{
    if (N <= 0) return hipSuccess;
    k_fill<<<stream_blocks(N), kThreads, 0, st>>>(N, v, x);
    return hipGetLastError();
}

hipError_t launch_dense_scatter(int n, int ld, const int *rp, const int *ci, const double *val,
                                double *M, hipStream_t st)
{
    k_dense_scatter<<<blocks_for(n), kThreads, 0, st>>>(n, ld, rp, ci, val, M);
    return hipGetLastError();
}


hipError_t launch_dgemm(int Mr, int Nc, int Kd, const double *A, int lda, const double *B, int ldb,
                        double *C, int ldc, double alpha, double beta, hipStream_t st)
{
    if (Mr <= 0 || Nc <= 0) return hipSuccess;
    const long long big_tiles = (long long)((Nc + kGT - 1) / kGT) * ((Mr + kGT - 1) / kGT);
    if (big_tiles >= kDgemmBigTiles) {
        k_dgemm<<<(unsigned)big_tiles, kGThreads, 0, st>>>(Mr, Nc, Kd, A, lda, B, ldb, C, ldc,
                                                          alpha, beta);
    } else {
        const long long tiles =
            (long long)((Nc + kGTs - 1) / kGTs) * ((Mr + kGTs - 1) / kGTs);
        k_dgemm_s<<<(unsigned)tiles, kGThreadsS, 0, st>>>(Mr, Nc, Kd, A, lda, B, ldb, C, ldc,
                                                         alpha, beta);
    }
    return hipGetLastError();
}


namespace {

// L rows of LU step s: [K + kb, lu_end(n, s, ends)), where ends[s] bounds the
// window of step s; the window always covers the next diagonal block (the
// pivot stream forms it from these rows).
int lu_end(int n, int s, const int *ends)
{
    const int K = s * kLuBlock;
    const int cover = n - K < 2 * kLuBlock ? n : K + 2 * kLuBlock;
    const int e = ends ? std::max(ends[s], cover) : n;
    return std::min(e, n);
}

}  // namespace

// M[r][0 .. kb) = 0 for r < nr
__global__ __launch_bounds__(kThreads) void k_zero_rect(int nr, int kb, int ld,
                                                        double *__restrict__ M)
{
    long long q = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (q >= (long long)nr * kb) return;
    M[(q / kb) * ld + q % kb] = 0.0;
}

// Y[i][i] = 1 for i < n
__global__ __launch_bounds__(kThreads) void k_unit_diag(int n, int ld, double *__restrict__ Y)
{
    int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) Y[(long long)i * ld + i] = 1.0;
}

// Rows [r0, r1) of block column s of L (Ls, ld P) into the row-block
// layout: row r of row block I = I0 + b goes to dst + off[b] + (r - I P) ld[b].
struct LrowMap {
    static constexpr int kMax = 16;
    long long off[kMax];
    int ld[kMax];
};
__global__ __launch_bounds__(kThreads) void k_lrow_scatter(int r0, int r1, int I0, int P,
                                                           const double *__restrict__ Ls,
                                                           const LrowMap map,
                                                           double *__restrict__ dst)
{
    long long q = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (q >= (long long)(r1 - r0) * P) return;
    const int r = r0 + (int)(q / P), t = (int)(q % P);
    const int b = r / P - I0;
    dst[map.off[b] + (long long)(r % P) * map.ld[b] + t] = Ls[q];
}

namespace {

// Row-block layout of L: row block I (1 <= I < steps) holds its blocks
// L(I, f_I .. I-1) side by side, P rows by (I - f_I) P columns, where f_I is
// the first block step whose L rows reach row block I.
struct LrowLayout {
    std::vector<int> f;
    std::vector<long long> off;  // steps + 1 entries
};

LrowLayout lrow_layout(int n, const int *rows_end)
{
    constexpr int P = kLuBlock;
    const int steps = (n + P - 1) / P;
    LrowLayout L;
    L.f.assign(steps, 0);
    L.off.assign(steps + 1, 0);
    for (int I = 1, s = 0; I < steps; ++I) {
        while (s < I - 1 && lu_end(n, s, rows_end) <= I * P) ++s;
        L.f[I] = s;
        L.off[I + 1] = L.off[I] + (long long)P * (I - s) * P;
    }
    if (steps > 0) L.off[1] = 0;
    return L;
}

size_t lband_col(int n, const int *rows_end)
{
    size_t q = 0;
    for (int K = 0, s = 0; K < n; K += kLuBlock, ++s) {
        const int r0 = std::min(K + kLuBlock, n);
        q += (size_t)(lu_end(n, s, rows_end) - r0) * kLuBlock;
    }
    return q;
}

}  // namespace

size_t dense_inverse_work(int n)
{
    return (size_t)kLuBlock * n + (size_t)2 * kLuBlock * kLuBlock;
}

size_t dense_inverse_lband(int n, const int *rows_end)
{
    const int steps = (n + kLuBlock - 1) / kLuBlock;
    return lband_col(n, rows_end) + (size_t)lrow_layout(n, rows_end).off[steps];
}


int dense_inverse_sweep_k(int n, const int *cols_end)
{
    constexpr int P = kLuBlock;
    const int steps = (n + P - 1) / P, J = steps - 1, K = J * P;
    int us = 0;
    while (us < J && lu_end(n, us, cols_end) <= K) ++us;
    return K - us * P;
}

hipError_t dense_inverse(int n, int ld, double *M, double *Y, double *lband, double *work, int *bad,
                         hipStream_t caller, const GjLookAhead *la, const int *rows_end,
                         const int *cols_end)
{
    hipError_t e;
    hipStream_t st = caller;
    if (la) {
        st = la->main;
        if ((e = hipStreamWaitEvent(st, la->ev_start, 0)) != hipSuccess) return e;
    }
    constexpr int P = kLuBlock;
    const int steps = (n + P - 1) / P;
    // the pivot blocks are inverted by one k_gj_diag each, in place of M
    static_assert(kLuBlock == kNB, "one pivot kernel per block");
    double *Tcol = work;                                // n x P
    double *Dblk[2] = {Tcol + (long long)P * n,         // P x P, two buffers
                       Tcol + (long long)P * n + (long long)P * P};
    const hipStream_t aux = la ? la->aux : st;
    // Y stream: the Y sweep in row form, row block I as soon as LU step I-1
    // has produced the last block of L's row block I
    const hipStream_t ys = la ? la->third : st;
    std::vector<long long> loff(steps + 1, 0);
    for (int s = 0; s < steps; ++s)
        loff[s + 1] = loff[s] + (long long)(lu_end(n, s, rows_end) - std::min((s + 1) * P, n)) * P;
    const LrowLayout lr = lrow_layout(n, rows_end);
    double *lrow = lband + loff[steps];
    if (la && (e = hipStreamWaitEvent(ys, la->ev_start, 0)) != hipSuccess) return e;
    if ((e = launch_fill((long long)n * ld, 0.0, Y, ys)) != hipSuccess) return e;
    k_unit_diag<<<blocks_for(n), kThreads, 0, ys>>>(n, ld, Y);
    if ((e = launch_fill(lr.off[steps], 0.0, lrow, ys)) != hipSuccess) return e;
    // after LU step s: its L rows into the row-block layout, then Y's row
    // block s + 1: Y(I, :I) = -L(I, f_I:I) Y(f_I:I, :I)
    auto y_row = [&](int s) -> hipError_t {
        const int K = s * P, r0 = K + P, r1 = lu_end(n, s, rows_end);
        for (int I0 = r0 / P; I0 * P < r1; I0 += LrowMap::kMax) {
            LrowMap map;
            for (int b = 0; b < LrowMap::kMax; ++b) {
                const int I = std::min(I0 + b, steps - 1);
                map.ld[b] = (I - lr.f[I]) * P;
                map.off[b] = lr.off[I] + (long long)(s - lr.f[I]) * P;
            }
            const int a0 = std::max(r0, I0 * P), a1 = std::min(r1, (I0 + LrowMap::kMax) * P);
            k_lrow_scatter<<<blocks_for((long long)(a1 - a0) * P), kThreads, 0, ys>>>(
                a0, a1, I0, P, lband + loff[s] + (long long)(a0 - r0) * P, map, lrow);
        }
        const int I = s + 1, kbI = std::min(P, n - I * P), w = (I - lr.f[I]) * P;
        return launch_dgemm(kbI, I * P, w, lrow + lr.off[I], w,
                            Y + (long long)lr.f[I] * P * ld, ld, Y + (long long)I * P * ld, ld,
                            -1.0, 0.0, ys);
    };
    // block 0: inverted on the pivot stream once the matrix is scattered
    if (la && (e = hipStreamWaitEvent(aux, la->ev_start, 0)) != hipSuccess) return e;
    k_gj_diag<<<1, 256, 0, aux>>>(ld, 0, std::min(n, P), M, Dblk[0], bad);
    // W = U^-1 in place, column block J on the Y stream (once LU step J has
    // put D_J on the diagonal and every earlier step has finished block
    // column J of U): W(:J, J) = -W(:J, lo:J) U(lo:J, J) D_J, where lo is the
    // first row of U's band in column block J (rows above it are zero in U).
    // Later LU steps touch only rows below block J, so the two never meet.
    int us = 0;
    auto w_column = [&](int J) -> hipError_t {
        const int K = J * P, kb = std::min(P, n - K);
        while (us < J && lu_end(n, us, cols_end) <= K) ++us;
        const int lo = us * P;
        if (lo >= K) return hipSuccess;
        hipError_t r = launch_dgemm(K - lo, kb, kb, M + (long long)lo * ld + K, ld,
                                    M + (long long)K * ld + K, ld, Tcol, P, 1.0, 0.0, ys);
        if (r != hipSuccess) return r;
        return launch_dgemm(K, kb, K - lo, M + lo, ld, Tcol, P, M + K, ld, -1.0, 0.0, ys);
    };
    // block LU: A = L U with unit block-lower L and U_ss = the pivot blocks,
    // whose inverses D_s replace them on the diagonal of M; the blocks of L
    // go to lband (column block s: rows [r0, r1) with ld P) and their places
    // in M are cleared.  Step s is split over the streams:
    //  - pivot stream (aux): once the Schur update of step s - 1 is done, the
    //    top block of L's column s (the next pivot block's rows), the next
    //    pivot block (updated in place) and its inverse D_{s+1};
    //  - update stream (main): the rest of L's block column s, its places in
    //    M cleared, D_s onto the diagonal, then the Schur update of everything
    //    but the next pivot block, the part the pivot stream needs for step
    //    s + 1 first;
    //  - Y stream: W's column block s and Y's row block s + 1.
    for (int s = 0; s < steps; ++s) {
        const int K = s * P, kb = std::min(P, n - K);
        const double *D = Dblk[s & 1];
        const int r0 = K + kb, r1 = lu_end(n, s, rows_end);
        const int c0 = K + kb, c1 = lu_end(n, s, cols_end);
        const int kb2 = r1 > r0 ? std::min(P, n - r0) : 0;
        double *Ls = lband + loff[s];
        double *Mn = M + (long long)r0 * ld + r0;  // the next pivot block
        if (la && s > 0 && (e = hipStreamWaitEvent(aux, la->ev_block[1], 0)) != hipSuccess)
            return e;
        if (r1 > r0) {
            // only the next pivot block's rows of L here; the update stream
            // forms the rest
            if ((e = launch_dgemm(kb2, kb, kb, M + (long long)r0 * ld + K, ld, D, P, Ls, P, 1.0,
                                  0.0, aux)) != hipSuccess)
                return e;
            if ((e = launch_dgemm(kb2, kb2, kb, Ls, P, M + (long long)K * ld + r0, ld, Mn, ld,
                                  -1.0, 1.0, aux)) != hipSuccess)
                return e;
        }
        if (la) {
            if ((e = hipEventRecord(la->ev_inv[0], aux)) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(st, la->ev_inv[0], 0)) != hipSuccess) return e;
        }
        if (r1 > r0)
            k_gj_diag<<<1, 256, 0, aux>>>(ld, r0, kb2, M, Dblk[(s + 1) & 1], bad);
        if (r1 > r0) {
            if ((e = launch_dgemm(r1 - r0 - kb2, kb, kb, M + (long long)(r0 + kb2) * ld + K, ld, D,
                                  P, Ls + (long long)kb2 * P, P, 1.0, 0.0, st)) != hipSuccess)
                return e;
            k_zero_rect<<<blocks_for((long long)(r1 - r0) * kb), kThreads, 0, st>>>(
                r1 - r0, kb, ld, M + (long long)r0 * ld + K);
        }
        k_copy_block<<<blocks_for((long long)kb * kb), kThreads, 0, st>>>(
            kb, D, P, M + (long long)K * ld + K, ld);
        if (la && (e = hipEventRecord(la->ev_l, st)) != hipSuccess) return e;
        // Schur update without the next pivot block (done on the pivot
        // stream): first the two block columns the pivot stream reads next
        // (L's column block s + 1 below its pivot block, and all of column
        // block s + 2), then the event it waits for, then the rest
        auto schur = [&](int rlo, int rhi, int clo, int chi) -> hipError_t {
            if (rhi <= rlo || chi <= clo) return hipSuccess;
            return launch_dgemm(rhi - rlo, chi - clo, kb, Ls + (long long)(rlo - r0) * P, P,
                                M + (long long)K * ld + clo, ld, M + (long long)rlo * ld + clo,
                                ld, -1.0, 1.0, st);
        };
        const int cn = std::min(c1, c0 + kb2 + P);
        if (r1 > r0) {
            if ((e = schur(r0 + kb2, r1, c0, c0 + kb2)) != hipSuccess) return e;
            if ((e = schur(r0, r1, c0 + kb2, cn)) != hipSuccess) return e;
        }
        if (la && (e = hipEventRecord(la->ev_block[1], st)) != hipSuccess) return e;
        if (r1 > r0 && (e = schur(r0, r1, cn, c1)) != hipSuccess) return e;
        // the Y stream: W's column block s and Y's row block s + 1, queued
        // after the critical work of this step
        if (la && (e = hipStreamWaitEvent(ys, la->ev_l, 0)) != hipSuccess) return e;
        if ((e = w_column(s)) != hipSuccess) return e;
        if (r1 > r0 && (e = y_row(s)) != hipSuccess) return e;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (la) {
        if ((e = hipEventRecord(la->ev_y, ys)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(st, la->ev_y, 0)) != hipSuccess) return e;
        if ((e = hipEventRecord(la->ev_done, st)) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace msp
