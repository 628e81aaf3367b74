// Aggregation chain of the AMG setup on the device (Sec. 5 hierarchy, the
// pairwise rule of the host builder): strength and candidate lists per row,
// the pairwise pass as rounds of locally first edges, the numbering of the
// aggregates in creation order and the Galerkin product per coarse row.  The
// results equal the host chain bit for bit; msp_chain.h gives the argument.
#include "msp_chain.h"

#include <cstring>

#include <algorithm>
#include <future>
#include <memory>
#include <vector>

// every sum and comparison below is a single IEEE operation, as on the host
#pragma clang fp contract(off)

namespace msp {
namespace {

constexpr int kThreads = 256;
constexpr int kScanTile = 1024;  // elements per block of the scan (4 per thread)
constexpr int kFree = 0, kSingle = 1, kLow = 2, kHigh = 3;
constexpr int kNone = 0x7fffffff;
constexpr int kBatch = 8;  // rounds queued between two reads of the free count (even)

inline unsigned nblocks(long long n, int per = kThreads)
{
    return (unsigned)std::max<long long>(1, (n + per - 1) / per);
}

__global__ void k_fill_i32(int *p, int v, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Row i of a structurally symmetric M: s_ij = -(m_ij + m_ji)/2 for every
// stored off-diagonal j (m_ji read through the mirror entry), the largest
// s_ij, and eligibility (a stored nonzero off-diagonal value, and a positive
// largest s_ij).  A missing mirror entry sets *asym.
__global__ void k_strength(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                           const double *__restrict__ val, double *__restrict__ s,
                           double *__restrict__ smax, unsigned char *__restrict__ elig,
                           int *__restrict__ asym)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool coupled = false, any = false;
    double mx = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
        const int j = ci[k];
        if (j == i) continue;
        const double aij = val[k];
        int lo = rp[j], hi = rp[j + 1];
        const int end = hi;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (ci[mid] < i)
                lo = mid + 1;
            else
                hi = mid;
        }
        double aji = 0.0;
        if (lo < end && ci[lo] == i)
            aji = val[lo];
        else
            atomicOr(asym, 1);
        if (aij != 0.0) coupled = true;
        const double sij = -(aij + aji) / 2.0;
        s[k] = sij;
        if (!any || sij > mx) mx = sij;
        any = true;
    }
    smax[i] = mx;
    elig[i] = (coupled && any && mx > 0.0) ? 1 : 0;
}

// Candidates of an eligible row i: eligible j > i with s_ij >= 0.25 max_k
// s_ik, ordered by s_ij descending then j ascending, written over the row's
// own slots [rp[i], rp[i] + ncand[i]).  (Candidates j < i never matter: they
// are placed before i is visited.)
__global__ void k_candidates(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                             const double *__restrict__ s, const double *__restrict__ smax,
                             const unsigned char *__restrict__ elig, int *__restrict__ cj,
                             double *__restrict__ cs, int *__restrict__ ncand)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int m = 0;
    if (elig[i]) {
        const double thr = 0.25 * smax[i];
        const int b0 = rp[i];
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            const int j = ci[k];
            if (j <= i || !elig[j]) continue;
            const double sj = s[k];
            if (!(sj >= thr)) continue;
            int r = m;
            while (r > 0 && (cs[b0 + r - 1] < sj || (cs[b0 + r - 1] == sj && cj[b0 + r - 1] > j))) {
                cj[b0 + r] = cj[b0 + r - 1];
                cs[b0 + r] = cs[b0 + r - 1];
                --r;
            }
            cj[b0 + r] = j;
            cs[b0 + r] = sj;
            ++m;
        }
    }
    ncand[i] = m;
}

// Lists of the lower rows pointing at each row: in_ptr/in_row, the
// transpose of the candidate lists (order inside a list is free).
__global__ void k_in_count(int n, const int *__restrict__ rp, const int *__restrict__ cj,
                           const int *__restrict__ ncand, int *__restrict__ indeg)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int q = 0; q < ncand[i]; ++q) atomicAdd(&indeg[cj[rp[i] + q]], 1);
}

__global__ void k_in_fill(int n, const int *__restrict__ rp, const int *__restrict__ cj,
                          const int *__restrict__ ncand, const int *__restrict__ in_ptr,
                          int *__restrict__ cursor, int *__restrict__ in_row)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int q = 0; q < ncand[i]; ++q) {
        const int j = cj[rp[i] + q];
        in_row[in_ptr[j] + atomicAdd(&cursor[j], 1)] = i;
    }
}

// lowest free row with a candidate edge into v (kNone if there is none)
__device__ inline int lowest_free_in(int v, const int *__restrict__ in_ptr,
                                     const int *__restrict__ in_row, const int *__restrict__ st)
{
    int m = kNone;
    for (int q = in_ptr[v]; q < in_ptr[v + 1]; ++q) {
        const int k = in_row[q];
        if (k < m && st[k] == kFree) m = k;
    }
    return m;
}

// first free candidate of v (its proposal), -1 if none is left
__device__ inline int first_free_cand(int v, const int *__restrict__ rp, const int *__restrict__ cj,
                                      const int *__restrict__ ncand, const int *__restrict__ st)
{
    const int b0 = rp[v], m = ncand[v];
    for (int q = 0; q < m; ++q) {
        const int j = cj[b0 + q];
        if (st[j] == kFree) return j;
    }
    return -1;
}

// Each row's first kRec in-rows and first kRec candidates (in order) held
// inline, so that a round loads the states of a whole list at once instead of
// walking it one dependent load after another.  kOver in a record's first
// slot: the list is longer, and the round walks it in full.  Unused slots are
// kNone (in-rows) and -1 (candidates).
constexpr int kRec = 4;
constexpr int kOver = -2;
__global__ void k_records(int n, const int *__restrict__ rp, const int *__restrict__ cj,
                          const int *__restrict__ ncand, const int *__restrict__ in_ptr,
                          const int *__restrict__ in_row, int4 *__restrict__ rin,
                          int4 *__restrict__ rcand)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int a[kRec] = {kNone, kNone, kNone, kNone};
    const int q0 = in_ptr[v], q1 = in_ptr[v + 1];
    if (q1 - q0 > kRec)
        a[0] = kOver;
    else
        for (int q = q0; q < q1; ++q) a[q - q0] = in_row[q];
    rin[v] = make_int4(a[0], a[1], a[2], a[3]);
    int c[kRec] = {-1, -1, -1, -1};
    const int m = ncand[v], b0 = rp[v];
    if (m > kRec)
        c[0] = kOver;
    else
        for (int q = 0; q < m; ++q) c[q] = cj[b0 + q];
    rcand[v] = make_int4(c[0], c[1], c[2], c[3]);
}

// lowest_free_in / first_free_cand through the records
__device__ inline int lowest_free_in_rec(int v, const int4 *__restrict__ rin,
                                         const int *__restrict__ in_ptr,
                                         const int *__restrict__ in_row,
                                         const int *__restrict__ st)
{
    const int4 a = rin[v];
    if (a.x == kOver) return lowest_free_in(v, in_ptr, in_row, st);
    const bool f0 = a.x != kNone && st[a.x] == kFree;
    const bool f1 = a.y != kNone && st[a.y] == kFree;
    const bool f2 = a.z != kNone && st[a.z] == kFree;
    const bool f3 = a.w != kNone && st[a.w] == kFree;
    int m = kNone;
    if (f0) m = a.x;
    if (f1 && a.y < m) m = a.y;
    if (f2 && a.z < m) m = a.z;
    if (f3 && a.w < m) m = a.w;
    return m;
}

__device__ inline int first_free_cand_rec(int v, const int4 *__restrict__ rcand,
                                          const int *__restrict__ rp, const int *__restrict__ cj,
                                          const int *__restrict__ ncand,
                                          const int *__restrict__ st)
{
    const int4 c = rcand[v];
    if (c.x == kOver) return first_free_cand(v, rp, cj, ncand, st);
    const bool f0 = c.x >= 0 && st[c.x] == kFree;
    const bool f1 = c.y >= 0 && st[c.y] == kFree;
    const bool f2 = c.z >= 0 && st[c.z] == kFree;
    const bool f3 = c.w >= 0 && st[c.w] == kFree;
    return f0 ? c.x : f1 ? c.y : f2 ? c.z : f3 ? c.w : -1;
}

// One round.  An edge (i, j) between free rows is taken when i has no free
// lower row pointing at it, j is i's first free candidate, and i is the
// lowest free row pointing at j: the edge then comes first at both of its
// ends.  A free row with no free lower row pointing at it and no free
// candidate stays alone.  Every row evaluates this from the round's input
// states (st) and writes only its own output state (st_next), so the two
// ends of a taken edge reach the same decision independently.  If nfree is
// set, the free rows of the input are counted into it (the host reads the
// count of one round per batch only: counting in every round would put
// thousands of atomics on one address each time); a set nfree_next is
// cleared for the next round's count.
__global__ void __launch_bounds__(kThreads)
k_round(int n, const int *__restrict__ rp, const int *__restrict__ cj,
        const int *__restrict__ ncand, const int *__restrict__ in_ptr,
        const int *__restrict__ in_row, const int4 *__restrict__ rin,
        const int4 *__restrict__ rcand, const int *__restrict__ st, int *__restrict__ st_next,
        int *__restrict__ partner, int *__restrict__ nfree, int *__restrict__ nfree_next)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v == 0 && nfree_next) *nfree_next = 0;
    bool fr = false;
    if (v < n) {
        const int s0 = st[v];
        int s1 = s0;
        if (s0 == kFree) {
            fr = true;
            const int m = lowest_free_in_rec(v, rin, in_ptr, in_row, st);
            if (m == kNone) {
                const int p = first_free_cand_rec(v, rcand, rp, cj, ncand, st);
                if (p < 0) {
                    s1 = kSingle;
                } else if (lowest_free_in_rec(p, rin, in_ptr, in_row, st) == v) {
                    s1 = kLow;
                    partner[v] = p;
                }
            } else if (lowest_free_in_rec(m, rin, in_ptr, in_row, st) == kNone &&
                       first_free_cand_rec(m, rcand, rp, cj, ncand, st) == v) {
                s1 = kHigh;
                partner[v] = m;
            }
        }
        st_next[v] = s1;
    }
    if (nfree) {  // the same for every block
        const int cnt = __syncthreads_count(fr);
        if (threadIdx.x == 0 && cnt) atomicAdd(nfree, cnt);
    }
}

// A row opens an aggregate when it is alone or the lower row of its pair.
__global__ void k_leaders(int n, const int *__restrict__ state, int *__restrict__ flag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = state[i] != kHigh;
}

// Aggregate numbers in order of their lowest row (= creation order of the
// ascending visit) and the member rows of every aggregate.
__global__ void k_number(int n, const int *__restrict__ state, const int *__restrict__ partner,
                         const int *__restrict__ pos, int *__restrict__ agg,
                         int *__restrict__ mem0, int *__restrict__ mem1)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int st = state[i];
    if (st == kHigh) {
        agg[i] = pos[partner[i]];
        return;
    }
    const int I = pos[i];
    agg[i] = I;
    mem0[I] = i;
    mem1[I] = st == kLow ? partner[i] : -1;
}

// ---- exclusive scan of n ints: out[0..n], out[n] = total ----------------
__device__ inline int block_inclusive(int *sh, int t)
{
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int d = 1; d < kThreads; d <<= 1) {
        const int x = threadIdx.x >= (unsigned)d ? sh[threadIdx.x - d] : 0;
        __syncthreads();
        sh[threadIdx.x] += x;
        __syncthreads();
    }
    return sh[threadIdx.x];
}

__global__ void __launch_bounds__(kThreads)
k_scan_tile(const int *__restrict__ in, int *__restrict__ out, int *__restrict__ tile_sum, int n)
{
    __shared__ int sh[kThreads];
    const long long base = (long long)blockIdx.x * kScanTile + threadIdx.x * 4;
    int v[4], t = 0;
    for (int q = 0; q < 4; ++q) {
        const long long i = base + q;
        v[q] = i < n ? in[i] : 0;
        t += v[q];
    }
    const int incl = block_inclusive(sh, t);
    int run = incl - t;
    for (int q = 0; q < 4; ++q) {
        const long long i = base + q;
        if (i < n) out[i] = run;
        run += v[q];
    }
    if (threadIdx.x == kThreads - 1) tile_sum[blockIdx.x] = incl;
}

__global__ void __launch_bounds__(kThreads)
k_scan_sums(int *__restrict__ tile_sum, int ntiles, int *__restrict__ total)
{
    __shared__ int sh[kThreads];
    __shared__ int carry_s;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int c0 = 0; c0 < ntiles; c0 += kThreads) {
        const int i = c0 + threadIdx.x;
        const int t = i < ntiles ? tile_sum[i] : 0;
        const int carry = carry_s;
        const int incl = block_inclusive(sh, t);
        if (i < ntiles) tile_sum[i] = carry + incl - t;
        __syncthreads();
        if (threadIdx.x == kThreads - 1) carry_s = carry + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry_s;
}

__global__ void k_scan_add(int *__restrict__ out, const int *__restrict__ tile_sum, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += tile_sum[i / kScanTile];
}

// ---- Galerkin product for aggregates of one or two rows -----------------
// Coarse row I gathers the rows mem0[I] < mem1[I] in order, column by column;
// entry (I, agg(j)) is the first term, then plus each later term, in that
// order (the host's (fine row, fine column) order).  The running list,
// sorted by coarse column, lives in the member rows' own slots of wj/wv
// (position t < len0 in row mem0, the rest in row mem1).
__device__ inline int gal_slot(int t, int b0, int len0, int b1)
{
    return t < len0 ? b0 + t : b1 + (t - len0);
}

__global__ void k_gal_rows(int nc, const int *__restrict__ rp, const int *__restrict__ ci,
                           const double *__restrict__ val, const int *__restrict__ agg,
                           const int *__restrict__ mem0, const int *__restrict__ mem1,
                           int *__restrict__ wj, double *__restrict__ wv, int *__restrict__ cnt)
{
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    const int r0 = mem0[I], r1 = mem1[I];
    const int b0 = rp[r0], len0 = rp[r0 + 1] - b0;
    const int b1 = r1 >= 0 ? rp[r1] : 0;
    int m = 0;
    for (int w = 0; w < 2; ++w) {
        const int r = w == 0 ? r0 : r1;
        if (r < 0) break;
        for (int k = rp[r]; k < rp[r + 1]; ++k) {
            const int J = agg[ci[k]];
            const double v = val[k];
            int lo = 0, hi = m;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (wj[gal_slot(mid, b0, len0, b1)] < J)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            if (lo < m && wj[gal_slot(lo, b0, len0, b1)] == J) {
                const int q = gal_slot(lo, b0, len0, b1);
                wv[q] = wv[q] + v;
                continue;
            }
            for (int t = m; t > lo; --t) {
                const int d = gal_slot(t, b0, len0, b1), sidx = gal_slot(t - 1, b0, len0, b1);
                wj[d] = wj[sidx];
                wv[d] = wv[sidx];
            }
            const int q = gal_slot(lo, b0, len0, b1);
            wj[q] = J;
            wv[q] = v;
            ++m;
        }
    }
    cnt[I] = m;
}

__global__ void k_gal_fill(int nc, const int *__restrict__ rp, const int *__restrict__ mem0,
                           const int *__restrict__ mem1, const int *__restrict__ wj,
                           const double *__restrict__ wv, const int *__restrict__ rpc,
                           int *__restrict__ cic, double *__restrict__ valc)
{
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nc) return;
    const int r0 = mem0[I], r1 = mem1[I];
    const int b0 = rp[r0], len0 = rp[r0 + 1] - b0;
    const int b1 = r1 >= 0 ? rp[r1] : 0;
    const int o = rpc[I], m = rpc[I + 1] - o;
    for (int t = 0; t < m; ++t) {
        const int q = gal_slot(t, b0, len0, b1);
        cic[o + t] = wj[q];
        valc[o + t] = wv[q];
    }
}

__global__ void k_compose(int n, const int *__restrict__ a1, const int *__restrict__ a2,
                          int *__restrict__ agg)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) agg[i] = a2[a1[i]];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct DevLevel {
    int n = 0;
    int *rp = nullptr, *ci = nullptr;
    double *val = nullptr;
};

struct Chain {
    hipStream_t st = nullptr;
    HipFail hip_fail = nullptr;
    int *pinned = nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev_lvl = nullptr;  // a new level is on the device
    // work arrays, sized for level 0 (no later matrix is larger)
    double *s = nullptr, *cs = nullptr, *smax = nullptr;
    int *cj = nullptr, *ncand = nullptr, *partner = nullptr;
    int *state[2] = {nullptr, nullptr};  // round input / output, alternating
    int *in_ptr = nullptr, *in_row = nullptr;
    int4 *rin = nullptr, *rcand = nullptr;  // per-row records of the two lists
    hipStream_t cap = nullptr;            // capture stream for the round batches
    int *pos = nullptr, *flag = nullptr, *cnt = nullptr, *tiles = nullptr, *ctr = nullptr;
    int *a1 = nullptr, *a2 = nullptr, *aggf = nullptr, *mem0 = nullptr, *mem1 = nullptr;
    unsigned char *elig = nullptr;
    DevLevel set[3];  // M1 and two alternating coarse levels

    void ck(hipError_t e) const
    {
        if (e != hipSuccess) {
            (void)hipGetLastError();
            hip_fail(e);
        }
    }
    void launched() const { ck(hipGetLastError()); }
    int read_int(const int *d, int slot)
    {
        ck(hipMemcpyAsync(pinned + slot, d, sizeof(int), hipMemcpyDeviceToHost, st));
        ck(hipStreamSynchronize(st));
        return pinned[slot];
    }
    void fill(int *p, int v, int n)
    {
        if (n <= 0) return;
        k_fill_i32<<<nblocks(n), kThreads, 0, st>>>(p, v, n);
        launched();
    }
    // out[0..n] = exclusive scan of in[0..n), out[n] = total
    void scan(const int *in, int *out, int n)
    {
        const int ntiles = (int)std::max<long long>(1, ((long long)n + kScanTile - 1) / kScanTile);
        k_scan_tile<<<ntiles, kThreads, 0, st>>>(in, out, tiles, n);
        launched();
        k_scan_sums<<<1, kThreads, 0, st>>>(tiles, ntiles, out + n);
        launched();
        k_scan_add<<<nblocks(n), kThreads, 0, st>>>(out, tiles, n);
        launched();
    }
    void strength(const DevLevel &L)
    {
        k_strength<<<nblocks(L.n), kThreads, 0, st>>>(L.n, L.rp, L.ci, L.val, s, smax, elig,
                                                      ctr + 2);
        launched();
    }
    // One pairwise pass on L (strength already computed when have_s); agg
    // into `agg`, members into mem0/mem1; returns the aggregate count.
    int pass(const DevLevel &L, bool have_s, int *agg)
    {
        const int n = L.n;
        if (!have_s) strength(L);
        k_candidates<<<nblocks(n), kThreads, 0, st>>>(n, L.rp, L.ci, s, smax, elig, cj, cs, ncand);
        launched();
        // in-lists (cnt counts, flag serves as the fill cursor)
        fill(cnt, 0, n);
        fill(flag, 0, n);
        k_in_count<<<nblocks(n), kThreads, 0, st>>>(n, L.rp, cj, ncand, cnt);
        launched();
        scan(cnt, in_ptr, n);
        k_in_fill<<<nblocks(n), kThreads, 0, st>>>(n, L.rp, cj, ncand, in_ptr, flag, in_row);
        launched();
        k_records<<<nblocks(n), kThreads, 0, st>>>(n, L.rp, cj, ncand, in_ptr, in_row, rin,
                                                   rcand);
        launched();
        fill(state[0], kFree, n);
        fill(ctr, 0, 2);
        // kBatch rounds (an even number: the states end in state[0]) as one graph
        hipGraphExec_t exec = nullptr;
        {
            ck(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
            // only the batch's last round counts its free rows (into ctr[1],
            // cleared by the round before it)
            for (int q = 0; q < kBatch; ++q) {
                const int a = q & 1;
                k_round<<<nblocks(n), kThreads, 0, cap>>>(
                    n, L.rp, cj, ncand, in_ptr, in_row, rin, rcand, state[a], state[a ^ 1], partner,
                    q == kBatch - 1 ? ctr + 1 : nullptr, q == kBatch - 2 ? ctr + 1 : nullptr);
            }
            hipGraph_t g = nullptr;
            const hipError_t e1 = hipStreamEndCapture(cap, &g);
            const hipError_t e2 = e1 == hipSuccess ? hipGraphInstantiate(&exec, g, nullptr, nullptr, 0)
                                                   : e1;
            if (g) (void)hipGraphDestroy(g);
            ck(e2);
        }
        struct ExecGuard {
            hipGraphExec_t e;
            hipStream_t s;
            ~ExecGuard()
            {
                (void)hipStreamSynchronize(s);
                (void)hipGraphExecDestroy(e);
            }
        } exec_guard{exec, st};
        // batches are queued two ahead of the one whose free count is read,
        // so the device always has rounds queued while the host checks
        long long r = 0;
        const long long cap_rounds = (long long)n + 6LL * kBatch + 4;
        for (int batch = 0;; ++batch) {
            ck(hipGraphLaunch(exec, st));
            r += kBatch;
            // free rows at the start of the batch's last round
            const int slot = batch % 3;
            ck(hipMemcpyAsync(pinned + slot, ctr + 1, sizeof(int),
                              hipMemcpyDeviceToHost, st));
            ck(hipEventRecord(ev[slot], st));
            if (batch >= 2) {
                const int old = (batch - 2) % 3;
                ck(hipEventSynchronize(ev[old]));
                if (pinned[old] == 0) break;
            }
            // every round settles at least the lowest free row
            if (r > cap_rounds) hip_fail(hipErrorUnknown);
        }
        k_leaders<<<nblocks(n), kThreads, 0, st>>>(n, state[0], flag);
        launched();
        scan(flag, pos, n);
        k_number<<<nblocks(n), kThreads, 0, st>>>(n, state[0], partner, pos, agg, mem0, mem1);
        launched();
        return read_int(pos + n, 4);
    }
    // C = P^T L P for the pass just numbered (aggregates of one or two rows),
    // queued without a wait (nnz(C) is C.rp[nc] on the device).  The
    // candidate arrays serve as the row lists.
    void galerkin(const DevLevel &L, const int *agg, int nc, DevLevel &C)
    {
        C.n = nc;
        k_gal_rows<<<nblocks(nc), kThreads, 0, st>>>(nc, L.rp, L.ci, L.val, agg, mem0, mem1, cj,
                                                     s, cnt);
        launched();
        scan(cnt, C.rp, nc);
        k_gal_fill<<<nblocks(nc), kThreads, 0, st>>>(nc, L.rp, mem0, mem1, cj, s, C.rp, C.ci,
                                                     C.val);
        launched();
    }
    void to_device(const Csr &H, DevLevel &C)
    {
        C.n = H.n;
        ck(hipMemcpyAsync(C.rp, H.rp.data(), sizeof(int) * (H.n + 1), hipMemcpyHostToDevice, st));
        if (H.nnz()) {
            ck(hipMemcpyAsync(C.ci, H.ci.data(), sizeof(int) * H.nnz(), hipMemcpyHostToDevice, st));
            ck(hipMemcpyAsync(C.val, H.val.data(), sizeof(double) * H.nnz(),
                              hipMemcpyHostToDevice, st));
        }
        ck(hipStreamSynchronize(st));
    }
};

struct EventGuard {
    hipEvent_t *ev;
    hipEvent_t *ev_lvl;
    ~EventGuard()
    {
        for (int i = 0; i < 3; ++i)
            if (ev[i]) (void)hipEventDestroy(ev[i]);
        if (*ev_lvl) (void)hipEventDestroy(*ev_lvl);
    }
};

// Sets every work array of X to its offset in one allocation at `base`,
// each sized for level 0 (no later matrix is larger) and 256-byte aligned;
// with base == nullptr it only measures.  Returns the bytes used.
size_t place(Chain &X, char *base, int n0, long long nnz0)
{
    const long long n1 = (long long)n0 + 1, ntiles = n0 / kScanTile + 2;
    size_t off = 0;
    auto take = [&](long long count, size_t sz) -> void * {
        void *r = base ? (void *)(base + off) : nullptr;
        off += (((size_t)std::max<long long>(count, 1) * sz) + 255) & ~(size_t)255;
        return r;
    };
    X.s = (double *)take(nnz0, sizeof(double));
    X.cs = (double *)take(nnz0, sizeof(double));
    X.smax = (double *)take(n0, sizeof(double));
    X.cj = (int *)take(nnz0, sizeof(int));
    X.in_row = (int *)take(nnz0, sizeof(int));
    X.ncand = (int *)take(n0, sizeof(int));
    X.state[0] = (int *)take(n0, sizeof(int));
    X.state[1] = (int *)take(n0, sizeof(int));
    X.partner = (int *)take(n0, sizeof(int));
    X.a1 = (int *)take(n0, sizeof(int));
    X.a2 = (int *)take(n0, sizeof(int));
    X.aggf = (int *)take(n0, sizeof(int));
    X.in_ptr = (int *)take(n1, sizeof(int));
    X.mem0 = (int *)take(n1, sizeof(int));
    X.mem1 = (int *)take(n1, sizeof(int));
    X.pos = (int *)take(n1, sizeof(int));
    X.cnt = (int *)take(n1, sizeof(int));
    X.flag = (int *)take(n1, sizeof(int));
    X.tiles = (int *)take(ntiles, sizeof(int));
    X.ctr = (int *)take(4, sizeof(int));
    X.elig = (unsigned char *)take(n0, 1);
    X.rin = (int4 *)take(n0, sizeof(int4));
    X.rcand = (int4 *)take(n0, sizeof(int4));
    for (int k = 0; k < 3; ++k) {
        X.set[k].rp = (int *)take(n1, sizeof(int));
        X.set[k].ci = (int *)take(nnz0, sizeof(int));
        X.set[k].val = (double *)take(nnz0, sizeof(double));
    }
    return off;
}

}  // namespace

size_t device_chain_bytes(int n0, long long nnz0)
{
    Chain X;
    return place(X, nullptr, n0, nnz0);
}

int device_hierarchy(Csr &A0, const int *rp0, const int *ci0, const double *val0,
                     int max_coarse, int max_levels, int max_dense, Hierarchy &H,
                     const LevelCallback &on_smoothed, const std::function<void()> &level0_values,
                     hipStream_t st, hipStream_t cap, hipStream_t copy_st,
                     const DeviceAlloc &alloc, HipFail hip_fail, int *pinned,
                     const PinnedBuffer &staging)
{
    const int n0 = A0.n;
    const long long nnz0 = A0.nnz();
    if (n0 <= max_coarse || max_levels <= 1) {
        H = Hierarchy();
        H.A.push_back(std::move(A0));
        level0_values();  // level 0 is the coarsest: the caller inverts it next
        return H.A.back().n > max_dense ? -9 : 0;
    }
    Chain X;
    X.st = st;
    X.cap = cap;
    X.hip_fail = hip_fail;
    X.pinned = pinned;
    EventGuard guard{X.ev, &X.ev_lvl};
    for (int i = 0; i < 3; ++i) X.ck(hipEventCreateWithFlags(&X.ev[i], hipEventDisableTiming));
    X.ck(hipEventCreateWithFlags(&X.ev_lvl, hipEventDisableTiming));
    // one allocation for every work array
    char *base = (char *)alloc(place(X, nullptr, n0, nnz0));
    place(X, base, n0, nnz0);
    // level 0: strength first, which also tells whether the pattern is
    // structurally symmetric
    DevLevel cur;
    cur.n = n0;
    cur.rp = const_cast<int *>(rp0);
    cur.ci = const_cast<int *>(ci0);
    cur.val = const_cast<double *>(val0);
    X.fill(X.ctr + 2, 0, 1);
    X.strength(cur);
    if (X.read_int(X.ctr + 2, 0) != 0) return 1;

    H = Hierarchy();
    H.A.push_back(std::move(A0));
    // The host copy of each new level (and of the aggregation map that made
    // it) runs on a copy thread while the device goes on with the next level;
    // that thread also starts the level's host work (on_smoothed).  A level
    // is joined before its device buffers can be reused: the previous level's
    // copy before this level's aggregation map is composed (aggf is shared,
    // the level buffers alternate), and every copy before the host reads it.
    // `pending` ends when the copy thread is done; `copied` as soon as its
    // device reads are (with staging, the host copies out of the page-locked
    // buffer may still run: they write only through pointers taken before)
    std::future<void> pending, copied;
    const auto join = [&pending, &copied]() {
        if (copied.valid()) copied.get();
        if (pending.valid()) pending.get();
    };
    // (a failure of the copy thread before its device reads ended comes
    // through `copied`)
    const auto join_device = [&copied]() {
        if (copied.valid()) copied.get();
    };
    bool have_s = true;
    bool main_calls = true;  // level l's on_smoothed is due on this thread
    int next = 1;  // set[0] holds M1; levels alternate between set[1] and set[2]
    for (int l = 0;; ++l) {
        const int nl = H.A[l].n;
        const bool last = nl <= max_coarse || l == max_levels - 1 ||
                          (l > 0 && (double)nl > 0.9 * (double)H.A[l - 1].n);
        if (last) break;
        if (main_calls && on_smoothed) {
            if (l > 0) join();
            const Csr &hc = H.A[l];
            on_smoothed(l, hc.n, hc.rp.data(), hc.ci.data());
        }
        const int nc1 = X.pass(cur, have_s, X.a1);
        have_s = false;
        DevLevel &M1 = X.set[0];
        X.galerkin(cur, X.a1, nc1, M1);
        const int nc2 = X.pass(M1, false, X.a2);
        DevLevel &C = X.set[next];
        X.galerkin(M1, X.a2, nc2, C);
        join_device();
        k_compose<<<nblocks(cur.n), kThreads, 0, st>>>(cur.n, X.a1, X.a2, X.aggf);
        X.launched();
        X.ck(hipEventRecord(X.ev_lvl, st));
        {
            // sized (and cleared) by the copy thread, off this thread's path
            Csr Cn;
            Cn.n = nc2;
            H.agg.emplace_back();
            H.A.push_back(std::move(Cn));
        }
        const bool stalled = (double)nc2 > 0.9 * (double)cur.n;
        // level l+1 is smoothed unless it is the last one (a stalled level
        // may still change below, so its host work starts on this thread)
        const bool next_smoothed =
            !stalled && !(nc2 <= max_coarse || l + 1 == max_levels - 1);
        {
            Csr &hn = H.A[l + 1];
            std::vector<int> &hagg = H.agg[l];
            const int nf = cur.n;
            const DevLevel Cd = C;
            const int *aggf = X.aggf;
            const hipEvent_t ready = X.ev_lvl;
            const int lnext = l + 1;
            const bool call = next_smoothed && on_smoothed;
            const PinnedBuffer *stg = staging ? &staging : nullptr;
            auto dev_done = std::make_shared<std::promise<void>>();
            copied = dev_done->get_future();
            pending = std::async(std::launch::async, [&hn, &hagg, nf, Cd, aggf, ready, copy_st,
                                                      hip_fail, call, lnext, &on_smoothed, stg,
                                                      dev_done]() {
                bool signalled = false;
                try {
                    hagg.resize(nf);
                    hn.rp.resize(Cd.n + 1);
                    auto ck = [hip_fail](hipError_t e) {
                        if (e != hipSuccess) {
                            (void)hipGetLastError();
                            hip_fail(e);
                        }
                    };
                    ck(hipStreamWaitEvent(copy_st, ready, 0));
                    ck(hipMemcpyAsync(hn.rp.data(), Cd.rp, sizeof(int) * (Cd.n + 1),
                                      hipMemcpyDeviceToHost, copy_st));
                    ck(hipStreamSynchronize(copy_st));
                    const long long nnzc = hn.rp[Cd.n];
                    hn.ci.resize(nnzc);
                    hn.val.resize(nnzc);
                    // page-locked staging: [ci | val | agg], one DMA each
                    char *sb = stg ? (char *)(*stg)(lnext, sizeof(int) * (size_t)nnzc +
                                                               sizeof(double) * (size_t)nnzc +
                                                               sizeof(int) * (size_t)nf)
                                   : nullptr;
                    int *sci = sb ? (int *)sb : hn.ci.data();
                    double *sval =
                        sb ? (double *)(sb + sizeof(int) * (size_t)nnzc) : hn.val.data();
                    int *sagg = sb ? (int *)(sb + (sizeof(int) + sizeof(double)) * (size_t)nnzc)
                                   : hagg.data();
                    // the pattern first: the level's host work (its groups) needs
                    // only that, and starts while the rest is copied
                    if (nnzc)
                        ck(hipMemcpyAsync(sci, Cd.ci, sizeof(int) * nnzc, hipMemcpyDeviceToHost,
                                          copy_st));
                    ck(hipStreamSynchronize(copy_st));
                    if (call) on_smoothed(lnext, hn.n, hn.rp.data(), sci);
                    if (nnzc)
                        ck(hipMemcpyAsync(sval, Cd.val, sizeof(double) * nnzc,
                                          hipMemcpyDeviceToHost, copy_st));
                    ck(hipMemcpyAsync(sagg, aggf, sizeof(int) * nf, hipMemcpyDeviceToHost,
                                      copy_st));
                    // H grows on the main thread once the device reads are done:
                    // the destinations are taken here (moving a vector keeps its
                    // storage)
                    int *dci = hn.ci.data(), *dagg = hagg.data();
                    double *dval = hn.val.data();
                    if (sb) std::memcpy(dci, sci, sizeof(int) * (size_t)nnzc);
                    ck(hipStreamSynchronize(copy_st));
                    signalled = true;
                    dev_done->set_value();
                    if (sb) {
                        std::memcpy(dval, sval, sizeof(double) * (size_t)nnzc);
                        std::memcpy(dagg, sagg, sizeof(int) * (size_t)nf);
                    }
                } catch (...) {
                    if (signalled) throw;
                    (void)hipStreamSynchronize(copy_st);
                    (void)hipGetLastError();
                    dev_done->set_exception(std::current_exception());
                }
            });
        }
        main_calls = !next_smoothed;
        if (stalled) {
            // stalled: absorb singletons, then one Galerkin product on A_l
            join();
            if (l == 0) level0_values();
            const int nc3 = absorb_singletons(H.A[l], H.agg[l], nc2);
            if (nc3 < nc2) {
                H.A[l + 1] = msp::galerkin(H.A[l], H.agg[l], nc3);
                X.to_device(H.A[l + 1], C);
            }
        }
        cur = C;
        next = 3 - next;
    }
    join();
    return H.A.back().n > max_dense ? -9 : 0;
}

}  // namespace msp
