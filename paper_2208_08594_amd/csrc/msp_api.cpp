// libmsp C-ABI: context, adaptive setup, two-stage preconditioner apply and
// the FGMRES driver.  Device work is in msp_kernels.hip; host graph work in
// msp_host.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <future>
#include <mutex>
#include <new>
#include <thread>
#include <numeric>
#include <type_traits>
#include <vector>

#include "msp.h"
#include "msp_chain.h"
#include "msp_host.h"
#include "msp_kernels.h"
#include "msp_stages.h"

namespace {

using namespace msp;

struct MspError {
    int code;
};

// parts of an FGMRES iteration timed by msp_stage_set_timing
constexpr int kTimedParts = 3;  // 0 SpMV, 1 preconditioner apply, 2 Gram-Schmidt step

[[noreturn]] void fail(int code) { throw MspError{code}; }
[[noreturn]] void fail_hip(hipError_t e)
{
    fail(e == hipErrorOutOfMemory ? MSP_ERR_NOMEM : MSP_ERR_HIP);
}

#define HIPCHK(expr)                                 \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) {                      \
            (void)hipGetLastError();                 \
            fail(e_ == hipErrorOutOfMemory ? MSP_ERR_NOMEM : MSP_ERR_HIP); \
        }                                            \
    } while (0)

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// A device sliced-ELL matrix (pattern on the device + the host layout).
struct DevSell {
    SellLayout lay;
    int4 *slices = nullptr;
    int *col = nullptr;
    int *src = nullptr;
    int lanes = 1;  // lanes per row of the scalar sweep and residual kernels
    std::vector<int4> slices_h;  // host source of `slices` (kept while the copy may run)
    SellView view(int seg) const
    {
        SellView v;
        v.slices = slices;
        v.col = col;
        v.slice_begin = lay.seg_slice[seg];
        v.slice_end = lay.seg_slice[seg + 1];
        v.lanes = lanes;
        return v;
    }
    SellView all() const
    {
        SellView v;
        v.slices = slices;
        v.col = col;
        v.slice_begin = 0;
        v.slice_end = (int)lay.slice_row0.size();
        v.lanes = lanes;
        return v;
    }
    int nseg() const { return (int)lay.seg_slice.size() - 1; }
};

struct Level {
    int n = 0, g = 0, nc = 0;
    Csr A;                      // natural order, FP64 setup values
    std::vector<int> color, agg;
    std::vector<int> perm, iperm;  // natural -> position, position -> natural
    std::vector<int> seg_row;
    DevSell S;                  // off-diagonal entries in position space
    double *val64 = nullptr, *diag64 = nullptr;
    float *val32 = nullptr, *diag32 = nullptr;
    int *perm_d = nullptr, *iperm_d = nullptr;
    int *agg_pos = nullptr, *mem_ptr = nullptr, *mem = nullptr;
    // the same maps in the coarse level's natural order (prepared before the
    // coarse level's positions are known) and the host sources of uploads
    int *natc_d = nullptr, *mptr_nat_d = nullptr, *mem_nat_d = nullptr;
    std::vector<int> natc_h, mptr_nat_h, mem_nat_h, mem_ptr_h;
    void *f = nullptr, *x = nullptr, *r = nullptr;  // work vectors in the precond precision
};

// N stage (concentration block, block Gauss-Seidel in the groups of the
// block graph): setup data and work vectors, valid with B.
struct NStage {
    bool on = false;
    std::vector<int> grp_ptr;  // cells of group k: cells[grp_ptr[k] .. grp_ptr[k+1])
    int *cells = nullptr;
    std::vector<int> cells_h;  // host source of `cells`
    double *Dn64 = nullptr, *Ann64 = nullptr;
    float *Dn32 = nullptr, *Ann32 = nullptr;
    void *gN = nullptr, *y = nullptr;  // preconditioner precision, n (b-1)
    double *w1 = nullptr, *r1 = nullptr;  // N
};

struct BiluData {
    std::vector<int> ord;  // elimination order
    std::vector<int> fwd_rows, fwd_ptr, bwd_rows, bwd_ptr;
    std::vector<int> fwd_vpos, bwd_vpos;  // elimination position of each level-ordered row
    std::vector<char> fwd_live;           // forward level with at least one stored entry
    DevSell L, U;
    int *fwd_rows_d = nullptr, *bwd_rows_d = nullptr;
    int *pos_d = nullptr;  // elimination position of each block row: the solves' vector order
    int *fwd_vpos_d = nullptr, *bwd_vpos_d = nullptr;
    int *dsrc = nullptr;  // per U slice-lane: block row (for the pivot inverses)
    double *F = nullptr, *Dinv = nullptr;  // natural layout FP64
    double *L64 = nullptr, *U64 = nullptr, *D64 = nullptr;
    float *L32 = nullptr, *U32 = nullptr, *D32 = nullptr;
};

}  // namespace

// FGMRES(m) workspace for N unknowns: the Arnoldi basis V (m+1 vectors),
// the preconditioned directions Z (m vectors), the new direction w, the
// per-block partial dot products, the Gram-Schmidt coefficients and norms, and
// the least-squares solution y.
struct Krylov {
    double *V = nullptr, *Z = nullptr, *w = nullptr, *partial = nullptr, *hbuf = nullptr,
           *ydev = nullptr;
};

struct msp_ctx {
    msp_options opt{};
    int device = 0;
    hipStream_t stream = nullptr;
    // allocation lists by lifetime
    std::vector<void *> allocA, allocB, allocW;
    // current matrix
    int n = 0, b = 0, p = 0;
    long long nnzb = 0;
    std::vector<int> rp, ci, diag_pos;
    DevSell SA;
    int *rp_d = nullptr, *diag_d = nullptr, *ci_d = nullptr;
    double *valA = nullptr;
    float *pcol32 = nullptr;
    bool haveA = false;
    // preconditioner
    bool hasB = false;
    int Bn = 0, Bb = 0, Bp = 0;
    long long Bnnzb = 0;
    double *omega = nullptr;
    std::vector<Level> lev;
    int nL = 0, ldL = 0, sweepK = 0;
    // coarsest-level solver A^-1 = W Y (W block upper, Y block unit lower
    // triangular, both nL x nL with leading dimension ldL) and its FP64 work
    // vector
    double *cinv = nullptr, *cY = nullptr, *ct = nullptr;
    BiluData bilu;
    NStage ns;
    void *e_nat = nullptr, *ybuf = nullptr;
    // captured preconditioner apply (valid for the current B and A layout)
    double *vin = nullptr, *zout = nullptr;
    ApplyIo *io = nullptr;  // the captured apply's vectors, set before each launch
    double *tC = nullptr, *tA = nullptr, *tB = nullptr;  // timing-stage scratch (with B)
    hipStream_t cap_stream = nullptr;
    // second stream of the setup: level uploads and the block ILU(0)
    // factorisation run on it while the coarsest inverse runs on `stream`
    hipStream_t side = nullptr;
    hipEvent_t ev_main = nullptr, ev_side = nullptr;
    hipStream_t copy_stream = nullptr;  // stream of upload(); null = `stream`
    // streams and events of the coarsest-level solver
    GjLookAhead gj{};
    hipGraphExec_t apply_exec = nullptr;
    // krylov workspace (allocated by the first msp_solve of a size)
    long long wsN = 0;
    int wsm = 0;
    Krylov kw{};
    double *hhost = nullptr;  // pinned
    int *flag = nullptr, *flag_host = nullptr;
    int *chain_host = nullptr;  // pinned, progress reads of the device aggregation chain
    // pinned staging of the chain's level copies, one buffer per level, kept
    // (and grown) across setups
    std::vector<std::pair<void *, size_t>> chain_stage;
    std::mutex chain_stage_mu;
    bool pattern_ok = false;    // rp/ci (host) and rp_d/ci_d hold a checked pattern
    bool pattern_sym = false;   // that pattern is structurally symmetric
    long long pattern_gen = 0;  // counts pattern changes
    long long lev0_gen = -1;    // pattern_gen when lev[0].A was built
    hipStream_t chain_copy = nullptr;  // device-to-host copies of the setup
    hipEvent_t ev_a0 = nullptr;
    // adaptive state and statistics
    int it_prev = -1, setup_calls = 0, solves = 0;
    msp_info info{};
    // optional HIP-event timing of the solve's parts (SpMV, preconditioner
    // apply, Gram-Schmidt step): summed ms and counts over the last solve
    bool timing = false;
    hipEvent_t tev[4] = {nullptr, nullptr, nullptr, nullptr};
    hipEvent_t ev_step = nullptr;  // end of the solve's last queued step
    double t_ms[kTimedParts] = {0, 0, 0};
    int t_calls[kTimedParts] = {0, 0, 0};

    void *dalloc(size_t bytes, std::vector<void *> &list)
    {
        if (bytes == 0) bytes = 16;
        void *p_ = nullptr;
        if (opt.dev_alloc) {
            p_ = opt.dev_alloc(bytes, opt.alloc_user);
            if (!p_) fail(MSP_ERR_NOMEM);
        } else {
            hipError_t e = hipMalloc(&p_, bytes);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                fail(MSP_ERR_NOMEM);
            }
        }
        list.push_back(p_);
        return p_;
    }
    void release(std::vector<void *> &list)
    {
        if (!list.empty()) {
            (void)hipStreamSynchronize(stream);
            if (side) (void)hipStreamSynchronize(side);
            if (gj.aux) (void)hipStreamSynchronize(gj.aux);
            if (gj.main) (void)hipStreamSynchronize(gj.main);
            if (gj.third) (void)hipStreamSynchronize(gj.third);
            if (chain_copy) (void)hipStreamSynchronize(chain_copy);
        }
        for (void *p_ : list) {
            if (opt.dev_free)
                opt.dev_free(p_, opt.alloc_user);
            else
                (void)hipFree(p_);
        }
        list.clear();
    }
    template <typename T, typename A>
    // Device copy of h, queued asynchronously: h must stay alive and unchanged
    // until the copy is done (the runtime may read pageable host memory after
    // the call returns), so callers pass context-owned arrays or synchronise
    // before h goes away.
    T *upload(const std::vector<T, A> &h, std::vector<void *> &list)
    {
        T *d = (T *)dalloc(sizeof(T) * std::max<size_t>(h.size(), 1), list);
        if (!h.empty())
            HIPCHK(hipMemcpyAsync(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice,
                                  copy_stream ? copy_stream : stream));
        return d;
    }
    void sync() { HIPCHK(hipStreamSynchronize(stream)); }
    // flag[0] is written by work on `stream`, flag[1] and flag[2] by work on `side`
    int read_flag(int i = 0)
    {
        hipStream_t s_ = i == 0 ? stream : side;
        HIPCHK(hipMemcpyAsync(flag_host + i, flag + i, sizeof(int), hipMemcpyDeviceToHost, s_));
        HIPCHK(hipStreamSynchronize(s_));
        return flag_host[i];
    }
    void clear_flag(int i = 0)
    {
        HIPCHK(hipMemsetAsync(flag + i, 0, sizeof(int), i == 0 ? stream : side));
    }
    bool fp32() const { return opt.precond_fp32 != 0; }
};

namespace {

void upload_sell(msp_ctx *c, DevSell &S, std::vector<void *> &list)
{
    std::vector<int4> &sl = S.slices_h;
    sl.resize(S.lay.slice_row0.size());
    for (size_t s = 0; s < sl.size(); ++s)
        sl[s] = make_int4(S.lay.slice_row0[s], S.lay.slice_rows[s], S.lay.slice_width[s],
                          S.lay.slice_off[s]);
    S.slices = c->upload(sl, list);
    S.col = c->upload(S.lay.col, list);
    S.src = c->upload(S.lay.src, list);
}

// --------------------------------------------------------------------------
// matrix ingest
// --------------------------------------------------------------------------
void drop_graph(msp_ctx *c);

void build_layout_A(msp_ctx *c)
{
    drop_graph(c);
    c->release(c->allocA);
    const int n = c->n;
    std::vector<int> seg_row = {0, n};
    std::vector<int> src(c->ci.size());
    std::iota(src.begin(), src.end(), 0);
    build_sell(n, seg_row, c->rp, c->ci, src, c->SA.lay);
    upload_sell(c, c->SA, c->allocA);
    const long long E = (long long)c->b * c->b;
    c->valA = (double *)c->dalloc(sizeof(double) * c->SA.lay.slot_lanes * E, c->allocA);
    c->pcol32 = c->fp32()
                    ? (float *)c->dalloc(sizeof(float) * c->SA.lay.slot_lanes * c->b, c->allocA)
                    : nullptr;
    c->rp_d = c->upload(c->rp, c->allocA);
    c->diag_d = c->upload(c->diag_pos, c->allocA);
    c->ci_d = c->upload(c->ci, c->allocA);
}

// --------------------------------------------------------------------------
// preconditioner regeneration
// --------------------------------------------------------------------------
void drop_graph(msp_ctx *c)
{
    if (c->apply_exec) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipGraphExecDestroy(c->apply_exec);
        c->apply_exec = nullptr;
    }
}

void release_B(msp_ctx *c)
{
    drop_graph(c);
    c->release(c->allocB);
    c->lev.clear();
    c->bilu = BiluData();
    c->ns = NStage();
    c->hasB = false;
    c->omega = nullptr;
    c->cinv = c->cY = c->ct = nullptr;
    c->e_nat = c->ybuf = nullptr;
    c->tC = c->tA = c->tB = nullptr;
}

template <typename T>
void *alloc_vec(msp_ctx *c, long long n)
{
    return c->dalloc(sizeof(T) * (size_t)std::max<long long>(n, 1), c->allocB);
}

// Host plan of a smoothed level: positions (color 1 rows ascending, then
// color 2, ... -- the PGS-MC groups) and the slice table of the off-diagonal
// entries in position space.  Pure host work on the pattern, so it runs on
// worker threads; the entries themselves are laid out on the device
// (launch_level_fill) from the level's CSR.
struct LevelLayout {
    std::vector<int> perm, iperm, seg_row;
    SellLayout lay;  // slice table only (col and src are built on the device)
};

void level_layout(int n, const int *rp, const int *ci, const std::vector<int> &color, int g,
                  LevelLayout &O, bool diag_once = false)
{
    O.perm.assign(n, 0);
    O.iperm.assign(n, 0);
    O.seg_row.assign(g + 1, 0);
    {
        std::vector<int> cnt(g + 2, 0);
        for (int i = 0; i < n; ++i) ++cnt[color[i]];
        for (int q = 1; q <= g; ++q) O.seg_row[q] = O.seg_row[q - 1] + cnt[q];
        std::vector<int> f(O.seg_row.begin(), O.seg_row.end() - 1);
        for (int i = 0; i < n; ++i) {
            int t = f[color[i] - 1]++;
            O.perm[i] = t;
            O.iperm[t] = i;
        }
    }
    // off-diagonal entries of the row at each position (diag_once: every row
    // is known to hold its diagonal exactly once)
    std::vector<int> cnt(n);
    if (diag_once) {
        for (int t = 0; t < n; ++t) {
            const int i = O.iperm[t];
            cnt[t] = rp[i + 1] - rp[i] - 1;
        }
    } else {
        for_chunks(n, host_parts(n), [&](int lo, int hi, int) {
            for (int t = lo; t < hi; ++t) {
                const int i = O.iperm[t];
                int m = 0;
                for (int k = rp[i]; k < rp[i + 1]; ++k) m += ci[k] != i;
                cnt[t] = m;
            }
        });
    }
    sell_slices(n, O.seg_row, cnt, O.lay);
}

// Device copy of a level's natural-order CSR (the source of its layout).
struct LevelCsr {
    const int *rp = nullptr, *ci = nullptr;
    const double *val = nullptr;
};

// Lanes per row for the sweeps and residuals of a smoothed level.  A level
// whose rows hold more stored entries than one batch of loads (the coarse
// levels: up to a few dozen) spreads each row over kRowLanes lanes, so a
// sweep's chain of dependent loads is one batch long; short rows (the 7-point
// level 0) keep one thread per row, which moves the fewest bytes.
int row_lanes(const SellLayout &lay)
{
    int w = 0;
    for (int x : lay.slice_width) w = std::max(w, x);
    return w > 8 ? kRowLanes : 1;
}

// Device arrays of level l (its layout computed by level_layout unless it is
// the coarsest level, whose positions are the natural order).
void build_level_device(msp_ctx *c, int l, bool last, LevelLayout *lay, const LevelCsr &csr)
{
    Level &L = c->lev[l];
    const size_t tsz = c->fp32() ? sizeof(float) : sizeof(double);
    L.f = c->dalloc(tsz * std::max(L.n, 1), c->allocB);
    L.x = c->dalloc(tsz * std::max(L.n, 1), c->allocB);
    if (last) {
        L.perm.resize(L.n);
        std::iota(L.perm.begin(), L.perm.end(), 0);
        L.iperm = L.perm;
        L.perm_d = c->upload(L.perm, c->allocB);
        L.iperm_d = L.perm_d;
        return;
    }
    L.r = c->dalloc(tsz * std::max(L.n, 1), c->allocB);
    L.perm = std::move(lay->perm);
    L.iperm = std::move(lay->iperm);
    L.seg_row = std::move(lay->seg_row);
    L.S.lay = std::move(lay->lay);
    L.S.lanes = row_lanes(L.S.lay);
    DevSell &S = L.S;
    S.slices_h.resize(S.lay.slice_row0.size());
    for (size_t q = 0; q < S.slices_h.size(); ++q)
        S.slices_h[q] = make_int4(S.lay.slice_row0[q], S.lay.slice_rows[q], S.lay.slice_width[q],
                                  S.lay.slice_off[q]);
    S.slices = c->upload(S.slices_h, c->allocB);
    const long long sl = std::max<long long>(S.lay.slot_lanes, 1);
    S.col = (int *)c->dalloc(sizeof(int) * sl, c->allocB);
    S.src = (int *)c->dalloc(sizeof(int) * sl, c->allocB);
    void *vals, *diag;
    if (c->fp32()) {
        vals = L.val32 = (float *)c->dalloc(sizeof(float) * sl, c->allocB);
        diag = L.diag32 = (float *)c->dalloc(sizeof(float) * std::max(L.n, 1), c->allocB);
    } else {
        vals = L.val64 = (double *)c->dalloc(sizeof(double) * sl, c->allocB);
        diag = L.diag64 = (double *)c->dalloc(sizeof(double) * std::max(L.n, 1), c->allocB);
    }
    L.perm_d = c->upload(L.perm, c->allocB);
    L.iperm_d = c->upload(L.iperm, c->allocB);
    HIPCHK(launch_level_fill(c->fp32(), (int)S.slices_h.size(), S.slices, csr.rp, csr.ci, csr.val,
                             L.perm_d, L.iperm_d, S.col, S.src, vals, diag,
                             c->copy_stream ? c->copy_stream : c->stream));
}

// The part of the maps between level l and level l + 1 that needs only
// level l's positions (level l built): the coarse row of every fine
// position, and the members of every coarse row (fine positions, natural
// fine index ascending), both in the coarse level's natural order.
void prepare_link(msp_ctx *c, int l, std::vector<void *> &tmp)
{
    Level &L = c->lev[l];
    const int nc = L.nc;
    L.natc_h.resize(L.n);
    for (int t = 0; t < L.n; ++t) L.natc_h[t] = L.agg[L.iperm[t]];
    std::vector<int> &mptr = L.mptr_nat_h, &mem = L.mem_nat_h;
    mptr.assign(nc + 1, 0);
    mem.resize(L.n);
    for (int i = 0; i < L.n; ++i) ++mptr[L.agg[i] + 1];
    for (int J = 0; J < nc; ++J) mptr[J + 1] += mptr[J];
    std::vector<int> f(mptr.begin(), mptr.end() - 1);
    for (int i = 0; i < L.n; ++i) mem[f[L.agg[i]]++] = L.perm[i];
    L.natc_d = c->upload(L.natc_h, tmp);
    L.mptr_nat_d = c->upload(mptr, tmp);
    L.mem_nat_d = c->upload(mem, tmp);
}

// Aggregation maps between level l and level l + 1 in position space (both
// levels built, level l's link prepared): the member offsets by coarse
// position on the host, the rest on the device.
void link_level(msp_ctx *c, int l)
{
    Level &L = c->lev[l];
    const Level &C = c->lev[l + 1];
    std::vector<int> &mptr = L.mem_ptr_h;
    mptr.assign(C.n + 1, 0);
    for (int J = 0; J < C.n; ++J) mptr[C.perm[J] + 1] = L.mptr_nat_h[J + 1] - L.mptr_nat_h[J];
    for (int P = 0; P < C.n; ++P) mptr[P + 1] += mptr[P];
    L.mem_ptr = c->upload(mptr, c->allocB);
    L.agg_pos = (int *)c->dalloc(sizeof(int) * std::max(L.n, 1), c->allocB);
    L.mem = (int *)c->dalloc(sizeof(int) * std::max(L.n, 1), c->allocB);
    HIPCHK(launch_link(L.n, C.n, L.natc_d, L.mptr_nat_d, L.mem_nat_d, C.perm_d, L.mem_ptr,
                       L.agg_pos, L.mem, c->copy_stream ? c->copy_stream : c->stream));
}

// Streams of the coarsest-level solver: the update stream and the stream of
// the Y sweep get all compute units but kGjAuxCUs, the pivot-block stream
// those few, so the short kernels of the pivot chain never queue for slots
// behind the large GEMMs.  Where a compute-unit mask cannot be set the
// streams are plain (same results, less overlap).
constexpr int kGjAuxCUs = 16;
void make_gj_streams(msp_ctx *c)
{
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, c->device));
    const int ncu = prop.multiProcessorCount;
    bool masked = false;
    if (ncu > 4 * kGjAuxCUs) {
        const int words = (ncu + 31) / 32;
        std::vector<uint32_t> mmain(words, 0), maux(words, 0);
        for (int cu = 0; cu < ncu; ++cu) {
            if (cu < kGjAuxCUs)
                maux[cu / 32] |= 1u << (cu % 32);
            else
                mmain[cu / 32] |= 1u << (cu % 32);
        }
        hipStream_t a = nullptr, m = nullptr, t = nullptr;
        if (hipExtStreamCreateWithCUMask(&m, (uint32_t)words, mmain.data()) == hipSuccess &&
            hipExtStreamCreateWithCUMask(&a, (uint32_t)words, maux.data()) == hipSuccess &&
            hipExtStreamCreateWithCUMask(&t, (uint32_t)words, mmain.data()) == hipSuccess) {
            c->gj.main = m;
            c->gj.aux = a;
            c->gj.third = t;
            masked = true;
        } else {
            (void)hipGetLastError();
            if (m) (void)hipStreamDestroy(m);
            if (a) (void)hipStreamDestroy(a);
            if (t) (void)hipStreamDestroy(t);
        }
    }
    if (!masked) {
        HIPCHK(hipStreamCreateWithFlags(&c->gj.main, hipStreamNonBlocking));
        HIPCHK(hipStreamCreateWithFlags(&c->gj.aux, hipStreamNonBlocking));
        HIPCHK(hipStreamCreateWithFlags(&c->gj.third, hipStreamNonBlocking));
    }
    HIPCHK(hipEventCreateWithFlags(&c->gj.ev_start, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->gj.ev_done, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->gj.ev_l, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->gj.ev_y, hipEventDisableTiming));
    for (int i = 0; i < 2; ++i) {
        HIPCHK(hipEventCreateWithFlags(&c->gj.ev_block[i], hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->gj.ev_inv[i], hipEventDisableTiming));
    }
}

// Starts the coarsest-level solver and returns without waiting: the dense
// matrix is scattered on `stream`, and a host thread queues the solver's
// kernels on the solver streams (several thousand launches, off the setup's
// own thread).  The returned future completes once everything is queued;
// then `stream` must wait for gj.ev_done.  flag[0] is set on a singular
// pivot block.  The upload and work buffers go to `tmp`, which the caller
// releases after the streams have drained.
std::future<void> launch_coarse(msp_ctx *c, const Csr &A, std::vector<void *> &tmp)
{
    const int m = A.n;
    c->nL = m;
    c->ldL = (m + 15) & ~15;  // rows 128-byte aligned for the streaming GEMV
    c->cinv = (double *)c->dalloc(sizeof(double) * (size_t)m * c->ldL, c->allocB);
    c->cY = (double *)c->dalloc(sizeof(double) * (size_t)m * c->ldL, c->allocB);
    c->ct = (double *)c->dalloc(sizeof(double) * (size_t)m, c->allocB);
    int *rp = c->upload(A.rp, tmp);
    int *ci = c->upload(A.ci, tmp);
    double *val = c->upload(A.val, tmp);
    double *work = (double *)c->dalloc(sizeof(double) * dense_inverse_work(m), tmp);
    HIPCHK(launch_fill((long long)m * c->ldL, 0.0, c->cinv, c->stream));
    HIPCHK(launch_dense_scatter(m, c->ldL, rp, ci, val, c->cinv, c->stream));
    if (!c->gj.aux) make_gj_streams(c);
    // fill bound of each block step: a row first takes part in the step of
    // the block holding its first stored column, a column in that of its
    // first stored row
    const int steps = (m + kLuBlock - 1) / kLuBlock;
    std::vector<int> rows_end(steps, 0), cols_end(steps, 0);
    {
        std::vector<int> first_row(m, m);
        for (int i = 0; i < m; ++i) {
            const int s0 = A.ci[A.rp[i]] / kLuBlock;  // columns ascending
            rows_end[s0] = std::max(rows_end[s0], i + 1);
            for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
                first_row[A.ci[k]] = std::min(first_row[A.ci[k]], i);
        }
        for (int j = 0; j < m; ++j) {
            const int s0 = first_row[j] / kLuBlock;
            cols_end[s0] = std::max(cols_end[s0], j + 1);
        }
        for (int s = 1; s < steps; ++s) {
            rows_end[s] = std::max(rows_end[s], rows_end[s - 1]);
            cols_end[s] = std::max(cols_end[s], cols_end[s - 1]);
        }
    }
    double *lband =
        (double *)c->dalloc(sizeof(double) * (dense_inverse_lband(m, rows_end.data()) + 1), tmp);
    c->sweepK = dense_inverse_sweep_k(m, cols_end.data());
    c->clear_flag(0);
    HIPCHK(hipEventRecord(c->gj.ev_start, c->stream));
    return std::async(std::launch::async, [c, m, lband, work, re = std::move(rows_end),
                                           ce = std::move(cols_end)]() {
        HIPCHK(dense_inverse(m, c->ldL, c->cinv, c->cY, lband, work, c->flag, c->stream, &c->gj,
                             re.data(), ce.data()));
    });
}

// A posteriori check of the coarsest-level direct solve.  Its block LU makes
// no row interchanges across 128-wide blocks, so a nonsingular matrix whose
// leading blocks are singular or nearly so yields an inaccurate W Y even
// when no pivot is exactly zero.  The setup therefore solves A_L x = f once
// for a fixed f in [-1, 1] and requires every row of the result to satisfy
// |(A_L x - f)_i| <= kCoarseBackwardTol (|A_L| |x| + |f|)_i (a componentwise
// backward error; a factorisation with interchanges gives about 1e-15 on
// these matrices).  On failure the setup reports MSP_ERR_SINGULAR instead of
// returning a direct solve that is not one.
constexpr double kCoarseBackwardTol = 1e-8;
bool coarse_solve_accurate(msp_ctx *c, std::vector<void *> &tmp)
{
    const Csr &A = c->lev.back().A;
    const int m = A.n;
    std::vector<double> f(m), x(m);
    for (int i = 0; i < m; ++i)  // a fixed, sign-changing right-hand side
        f[i] = (double)((unsigned)(i + 1) * 2654435761u % 2001u) / 1000.0 - 1.0;
    double *fd = c->upload(f, tmp);
    double *xd = (double *)c->dalloc(sizeof(double) * (size_t)std::max(m, 1), tmp);
    HIPCHK(launch_coarse_solve<double>(m, c->ldL, kLuBlock, c->cY, c->cinv, fd, c->ct, xd,
                                       c->stream));
    HIPCHK(hipMemcpyAsync(x.data(), xd, sizeof(double) * (size_t)m, hipMemcpyDeviceToHost,
                          c->stream));
    c->sync();
    for (int i = 0; i < m; ++i) {
        double r = -f[i], sc = std::fabs(f[i]);
        for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            r += A.val[k] * x[A.ci[k]];
            sc += std::fabs(A.val[k] * x[A.ci[k]]);
        }
        if (!(std::fabs(r) <= kCoarseBackwardTol * sc)) return false;  // also catches NaN
    }
    return true;
}

// Host-only part of the block ILU(0) setup: elimination order, dependency
// levels, factorisation tasks and the sliced layouts of L and U.  Touches no
// device state, so it can run on a second host thread.
struct BiluPlan {
    std::vector<int> pos;   // elimination position of each block row
    std::vector<int> dsrc;  // per U slice-lane: block row (for the pivot inverses)
};

// color/g: the Alg. 4.2 groups of the block pattern (used for the
// multi-color elimination order).
void bilu_plan(const msp_ctx *c, const std::vector<int> &color, int g, BiluData &D, BiluPlan &P)
{
    const int n = c->n;
    D.ord.resize(n);
    std::vector<int> grp;  // group k of the multi-color order: [grp[k], grp[k+1])
    if (c->opt.bilu_order == 1) {
        std::vector<int> start(g + 2, 0);
        for (int i = 0; i < n; ++i) ++start[color[i] + 1];
        for (int l = 1; l <= g; ++l) start[l + 1] += start[l];
        grp = start;  // colors may start at 0 or 1: an empty group is harmless
        for (int i = 0; i < n; ++i) D.ord[start[color[i]]++] = i;
    } else {
        std::iota(D.ord.begin(), D.ord.end(), 0);
    }
    std::vector<int> &pos = P.pos;
    pos.resize(n);
    for (int t = 0; t < n; ++t) pos[D.ord[t]] = t;
    const int *rp = c->rp.data(), *ci = c->ci.data();
    {
        // the groups of Alg. 4.2 are independent sets, so each is levelled
        // in parallel; any other order takes the sequential pass
        auto levels = [&](bool lower, std::vector<int> &rows, std::vector<int> &ptr) {
            if (grp.empty() ||
                !triangular_levels_groups(n, rp, ci, D.ord, grp, lower, rows, ptr))
                triangular_levels(n, rp, ci, D.ord, lower, rows, ptr);
        };
        auto bwd = std::async(std::launch::async, [&]() { levels(false, D.bwd_rows, D.bwd_ptr); });
        levels(true, D.fwd_rows, D.fwd_ptr);
        bwd.get();
    }
    // slice tables of the lower (forward levels) and upper (backward levels)
    // parts; the entries themselves are laid out on the device (launch_tri_fill)
    const int parts = host_parts(n);
    auto make = [&](const std::vector<int> &rows, const std::vector<int> &lptr, bool lower,
                    SellLayout &lay) {
        std::vector<int> cnt(n);
        for_chunks(n, parts, [&](int lo, int hi, int) {
            for (int r = lo; r < hi; ++r) {
                const int i = rows[r], pi = pos[i];
                int m = 0;
                for (int q = rp[i]; q < rp[i + 1]; ++q) {
                    const int pj = pos[ci[q]];
                    m += lower ? pj < pi : pj > pi;
                }
                cnt[r] = m;
            }
        });
        sell_slices(n, lptr, cnt, lay);
    };
    {
        auto up = std::async(std::launch::async,
                             [&]() { make(D.bwd_rows, D.bwd_ptr, false, D.U.lay); });
        make(D.fwd_rows, D.fwd_ptr, true, D.L.lay);
        up.get();
    }
    P.dsrc.assign(D.U.lay.slice_row0.size() * 64, -1);
    for (size_t s = 0; s < D.U.lay.slice_row0.size(); ++s)
        for (int l = 0; l < D.U.lay.slice_rows[s]; ++l)
            P.dsrc[s * 64 + l] = D.bwd_rows[D.U.lay.slice_row0[s] + l];
    // the solves run on vectors in elimination order
    D.fwd_vpos.resize(n);
    D.bwd_vpos.resize(n);
    for (int r = 0; r < n; ++r) {
        D.fwd_vpos[r] = pos[D.fwd_rows[r]];
        D.bwd_vpos[r] = pos[D.bwd_rows[r]];
    }
    // a forward level whose rows have no lower entries leaves y unchanged
    D.fwd_live.assign(D.L.nseg(), 0);
    for (int g2 = 0; g2 < D.L.nseg(); ++g2)
        for (int q = D.L.lay.seg_slice[g2]; q < D.L.lay.seg_slice[g2 + 1]; ++q)
            if (D.L.lay.slice_width[q] > 0) D.fwd_live[g2] = 1;
}

// Device part: factorise level by level and lay the factors out, on the side
// stream (flag[1] is set on a singular pivot block).  The task arrays go to
// `tmp`, released by the caller after the side stream has drained.
void bilu_device(msp_ctx *c, const double *vals, BiluPlan &P, std::vector<void *> &tmp)
{
    const hipStream_t st = c->side;
    BiluData &D = c->bilu;
    const int n = c->n, b = c->b;
    const long long E = (long long)b * b;
    const int *pos_d = D.pos_d = c->upload(P.pos, c->allocB);
    D.fwd_rows_d = c->upload(D.fwd_rows, c->allocB);
    D.bwd_rows_d = c->upload(D.bwd_rows, c->allocB);
    D.fwd_vpos_d = c->upload(D.fwd_vpos, c->allocB);
    D.bwd_vpos_d = c->upload(D.bwd_vpos, c->allocB);
    BiluTasks T;
    T.rp = c->rp_d;
    T.ci = c->ci_d;
    T.pos = pos_d;
    T.diag_pos = c->diag_d;
    D.F = (double *)c->dalloc(sizeof(double) * (size_t)(c->nnzb * E), c->allocB);
    D.Dinv = (double *)c->dalloc(sizeof(double) * (size_t)(n * E), c->allocB);
    HIPCHK(hipMemcpyAsync(D.F, vals, sizeof(double) * (size_t)(c->nnzb * E),
                          hipMemcpyDeviceToDevice, st));
    c->clear_flag(1);
    for (size_t lv = 0; lv + 1 < D.fwd_ptr.size(); ++lv) {
        T.rows = D.fwd_rows_d + D.fwd_ptr[lv];
        T.nrows = D.fwd_ptr[lv + 1] - D.fwd_ptr[lv];
        HIPCHK(launch_bilu_factor_level(b, T, D.F, D.Dinv, c->flag + 1, st));
    }
    // the two triangles' layouts, built on the device from the pattern
    auto layout = [&](DevSell &S, const int *rows_d, bool lower) {
        S.slices_h.resize(S.lay.slice_row0.size());
        for (size_t q = 0; q < S.slices_h.size(); ++q)
            S.slices_h[q] = make_int4(S.lay.slice_row0[q], S.lay.slice_rows[q],
                                      S.lay.slice_width[q], S.lay.slice_off[q]);
        S.slices = c->upload(S.slices_h, c->allocB);
        const long long sl = std::max<long long>(S.lay.slot_lanes, 1);
        S.col = (int *)c->dalloc(sizeof(int) * sl, c->allocB);
        S.src = (int *)c->dalloc(sizeof(int) * sl, c->allocB);
        HIPCHK(launch_tri_fill((int)S.slices_h.size(), S.slices, rows_d, c->rp_d, c->ci_d, pos_d,
                               lower, S.col, S.src, st));
    };
    layout(D.L, D.fwd_rows_d, true);
    layout(D.U, D.bwd_rows_d, false);
    D.dsrc = c->upload(P.dsrc, c->allocB);
    const long long dsl = (long long)P.dsrc.size();
    if (c->fp32()) {
        D.L32 = (float *)c->dalloc(sizeof(float) * D.L.lay.slot_lanes * E, c->allocB);
        D.U32 = (float *)c->dalloc(sizeof(float) * D.U.lay.slot_lanes * E, c->allocB);
        D.D32 = (float *)c->dalloc(sizeof(float) * dsl * E, c->allocB);
        HIPCHK(launch_gather_blocks(b, D.L.lay.slot_lanes, D.L.src, D.F, nullptr, D.L32, st));
        HIPCHK(launch_gather_blocks(b, D.U.lay.slot_lanes, D.U.src, D.F, nullptr, D.U32, st));
        HIPCHK(launch_gather_blocks(b, dsl, D.dsrc, D.Dinv, nullptr, D.D32, st));
    } else {
        D.L64 = (double *)c->dalloc(sizeof(double) * D.L.lay.slot_lanes * E, c->allocB);
        D.U64 = (double *)c->dalloc(sizeof(double) * D.U.lay.slot_lanes * E, c->allocB);
        D.D64 = (double *)c->dalloc(sizeof(double) * dsl * E, c->allocB);
        HIPCHK(launch_gather_blocks(b, D.L.lay.slot_lanes, D.L.src, D.F, D.L64, nullptr, st));
        HIPCHK(launch_gather_blocks(b, D.U.lay.slot_lanes, D.U.src, D.F, D.U64, nullptr, st));
        HIPCHK(launch_gather_blocks(b, dsl, D.dsrc, D.Dinv, D.D64, nullptr, st));
    }
}

// Block Jacobi R stage: the inverse of every diagonal block (FP64, natural
// block order) on the side stream, with its FP32 copy (flag[1] on a singular
// block).
void block_jacobi_device(msp_ctx *c, const double *vals)
{
    BiluData &D = c->bilu;
    const int n = c->n, b = c->b;
    const long long E = (long long)b * b;
    D.Dinv = (double *)c->dalloc(sizeof(double) * (size_t)(n * E), c->allocB);
    c->clear_flag(1);
    HIPCHK(launch_block_inverse(b, n, c->diag_d, vals, D.Dinv, c->flag + 1, c->side));
    if (c->fp32()) {
        D.D32 = (float *)c->dalloc(sizeof(float) * (size_t)(n * E), c->allocB);
        HIPCHK(launch_from_double<float>((long long)n * E, D.Dinv, D.D32, c->side));
    }
}

// N stage setup on the side stream: the groups of the block graph (cells
// sorted by group, host) and the decoupled concentration blocks (device;
// flag[2] on a singular diagonal block).
void n_stage_device(msp_ctx *c, const double *vals, const std::vector<int> &color, int g)
{
    NStage &S = c->ns;
    const int n = c->n, b = c->b, m = b - 1;
    S.on = true;
    S.grp_ptr.assign(g + 1, 0);
    std::vector<int> &cells = S.cells_h;
    cells.assign(n, 0);
    {
        std::vector<int> cnt(g + 1, 0);
        for (int i = 0; i < n; ++i) ++cnt[color[i]];
        for (int k = 1; k <= g; ++k) S.grp_ptr[k] = S.grp_ptr[k - 1] + cnt[k];
        std::vector<int> f(S.grp_ptr.begin(), S.grp_ptr.end() - 1);
        for (int i = 0; i < n; ++i) cells[f[color[i] - 1]++] = i;
    }
    S.cells = c->upload(cells, c->allocB);
    S.Dn64 = (double *)c->dalloc(sizeof(double) * (size_t)n * m * b, c->allocB);
    S.Ann64 = (double *)c->dalloc(sizeof(double) * (size_t)c->nnzb * m * m, c->allocB);
    c->clear_flag(2);
    HIPCHK(launch_decouple_n(b, c->p, n, c->rp_d, c->ci_d, c->diag_d, vals, S.Dn64, S.Ann64,
                             c->flag + 2, c->side));
    const size_t tsz = c->fp32() ? sizeof(float) : sizeof(double);
    if (c->fp32()) {
        S.Dn32 = (float *)c->dalloc(sizeof(float) * (size_t)n * m * b, c->allocB);
        S.Ann32 = (float *)c->dalloc(sizeof(float) * (size_t)c->nnzb * m * m, c->allocB);
        HIPCHK(launch_from_double<float>((long long)n * m * b, S.Dn64, S.Dn32, c->side));
        HIPCHK(launch_from_double<float>((long long)c->nnzb * m * m, S.Ann64, S.Ann32, c->side));
    }
    S.gN = c->dalloc(tsz * (size_t)n * m, c->allocB);
    S.y = c->dalloc(tsz * (size_t)n * m, c->allocB);
    S.w1 = (double *)c->dalloc(sizeof(double) * (size_t)n * b, c->allocB);
    S.r1 = (double *)c->dalloc(sizeof(double) * (size_t)n * b, c->allocB);
}

// Scope guards for the setup: temporary device buffers are released (after
// both setup streams drained) and uploads return to `stream` on every exit.
struct ReleaseScope {
    msp_ctx *c;
    std::vector<void *> &list;
    ReleaseScope(msp_ctx *c_, std::vector<void *> &l_) : c(c_), list(l_) {}
    ~ReleaseScope() { c->release(list); }
};
struct CopyStreamScope {
    msp_ctx *c;
    CopyStreamScope(msp_ctx *c_, hipStream_t s_) : c(c_) { c->copy_stream = s_; }
    ~CopyStreamScope() { c->copy_stream = nullptr; }
};

// The chain's page-locked staging buffer for level l (at least `bytes`), or
// nullptr if none can be had (the copy then goes to pageable memory).
void *chain_staging(msp_ctx *c, int l, size_t bytes)
{
    std::lock_guard<std::mutex> lock(c->chain_stage_mu);
    if ((int)c->chain_stage.size() <= l) c->chain_stage.resize(l + 1, {nullptr, 0});
    auto &b = c->chain_stage[l];
    if (b.second < bytes) {
        // a buffer of an earlier setup: nothing uses it any more
        if (b.first) (void)hipHostFree(b.first);
        b = {nullptr, 0};
        const size_t sz = bytes + bytes / 8;
        void *p = nullptr;
        if (hipHostMalloc(&p, sz, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        b = {p, sz};
    }
    return b.first;
}

void rebuild_B(msp_ctx *c, const double *vals)
{
    // Level 0 of the previous hierarchy has the same pattern arrays when the
    // pattern has not changed since: its host arrays are taken over (the
    // values are overwritten below) instead of copied and cleared again.
    Csr A0;
    if (!c->lev.empty() && c->lev0_gen == c->pattern_gen && c->lev[0].A.n == c->n &&
        (long long)c->lev[0].A.ci.size() == c->nnzb)
        A0 = std::move(c->lev[0].A);
    release_B(c);
    const int n = c->n, b = c->b;
    double tp = now_ms();
    auto phase = [&](int i) {
        double t = now_ms();
        c->info.phase_ms[i] += t - tp;
        tp = t;
    };
    // decoupling and pressure extraction (device), pressure matrix to the host
    c->omega = (double *)c->dalloc(sizeof(double) * (size_t)n * b, c->allocB);
    std::vector<void *> tmp;
    ReleaseScope release_tmp(c, tmp);
    // H is declared before every future that reads or writes its arrays, so
    // those are joined first on every exit; the level arrays only move
    // (never copy) as the level list grows.
    Hierarchy H;
    static_assert(std::is_nothrow_move_constructible<Csr>::value,
                  "level arrays must move, not copy, when the level list grows");
    double *ap = (double *)c->dalloc(sizeof(double) * (size_t)c->nnzb, tmp);
    c->clear_flag();
    HIPCHK(launch_decouple(b, c->p, n, c->rp_d, c->diag_d, vals, c->omega, ap, c->flag,
                           c->stream));
    if (!c->ev_a0) HIPCHK(hipEventCreateWithFlags(&c->ev_a0, hipEventDisableTiming));
    if (!c->chain_copy) HIPCHK(hipStreamCreateWithFlags(&c->chain_copy, hipStreamNonBlocking));
    HIPCHK(hipEventRecord(c->ev_a0, c->stream));
    if (A0.n != n) {
        A0.n = n;
        A0.rp = c->rp;
        A0.ci = c->ci;
        A0.val.resize(c->nnzb);
    }
    // the decoupled pressure values reach the host on a copy thread; the
    // device chain below does not need them
    std::shared_future<void> a0_ready =
        std::async(std::launch::async, [c, dst = A0.val.data(), ap]() {
            HIPCHK(hipStreamWaitEvent(c->chain_copy, c->ev_a0, 0));
            HIPCHK(hipMemcpyAsync(dst, ap, sizeof(double) * c->nnzb, hipMemcpyDeviceToHost,
                                  c->chain_copy));
            HIPCHK(hipStreamSynchronize(c->chain_copy));
        }).share();
    if (c->read_flag()) fail(MSP_ERR_SINGULAR);
    phase(2);
    // Host setup after the decoupling.  The aggregation chain (pairwise passes
    // and Galerkin products, level by level) is the critical path; the Alg.
    // 4.2 groups of the block pattern (level 0, shared with the multi-color
    // block ILU(0) order) and the host part of the block ILU(0) setup run on
    // worker threads beside it.  Once the coarsest level is known its inverse
    // is queued on `stream`; the groups of the other levels, the level layouts
    // and uploads, and the block ILU(0) factorisation (on the side stream)
    // then overlap that inverse.
    if (!c->side) HIPCHK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    if (!c->ev_main) HIPCHK(hipEventCreateWithFlags(&c->ev_main, hipEventDisableTiming));
    if (!c->ev_side) HIPCHK(hipEventCreateWithFlags(&c->ev_side, hipEventDisableTiming));
    HIPCHK(hipEventRecord(c->ev_main, c->stream));
    HIPCHK(hipStreamWaitEvent(c->side, c->ev_main, 0));
    struct Groups {
        std::vector<int> color;
        int g = 0;
    };
    struct LevelWork {
        Groups G;
        LevelLayout lay;
    };
    const bool level0_smoothed = n > c->opt.max_coarse;
    std::shared_future<Groups> groups0 = std::async(std::launch::async, [c]() {
        Groups G;
        Adjacency adj = build_adjacency(c->n, c->rp.data(), c->ci.data(), c->pattern_sym);
        G.g = vertices_grouping(adj, G.color);
        return G;
    }).share();
    std::future<LevelLayout> layout0;
    if (level0_smoothed)
        layout0 = std::async(std::launch::async, [c, groups0]() {
            const Groups &G = groups0.get();
            LevelLayout O;
            level_layout(c->n, c->rp.data(), c->ci.data(), G.color, G.g, O);
            return O;
        });
    BiluPlan plan;
    std::future<void> planned;
    if (c->opt.full_smoother == 0)
        planned = std::async(std::launch::async, [c, &plan, groups0]() {
            const Groups &G = groups0.get();
            bilu_plan(c, G.color, G.g, c->bilu, plan);
        });
    // groups and layout of each coarser smoothed level start as soon as the
    // chain has produced it
    std::vector<std::future<LevelWork>> work(MSP_MAX_LEVELS);
    // levels that the device chain produced are structurally symmetric (it
    // runs only on a symmetric level 0, and Galerkin products keep that)
    bool device_levels = false;
    const LevelCallback start_level = [&work, &device_levels](int l, int nl, const int *rp,
                                                              const int *ci) {
        if (l == 0) return;  // level 0: the pattern's groups above
        const bool sym = device_levels;
        work[l] = std::async(std::launch::async, [nl, rp, ci, sym]() {
            LevelWork W;
            bool diag_once = false;
            W.G.g = sym ? vertices_grouping_symmetric(nl, rp, ci, W.G.color, &diag_once)
                        : vertices_grouping(build_adjacency(nl, rp, ci, false), W.G.color);
            level_layout(nl, rp, ci, W.G.color, W.G.g, W.lay, diag_once);
            return W;
        });
    };
    // the chain on the device (structurally symmetric patterns), else on the host
    int st = 1;
    if (c->opt.host_chain == 0) {
        if (!c->cap_stream)
            HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        device_levels = true;  // no level callback runs if the chain declines (st == 1)
        st = device_hierarchy(
            A0, c->rp_d, c->ci_d, ap, c->opt.max_coarse, MSP_MAX_LEVELS, 16384, H, start_level,
            [&a0_ready]() { a0_ready.get(); }, c->stream, c->cap_stream, c->chain_copy,
            [c, &tmp](size_t bytes) { return c->dalloc(bytes, tmp); }, fail_hip, c->chain_host,
            [c](int l, size_t bytes) { return chain_staging(c, l, bytes); });
    }
    if (st == 1) {
        device_levels = false;
        a0_ready.get();
        st = build_hierarchy(std::move(A0), c->opt.max_coarse, MSP_MAX_LEVELS, 16384, H, false,
                             start_level);
    }
    if (st == -3) fail(MSP_ERR_SINGULAR);
    if (st == -9) fail(MSP_ERR_COARSE);
    const int nlev = (int)H.A.size();
    std::future<void> coarse_queued = launch_coarse(c, H.A.back(), tmp);
    // zero diagonals on the smoothed levels (the device chain leaves this
    // test to here, behind the coarsest inverse already queued)
    a0_ready.get();
    if (device_levels && check_diagonals(H) != 0) fail(MSP_ERR_SINGULAR);
    phase(3);
    std::vector<LevelLayout> lays(nlev);
    {
        CopyStreamScope on_side(c, c->side);
        // the natural-order CSR of every smoothed level on the device, the
        // source of its layout: level 0 is already there (pattern and
        // decoupled values), the coarser levels are copied up now, while
        // their groups (and the block ILU(0) plan) are still being computed
        std::vector<LevelCsr> csr(nlev);
        for (int l = 0; l + 1 < nlev; ++l) {
            if (l == 0) {
                csr[0] = LevelCsr{c->rp_d, c->ci_d, ap};
            } else {
                const Csr &A = H.A[l];
                csr[l] = LevelCsr{c->upload(A.rp, tmp), c->upload(A.ci, tmp), c->upload(A.val, tmp)};
            }
        }
        // The R stage first: its plan needs only the level-0 groups, so it is
        // usually ready well before the coarse levels' host work, and its
        // uploads and factorisation then overlap that work.
        if (c->opt.full_smoother == 0) {
            planned.get();
            phase(7);
            bilu_device(c, vals, plan, tmp);
        } else {
            block_jacobi_device(c, vals);
        }
        if (c->opt.n_stage == 1 && b > 1) {
            const Groups &G0 = groups0.get();
            n_stage_device(c, vals, G0.color, G0.g);
        }
        phase(6);
        c->lev.resize(nlev);
        for (int l = 0; l < nlev; ++l) {
            Level &L = c->lev[l];
            L.A = std::move(H.A[l]);
            if (l == 0) c->lev0_gen = c->pattern_gen;
            L.n = L.A.n;
            if (l + 1 < nlev) L.agg = std::move(H.agg[l]);
        }
        for (int l = 0; l + 1 < nlev; ++l) c->lev[l].nc = c->lev[l + 1].A.n;
        // Each level's device arrays are built as soon as its host work is
        // done (the largest coarse level's groups usually end last), and the
        // maps between two levels as soon as both exist.
        std::vector<char> built(nlev, 0);
        auto ready = [&](int l) {
            if (l == nlev - 1) return true;
            std::future_status st = l == 0 ? layout0.wait_for(std::chrono::seconds(0))
                                           : work[l].wait_for(std::chrono::seconds(0));
            return st == std::future_status::ready;
        };
        auto build = [&](int l) {
            if (l + 1 < nlev) {
                Groups G;
                if (l == 0) {
                    G = groups0.get();
                    lays[0] = layout0.get();
                } else {
                    LevelWork W = work[l].get();
                    G = std::move(W.G);
                    lays[l] = std::move(W.lay);
                }
                c->lev[l].color = std::move(G.color);
                c->lev[l].g = G.g;
                phase(7);
            }
            build_level_device(c, l, l == nlev - 1, &lays[l], csr[l]);
            if (l + 1 < nlev) prepare_link(c, l, tmp);
            built[l] = 1;
            if (l > 0 && built[l - 1]) link_level(c, l - 1);
            if (l + 1 < nlev && built[l + 1]) link_level(c, l);
            phase(4);
        };
        for (int left = nlev; left > 0;) {
            int next = -1;
            for (int l = 0; l < nlev && next < 0; ++l)
                if (!built[l] && ready(l)) next = l;
            if (next < 0) {  // none ready yet
                std::this_thread::sleep_for(std::chrono::microseconds(100));
                continue;
            }
            build(next);
            --left;
        }
    }
    coarse_queued.get();
    HIPCHK(hipStreamWaitEvent(c->stream, c->gj.ev_done, 0));
    HIPCHK(hipEventRecord(c->ev_side, c->side));
    HIPCHK(hipStreamWaitEvent(c->stream, c->ev_side, 0));
    const int bad_bilu = c->read_flag(1) | (c->ns.on ? c->read_flag(2) : 0);
    phase(6);
    const int bad_coarse = c->read_flag(0) || !coarse_solve_accurate(c, tmp);
    c->release(tmp);
    if (bad_coarse || bad_bilu) fail(MSP_ERR_SINGULAR);
    phase(5);
    const size_t tsz = c->fp32() ? sizeof(float) : sizeof(double);
    c->e_nat = c->dalloc(tsz * n, c->allocB);
    c->ybuf = c->dalloc(tsz * (size_t)n * b, c->allocB);
    c->vin = (double *)c->dalloc(sizeof(double) * (size_t)n * b, c->allocB);
    c->zout = (double *)c->dalloc(sizeof(double) * (size_t)n * b, c->allocB);
    c->io = (ApplyIo *)c->dalloc(sizeof(ApplyIo), c->allocB);
    c->sync();
    c->Bn = n;
    c->Bb = b;
    c->Bp = c->p;
    c->Bnnzb = c->nnzb;
    c->hasB = true;
    c->setup_calls++;
}

// --------------------------------------------------------------------------
// preconditioner apply (Alg. 3.1, reduced form)
// --------------------------------------------------------------------------
template <typename T>
const T *lev_val(const Level &L);
template <>
const double *lev_val<double>(const Level &L) { return L.val64; }
template <>
const float *lev_val<float>(const Level &L) { return L.val32; }
template <typename T>
const T *lev_diag(const Level &L);
template <>
const double *lev_diag<double>(const Level &L) { return L.diag64; }
template <>
const float *lev_diag<float>(const Level &L) { return L.diag32; }

// nu smoothing sweeps on level L (x in place; from_zero: x starts at 0).
// PGS-MC runs colors 1..g (forward) or g..1 (backward) per sweep, Alg. 4.3;
// point Jacobi is direction-free and uses L.r for its residual.
// first_done: the first color of the first forward sweep from zero has
// already been applied (by the restriction into this level).
template <typename T>
void smooth(msp_ctx *c, Level &L, bool forward, bool from_zero, int nu, bool first_done = false)
{
    T *f = (T *)L.f, *x = (T *)L.x;
    const T *val = lev_val<T>(L);
    const T *diag = lev_diag<T>(L);
    if (nu <= 0) {
        if (from_zero) HIPCHK(launch_zero<T>(L.n, x, c->stream));
        return;
    }
    if (c->opt.smoother == 1) {
        const T w = (T)c->opt.jacobi_weight;
        int s0 = 0;
        if (from_zero) {
            HIPCHK(launch_jacobi_first<T>(L.n, w, diag, f, x, c->stream));
            s0 = 1;
        }
        for (int s = s0; s < nu; ++s) {
            HIPCHK(launch_residual<T>(L.S.all(), val, diag, f, x, (T *)L.r, c->stream));
            HIPCHK(launch_jacobi_update<T>(L.n, w, diag, (const T *)L.r, x, c->stream));
        }
        return;
    }
    for (int s = 0; s < nu; ++s) {
        if (forward) {
            int g0 = 0;
            if (from_zero && s == 0) {
                if (!first_done)
                    HIPCHK(launch_gs_first<T>(L.S.all(), L.n, diag, f, x, L.seg_row[0],
                                              L.seg_row[1], c->stream));
                g0 = 1;
            }
            for (int g = g0; g < L.g; ++g)
                HIPCHK(launch_gs_color<T>(L.S.view(g), val, diag, f, x, c->stream));
        } else {
            for (int g = L.g - 1; g >= 0; --g)
                HIPCHK(launch_gs_color<T>(L.S.view(g), val, diag, f, x, c->stream));
        }
    }
}

// first_done: level l's first pre-smoothing color is already applied.
template <typename T>
void vcycle(msp_ctx *c, int l, bool first_done = false)
{
    Level &L = c->lev[l];
    if (l == (int)c->lev.size() - 1) {
        HIPCHK(launch_coarse_solve<T>(L.n, c->ldL, kLuBlock, c->cY, c->cinv, (const T *)L.f,
                                      c->ct, (T *)L.x, c->stream));
        return;
    }
    Level &C = c->lev[l + 1];
    smooth<T>(c, L, true, true, c->opt.nu_pre, first_done);
    HIPCHK(launch_residual<T>(L.S.all(), lev_val<T>(L), lev_diag<T>(L), (const T *)L.f,
                              (const T *)L.x, (T *)L.r, c->stream));
    // a smoothed coarse level whose pre-smoothing starts with a Gauss-Seidel
    // color from zero gets that color from the restriction itself
    const bool fuse = l + 1 < (int)c->lev.size() - 1 && c->opt.smoother == 0 &&
                      c->opt.nu_pre > 0 && C.g > 0;
    if (fuse)
        HIPCHK(launch_restrict_first<T>(C.n, L.mem_ptr, L.mem, (const T *)L.r, (T *)C.f,
                                        C.seg_row[0], C.seg_row[1], lev_diag<T>(C), (T *)C.x,
                                        c->stream));
    else
        HIPCHK(launch_restrict<T>(C.n, L.mem_ptr, L.mem, (const T *)L.r, (T *)C.f, c->stream));
    vcycle<T>(c, l + 1, fuse);
    HIPCHK(launch_prolong<T>(L.n, L.agg_pos, (const T *)C.x, (T *)L.x, c->stream));
    smooth<T>(c, L, false, false, c->opt.nu_post);
}

// The R stage in place on y: block ILU(0) triangular solves, or block Jacobi.
template <typename T>
void bilu_solve(msp_ctx *c, T *y)
{
    BiluData &D = c->bilu;
    if (c->opt.full_smoother == 1) {
        const T *Dj = std::is_same<T, float>::value ? (const T *)D.D32 : (const T *)D.Dinv;
        HIPCHK(launch_block_jacobi<T>(c->b, c->n, Dj, y, c->stream));
        return;
    }
    const T *Lv, *Uv, *Dv;
    if (std::is_same<T, float>::value) {
        Lv = (const T *)D.L32; Uv = (const T *)D.U32; Dv = (const T *)D.D32;
    } else {
        Lv = (const T *)D.L64; Uv = (const T *)D.U64; Dv = (const T *)D.D64;
    }
    for (int s = 0; s < D.L.nseg(); ++s)
        if (D.fwd_live[s])
            HIPCHK(launch_bilu_fwd<T>(c->b, D.L.view(s), D.fwd_vpos_d, Lv, y, c->stream));
    for (int s = 0; s < D.U.nseg(); ++s)
        HIPCHK(launch_bilu_bwd<T>(c->b, D.U.view(s), D.bwd_vpos_d, Uv, Dv, y, c->stream));
}

// Block order of the R stage's vectors: elimination order for block ILU(0),
// natural for block Jacobi.
const int *r_order(const msp_ctx *c)
{
    return c->opt.full_smoother == 0 ? c->bilu.pos_d : nullptr;
}

// io != nullptr: the vectors are read from *io when the kernels run (the
// N stage, which is not captured this way, needs them as arguments).
template <typename T>
void apply_T(msp_ctx *c, const double *v_in, double *z, const ApplyIo *io = nullptr)
{
    Level &L0 = c->lev[0];
    const double *v = v_in;
    NStage &S = c->ns;
    if (S.on) {
        // N stage: y = block GS sweep from 0, w1 = Pi_N y, r1 = v - A w1
        const bool f32 = std::is_same<T, float>::value;
        const T *Dn = f32 ? (const T *)S.Dn32 : (const T *)S.Dn64;
        const T *Ann = f32 ? (const T *)S.Ann32 : (const T *)S.Ann64;
        const int m = c->b - 1;
        HIPCHK(launch_n_rhs<T>(c->b, c->n, Dn, v_in, (T *)S.gN, c->stream));
        HIPCHK(launch_zero<T>(c->n * m, (T *)S.y, c->stream));
        for (size_t k = 0; k + 1 < S.grp_ptr.size(); ++k)
            HIPCHK(launch_bgs_group<T>(c->b, S.grp_ptr[k + 1] - S.grp_ptr[k],
                                       S.cells + S.grp_ptr[k], c->rp_d, c->ci_d, Ann,
                                       (const T *)S.gN, (T *)S.y, c->stream));
        HIPCHK(launch_expand_n<T>(c->b, c->p, c->n, (const T *)S.y, S.w1, c->stream));
        HIPCHK(launch_spmv(c->b, c->SA.all(), c->valA, S.w1, v_in, S.r1, c->stream));
        v = S.r1;
    }
    HIPCHK(launch_decouple_restrict<T>(c->b, c->n, L0.iperm_d, c->omega, v, io, (T *)L0.f,
                                       c->stream));
    vcycle<T>(c, 0);
    HIPCHK(launch_unpermute<T>(c->n, L0.perm_d, (const T *)L0.x, (T *)c->e_nat, c->stream));
    HIPCHK(launch_pcol_residual<T>(c->b, c->p, c->SA.all(), c->valA, c->pcol32, v, io,
                                   (const T *)c->e_nat, r_order(c), (T *)c->ybuf, c->stream));
    bilu_solve<T>(c, (T *)c->ybuf);
    HIPCHK(launch_finish<T>(c->b, c->p, c->n, (const T *)c->ybuf, r_order(c),
                            (const T *)c->e_nat, S.on ? S.w1 : nullptr, z, io, c->stream));
}

void apply_eager(msp_ctx *c, const double *v, double *z, const ApplyIo *io = nullptr)
{
    if (c->fp32())
        apply_T<float>(c, v, z, io);
    else
        apply_T<double>(c, v, z, io);
}

// The captured apply reads its vectors through c->io unless the N stage is
// on; then it works on the fixed vin -> zout and the vectors are copied.
bool apply_via_io(const msp_ctx *c) { return !c->ns.on; }

// Capture the whole preconditioner apply (*io, or vin -> zout) into a HIP
// graph on a private capture stream; nothing runs during capture.  The graph
// holds only kernel nodes.
void capture_apply(msp_ctx *c)
{
    if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t user = c->stream;
    HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    c->stream = c->cap_stream;
    hipGraph_t g = nullptr;
    try {
        if (apply_via_io(c))
            apply_eager(c, nullptr, nullptr, c->io);
        else
            apply_eager(c, c->vin, c->zout);
    } catch (...) {
        c->stream = user;
        (void)hipStreamEndCapture(c->cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    c->stream = user;
    HIPCHK(hipStreamEndCapture(c->cap_stream, &g));
    hipError_t e = hipGraphInstantiate(&c->apply_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->apply_exec = nullptr;
        HIPCHK(e);
    }
}

void apply(msp_ctx *c, const double *v, double *z, bool capture_ok = true)
{
    if (!c->opt.use_graphs || (!c->apply_exec && !capture_ok)) {
        apply_eager(c, v, z);
        return;
    }
    if (!c->apply_exec) capture_apply(c);
    if (apply_via_io(c)) {
        HIPCHK(launch_set_io(c->io, v, z, c->stream));
        HIPCHK(hipGraphLaunch(c->apply_exec, c->stream));
        return;
    }
    const size_t bytes = sizeof(double) * (size_t)c->n * c->b;
    HIPCHK(hipMemcpyAsync(c->vin, v, bytes, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipGraphLaunch(c->apply_exec, c->stream));
    HIPCHK(hipMemcpyAsync(z, c->zout, bytes, hipMemcpyDeviceToDevice, c->stream));
}

void spmv(msp_ctx *c, const double *x, const double *sub, double *y)
{
    HIPCHK(launch_spmv(c->b, c->SA.all(), c->valA, x, sub, y, c->stream));
}

// --------------------------------------------------------------------------
// FGMRES
// --------------------------------------------------------------------------
// Sub-buffer sizes of a Krylov workspace, in doubles, each rounded up to a
// multiple of 32 (256 bytes): V, Z, w, partial, hbuf, ydev.
void krylov_sizes(long long N, int m, size_t sz[6])
{
    auto r = [](long long d) { return (size_t)((d + 31) & ~31LL); };
    sz[0] = r(N * (m + 1));
    sz[1] = r(N * m);
    sz[2] = r(N);
    sz[3] = r((long long)kDotBlocks * (m + 2));
    sz[4] = r(2 * (m + 2) + 2);
    sz[5] = r(m + 1);
}

size_t krylov_bytes(long long N, int m)
{
    size_t sz[6], t = 0;
    krylov_sizes(N, m, sz);
    for (size_t v : sz) t += v;
    return t * sizeof(double);
}

// Carve a Krylov workspace out of one device region of krylov_bytes(N, m).
Krylov krylov_carve(double *base, long long N, int m)
{
    size_t sz[6];
    krylov_sizes(N, m, sz);
    double *ptrs[6];
    for (int i = 0; i < 6; ++i) {
        ptrs[i] = base;
        base += sz[i];
    }
    Krylov K;
    K.V = ptrs[0];
    K.Z = ptrs[1];
    K.w = ptrs[2];
    K.partial = ptrs[3];
    K.hbuf = ptrs[4];
    K.ydev = ptrs[5];
    return K;
}

void ensure_workspace(msp_ctx *c)
{
    const long long N = (long long)c->n * c->b;
    const int m = c->opt.restart;
    if (c->wsN == N && c->wsm == m) return;
    c->release(c->allocW);
    c->kw = krylov_carve((double *)c->dalloc(krylov_bytes(N, m), c->allocW), N, m);
    c->wsN = N;
    c->wsm = m;
}

// One FGMRES(m) solve (Sec. 5) as a sequence of device steps, each ended by
// a copy of its scalars to the context's pinned buffer and an event: the
// host waits for the event, does its part (Givens rotations, stopping test)
// and queues the next step.  Several solves on different contexts can thus
// be advanced in turn by one host thread, each queuing its next step as soon
// as its previous one is done, so their device work overlaps (msp_solve_batch);
// msp_solve runs one.  The steps, kernels and host arithmetic of a solve are
// the same either way.  graph_ok = false keeps the preconditioner apply eager
// unless its graph already exists, so the solve itself creates nothing on the
// device.
struct Fgmres {
    msp_ctx *c = nullptr;
    Krylov K;
    bool graph_ok = true;
    const double *rhs = nullptr;
    double *x = nullptr;
    double rtol = 0.0;
    long long N = 0;
    int m = 0;
    std::vector<double> H, cs, sn, g, y;
    double bnorm = 0.0, tol = 0.0, beta = 0.0, relres = 0.0;
    int iters = 0, restarts = 0, j = 0, status = MSP_OK;
    enum Stage { kBnorm, kBeta, kStep, kDone } stage = kBnorm;
    double t0 = 0.0, ms = 0.0;

    double *h1() const { return K.hbuf; }
    double *h2() const { return K.hbuf + (m + 1); }
    double *hn() const { return K.hbuf + 2 * (m + 1); }
    void mark() { HIPCHK(hipEventRecord(c->ev_step, c->stream)); }
    // queue sum_i v_i^2 into hhost[0]
    void queue_norm2(const double *v)
    {
        HIPCHK(launch_dot_multi(N, 1, v, N, v, K.partial, c->stream));
        HIPCHK(launch_reduce_partials(1, K.partial, K.hbuf, 0, c->stream));
        HIPCHK(hipMemcpyAsync(c->hhost, K.hbuf, sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
        mark();
    }
    void finish(int st)
    {
        status = st;
        stage = kDone;
        ms = now_ms() - t0;
    }
    void start()
    {
        t0 = now_ms();
        N = (long long)c->n * c->b;
        m = c->opt.restart;
        H.assign((size_t)(m + 1) * m, 0.0);
        cs.assign(m, 0.0);
        sn.assign(m, 0.0);
        g.assign(m + 1, 0.0);
        y.assign(m, 0.0);
        for (int q = 0; q < kTimedParts; ++q) {
            c->t_ms[q] = 0.0;
            c->t_calls[q] = 0;
        }
        stage = kBnorm;
        queue_norm2(rhs);
    }
    // Arnoldi step j: z_j = B v_j, w = A z_j, classical Gram-Schmidt twice
    // (h1 = V^T w, w -= V h1, h2 = V^T w, w -= V h2, hn = w^T w; each update
    // pass also forms the next dot products: three passes over V), the
    // coefficients to the host
    void queue_step()
    {
        double *vj = K.V + (size_t)j * N;
        double *zj = K.Z + (size_t)j * N;
        if (c->timing) HIPCHK(hipEventRecord(c->tev[0], c->stream));
        apply(c, vj, zj, graph_ok);
        if (c->timing) HIPCHK(hipEventRecord(c->tev[1], c->stream));
        spmv(c, zj, nullptr, K.w);
        if (c->timing) HIPCHK(hipEventRecord(c->tev[2], c->stream));
        const int nv = j + 1;
        if (nv <= kFusedGsMax) {
            HIPCHK(launch_gs_pass(0, N, nv, K.V, N, nullptr, K.w, K.partial, c->stream));
            HIPCHK(launch_reduce_partials(nv, K.partial, h1(), 0, c->stream));
            HIPCHK(launch_gs_pass(1, N, nv, K.V, N, h1(), K.w, K.partial, c->stream));
            HIPCHK(launch_reduce_partials(nv, K.partial, h2(), 0, c->stream));
            HIPCHK(launch_gs_pass(2, N, nv, K.V, N, h2(), K.w, K.partial, c->stream));
        } else {
            HIPCHK(launch_dot_multi(N, nv, K.V, N, K.w, K.partial, c->stream));
            HIPCHK(launch_reduce_partials(nv, K.partial, h1(), 0, c->stream));
            HIPCHK(launch_axpy_multi(N, nv, K.V, N, h1(), K.w, c->stream));
            HIPCHK(launch_dot_multi(N, nv, K.V, N, K.w, K.partial, c->stream));
            HIPCHK(launch_reduce_partials(nv, K.partial, h2(), 0, c->stream));
            HIPCHK(launch_axpy_multi(N, nv, K.V, N, h2(), K.w, c->stream));
            HIPCHK(launch_dot_multi(N, 1, K.w, N, K.w, K.partial, c->stream));
        }
        HIPCHK(launch_reduce_partials(1, K.partial, hn(), 0, c->stream));
        if (c->timing) HIPCHK(hipEventRecord(c->tev[3], c->stream));
        HIPCHK(hipMemcpyAsync(c->hhost, K.hbuf, sizeof(double) * (2 * (m + 1) + 1),
                              hipMemcpyDeviceToHost, c->stream));
        mark();
    }
    // x += Z y for the k steps of the cycle, then the true residual's norm
    void queue_update(int k)
    {
        for (int i = k - 1; i >= 0; --i) {
            double acc = g[i];
            for (int q = i + 1; q < k; ++q) acc -= H[(size_t)i * m + q] * y[q];
            y[i] = acc / H[(size_t)i * m + i];
        }
        std::memcpy(c->hhost + 2 * (m + 2), y.data(), sizeof(double) * k);
        HIPCHK(hipMemcpyAsync(K.ydev, c->hhost + 2 * (m + 2), sizeof(double) * k,
                              hipMemcpyHostToDevice, c->stream));
        HIPCHK(launch_update_x(N, k, K.Z, N, K.ydev, x, c->stream));
        spmv(c, x, rhs, K.w);
        queue_norm2(K.w);
        ++restarts;
        stage = kBeta;
    }
    // The step just waited for is complete: do the host part, queue the next.
    void advance()
    {
        if (stage == kBnorm) {
            const double bn2 = c->hhost[0];
            if (!std::isfinite(bn2)) return finish(MSP_ERR_NONFINITE);
            bnorm = std::sqrt(bn2);
            if (bnorm == 0.0) {
                HIPCHK(launch_fill(N, 0.0, x, c->stream));
                relres = 0.0;
                return finish(MSP_OK);
            }
            tol = rtol * bnorm;
            spmv(c, x, rhs, K.w);
            queue_norm2(K.w);
            stage = kBeta;
            return;
        }
        if (stage == kBeta) {
            beta = std::sqrt(c->hhost[0]);
            if (!std::isfinite(beta)) return finish(MSP_ERR_NONFINITE);
            relres = beta / bnorm;
            if (beta <= tol) return finish(MSP_OK);
            if (iters >= c->opt.max_iter) return finish(MSP_NOT_CONVERGED);
            HIPCHK(launch_scale(N, K.w, beta, K.V, c->stream));
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            j = 0;
            stage = kStep;
            queue_step();
            return;
        }
        // kStep: the coefficients of Arnoldi step j are in hhost
        if (c->timing) {
            for (int q = 0; q < kTimedParts; ++q) {
                // events 0..3 bracket apply (0,1), SpMV (1,2), Gram-Schmidt (2,3)
                static const int a_[kTimedParts] = {1, 0, 2}, b_[kTimedParts] = {2, 1, 3};
                float e = 0.f;
                HIPCHK(hipEventElapsedTime(&e, c->tev[a_[q]], c->tev[b_[q]]));
                c->t_ms[q] += e;
                c->t_calls[q]++;
            }
        }
        const double *hh1 = c->hhost, *hh2 = c->hhost + (m + 1);
        const double hnorm = std::sqrt(c->hhost[2 * (m + 1)]);
        if (!std::isfinite(hnorm)) return finish(MSP_ERR_NONFINITE);
        for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hh1[i] + hh2[i];
        H[(size_t)(j + 1) * m + j] = hnorm;
        for (int i = 0; i < j; ++i) {
            double a = H[(size_t)i * m + j], bq = H[(size_t)(i + 1) * m + j];
            H[(size_t)i * m + j] = cs[i] * a + sn[i] * bq;
            H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bq;
        }
        double a = H[(size_t)j * m + j], bq = H[(size_t)(j + 1) * m + j];
        double d = std::hypot(a, bq);
        cs[j] = a / d;
        sn[j] = bq / d;
        H[(size_t)j * m + j] = d;
        H[(size_t)(j + 1) * m + j] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        ++iters;
        if (hnorm == 0.0 || std::fabs(g[j + 1]) <= tol || iters >= c->opt.max_iter ||
            j + 1 == m)
            return queue_update(j + 1);
        HIPCHK(launch_scale(N, K.w, hnorm, K.V + (size_t)(j + 1) * N, c->stream));
        ++j;
        queue_step();
    }
};

// Advance every solve of `runs` to its end: wait for each one's queued step
// in turn, do its host part and queue its next step.  A solve that throws is
// ended with the error code; the others go on.
void run_solves(std::vector<Fgmres> &runs)
{
    auto guard = [](Fgmres &r, auto &&f) {
        try {
            f();
        } catch (const MspError &e) {
            r.finish(e.code);
        } catch (const std::bad_alloc &) {
            r.finish(MSP_ERR_NOMEM);
        } catch (...) {
            r.finish(MSP_ERR_HIP);
        }
    };
    for (Fgmres &r : runs) guard(r, [&]() { r.start(); });
    for (bool busy = true; busy;) {
        busy = false;
        for (Fgmres &r : runs) {
            if (r.stage == Fgmres::kDone) continue;
            busy = true;
            guard(r, [&]() {
                HIPCHK(hipEventSynchronize(r.c->ev_step));
                r.advance();
            });
        }
    }
    for (Fgmres &r : runs) {
        const hipError_t e = hipStreamSynchronize(r.c->stream);
        if (e != hipSuccess && r.status >= 0) {
            (void)hipGetLastError();
            r.status = MSP_ERR_HIP;
        }
    }
}

template <typename F>
int guarded(F &&f)
{
    try {
        return f();
    } catch (const MspError &e) {
        return e.code;
    } catch (const std::bad_alloc &) {
        return MSP_ERR_NOMEM;
    } catch (...) {
        return MSP_ERR_HIP;
    }
}

bool valid_options(const msp_options &o)
{
    return o.mu >= 0 && o.restart >= 1 && o.restart <= 200 && o.max_iter >= 1 &&
           o.max_coarse >= 1 && (o.precond_fp32 == 0 || o.precond_fp32 == 1) &&
           (o.bilu_order == 0 || o.bilu_order == 1) && (o.use_graphs == 0 || o.use_graphs == 1) &&
           ((o.dev_alloc == nullptr) == (o.dev_free == nullptr)) &&
           (o.smoother == 0 || o.smoother == 1) && o.nu_pre >= 0 && o.nu_pre <= 8 &&
           o.nu_post >= 0 && o.nu_post <= 8 && (o.full_smoother == 0 || o.full_smoother == 1) &&
           o.jacobi_weight > 0.0 && o.jacobi_weight <= 2.0 && (o.n_stage == 0 || o.n_stage == 1) &&
           (o.host_chain == 0 || o.host_chain == 1);
}

// copy a device sliced layout back to natural block order (host)
template <typename T>
void ungather(msp_ctx *c, const DevSell &S, const T *dev, long long E, T *out)
{
    const long long sl = S.lay.slot_lanes;
    std::vector<T> h((size_t)(sl * E));
    std::vector<int> src((size_t)sl);
    HIPCHK(hipMemcpyAsync(h.data(), dev, sizeof(T) * sl * E, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(src.data(), S.src, sizeof(int) * sl, hipMemcpyDeviceToHost, c->stream));
    c->sync();
    for (long long q = 0; q < sl; ++q) {
        int s = src[q];
        if (s < 0) continue;
        for (long long e = 0; e < E; ++e)
            out[(long long)s * E + e] = h[(q >> 6) * 64 * E + e * 64 + (q & 63)];
    }
}

template <typename T>
void stage_vcycle_T(msp_ctx *c, const double *f, double *e)
{
    Level &L0 = c->lev[0];
    // natural -> positions in the preconditioner precision
    T *tmp = (T *)c->ybuf;  // n*b >= n entries
    HIPCHK(launch_from_double<T>(c->n, f, tmp, c->stream));
    HIPCHK(launch_unpermute<T>(c->n, L0.iperm_d, tmp, (T *)L0.f, c->stream));
    vcycle<T>(c, 0);
    HIPCHK(launch_unpermute<T>(c->n, L0.perm_d, (const T *)L0.x, tmp, c->stream));
    HIPCHK(launch_to_double<T>(c->n, tmp, e, c->stream));
}

template <typename T>
void stage_smooth_T(msp_ctx *c, int level, const double *f, double *x, int forward)
{
    Level &L = c->lev[level];
    T *tmp = (T *)c->ybuf;
    HIPCHK(launch_from_double<T>(L.n, f, tmp, c->stream));
    HIPCHK(launch_unpermute<T>(L.n, L.iperm_d, tmp, (T *)L.f, c->stream));
    HIPCHK(launch_from_double<T>(L.n, x, tmp, c->stream));
    HIPCHK(launch_unpermute<T>(L.n, L.iperm_d, tmp, (T *)L.x, c->stream));
    smooth<T>(c, L, forward != 0, false, 1);
    HIPCHK(launch_unpermute<T>(L.n, L.perm_d, (const T *)L.x, tmp, c->stream));
    HIPCHK(launch_to_double<T>(L.n, tmp, x, c->stream));
}

template <typename T>
void stage_bilu_T(msp_ctx *c, const double *r, double *z)
{
    const long long N = (long long)c->n * c->b;
    const int *ord = r_order(c);
    if (ord)
        HIPCHK(launch_perm_blocks<T>(c->n, c->b, ord, r, (T *)c->ybuf, nullptr, nullptr,
                                     c->stream));
    else
        HIPCHK(launch_from_double<T>(N, r, (T *)c->ybuf, c->stream));
    bilu_solve<T>(c, (T *)c->ybuf);
    if (ord)
        HIPCHK(launch_perm_blocks<T>(c->n, c->b, ord, nullptr, nullptr, z, (const T *)c->ybuf,
                                     c->stream));
    else
        HIPCHK(launch_to_double<T>(N, (const T *)c->ybuf, z, c->stream));
}

// Record a finished solve in its context (iteration count for the adaptive
// setup, info) and return its status.
int record_solve(const Fgmres &r, msp_info *info)
{
    msp_ctx *c = r.c;
    c->info.status = r.status;
    c->info.iterations = r.iters;
    c->info.restarts = r.restarts;
    c->info.rel_true_residual = r.relres;
    c->info.solve_ms = r.ms;
    c->solves++;
    c->info.solves = c->solves;
    c->it_prev = r.iters;
    if (info) *info = c->info;
    return r.status;
}

Fgmres make_run(msp_ctx *c, const Krylov &K, bool graph_ok, const double *rhs, double *x,
                double rtol)
{
    Fgmres r;
    r.c = c;
    r.K = K;
    r.graph_ok = graph_ok;
    r.rhs = rhs;
    r.x = x;
    r.rtol = rtol;
    return r;
}

}  // namespace

// --------------------------------------------------------------------------
// Fixed device scratch of msp_solve_noalloc: the FGMRES workspace of solves
// that may not allocate.  One copy per GPU, held from the library's load until
// the process ends.  Host code never passes `scratch` itself to a kernel (on
// the host that name is only a stand-in for the symbol): it passes the device
// address found by hipGetSymbolAddress once per device, in msp_create.
// --------------------------------------------------------------------------
constexpr size_t kScratchBytes = MSP_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxScratchDevices] = {};

// Look up (once per device, with `dev` current) the device address of this
// GPU's copy of `scratch`.  Returns MSP_OK or MSP_ERR_HIP.
int init_scratch(int dev)
{
    if (dev < 0 || dev >= kMaxScratchDevices) return MSP_ERR_HIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return MSP_OK;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return MSP_ERR_HIP;
    }
    g_scratch_ptr[dev] = (double *)ptr;
    return MSP_OK;
}

double *scratch_ptr(int dev)
{
    if (dev < 0 || dev >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[dev];
}

}  // namespace

// ==========================================================================
// C-ABI
// ==========================================================================
extern "C" {

int msp_default_options(msp_options *opt)
{
    if (!opt) return MSP_ERR_ARG;
    std::memset(opt, 0, sizeof(*opt));
    opt->mu = 0;
    opt->restart = 30;
    opt->max_iter = 1000;
    opt->max_coarse = 10000;
    opt->precond_fp32 = 0;
    opt->bilu_order = 1;
    opt->use_graphs = 1;
    opt->smoother = 0;
    opt->nu_pre = 1;
    opt->nu_post = 1;
    opt->full_smoother = 0;
    opt->jacobi_weight = 1.0;
    opt->n_stage = 0;
    opt->host_chain = 0;
    return MSP_OK;
}

int msp_create(msp_ctx **ctx, const msp_options *opt)
{
    if (!ctx) return MSP_ERR_ARG;
    *ctx = nullptr;
    msp_options o;
    msp_default_options(&o);
    if (opt) o = *opt;
    if (!valid_options(o)) return MSP_ERR_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return MSP_ERR_NO_DEVICE;
    }
    msp_ctx *c = new (std::nothrow) msp_ctx();
    if (!c) return MSP_ERR_NOMEM;
    c->opt = o;
    int st = guarded([&]() {
        HIPCHK(hipGetDevice(&c->device));
        if (int e = init_scratch(c->device)) return e;
        c->stream = (hipStream_t)o.stream;
        HIPCHK(hipEventCreateWithFlags(&c->ev_step, hipEventDisableTiming));
        HIPCHK(hipHostMalloc((void **)&c->hhost, sizeof(double) * 1024, hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void **)&c->flag_host, sizeof(int) * 4, hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void **)&c->chain_host, sizeof(int) * 16, hipHostMallocDefault));
        c->flag = (int *)c->dalloc(sizeof(int) * 4, c->allocW);
        c->wsN = -1;
        return MSP_OK;
    });
    if (st != MSP_OK) {
        msp_destroy(c);
        return st;
    }
    // the workspace list owns only the flag so far; keep it across workspace resizes
    c->allocW.clear();
    *ctx = c;
    return MSP_OK;
}

int msp_destroy(msp_ctx *c)
{
    if (!c) return MSP_OK;
    int st = guarded([&]() {
        // Device memory first: release() synchronises every stream of the
        // context, so the streams must still exist at that point.
        drop_graph(c);
        c->release(c->allocA);
        c->release(c->allocB);
        c->release(c->allocW);
        if (c->flag) {
            if (c->opt.dev_free)
                c->opt.dev_free(c->flag, c->opt.alloc_user);
            else
                (void)hipFree(c->flag);
            c->flag = nullptr;
        }
        auto kill_stream = [](hipStream_t &s) {
            if (s) (void)hipStreamDestroy(s);
            s = nullptr;
        };
        auto kill_event = [](hipEvent_t &e) {
            if (e) (void)hipEventDestroy(e);
            e = nullptr;
        };
        kill_stream(c->cap_stream);
        kill_stream(c->chain_copy);
        kill_event(c->ev_a0);
        for (auto &e : c->tev) kill_event(e);
        kill_event(c->ev_step);
        kill_stream(c->side);
        kill_stream(c->gj.aux);
        kill_stream(c->gj.main);
        kill_stream(c->gj.third);
        kill_event(c->gj.ev_start);
        kill_event(c->gj.ev_done);
        kill_event(c->gj.ev_l);
        kill_event(c->gj.ev_y);
        for (int i = 0; i < 2; ++i) {
            kill_event(c->gj.ev_block[i]);
            kill_event(c->gj.ev_inv[i]);
        }
        kill_event(c->ev_main);
        kill_event(c->ev_side);
        if (c->hhost) (void)hipHostFree(c->hhost);
        if (c->flag_host) (void)hipHostFree(c->flag_host);
        if (c->chain_host) (void)hipHostFree(c->chain_host);
        for (auto &b : c->chain_stage)
            if (b.first) (void)hipHostFree(b.first);
        return MSP_OK;
    });
    delete c;
    return st;
}

int msp_setup(msp_ctx *c, int n, int b, int p, const int *row_ptr, const int *col_ind,
              const double *vals, long long nnzb)
{
    if (!c || !row_ptr || !col_ind || !vals) return MSP_ERR_ARG;
    if (n < 1 || b < 1 || b > 8 || p < 0 || p >= b || nnzb < n) return MSP_ERR_ARG;
    if (nnzb * b * b >= (1LL << 31) * 8LL || nnzb >= (1LL << 31) - 1) return MSP_ERR_ARG;
    const double t0 = now_ms();
    int st = guarded([&]() {
        c->haveA = false;
        for (double &ph : c->info.phase_ms) ph = 0.0;
        // Same sizes as the pattern already ingested (and checked): compare
        // the caller's arrays with the context's device copy on the device;
        // only a new pattern comes to the host to be checked and laid out.
        bool same = false;
        if (c->pattern_ok && n == c->n && b == c->b && p == c->p && nnzb == c->nnzb) {
            c->clear_flag();
            HIPCHK(launch_diff_i32(row_ptr, c->rp_d, (long long)n + 1, c->flag, c->stream));
            HIPCHK(launch_diff_i32(col_ind, c->ci_d, nnzb, c->flag, c->stream));
            same = c->read_flag() == 0;
        }
        std::vector<int> rp, ci;
        if (!same) {
            rp.resize(n + 1);
            ci.resize(nnzb);
            HIPCHK(hipMemcpyAsync(rp.data(), row_ptr, sizeof(int) * (n + 1),
                                  hipMemcpyDeviceToHost, c->stream));
            c->sync();
            if (rp[0] != 0 || (long long)rp[n] != nnzb) fail(MSP_ERR_PATTERN);
            HIPCHK(hipMemcpyAsync(ci.data(), col_ind, sizeof(int) * nnzb, hipMemcpyDeviceToHost,
                                  c->stream));
            c->sync();
            if (check_pattern(n, rp.data(), ci.data(), nnzb) != 0) fail(MSP_ERR_PATTERN);
        }
        const bool layout_changed = !same && (!c->pattern_ok || n != c->n || b != c->b ||
                                              p != c->p || nnzb != c->nnzb || rp != c->rp ||
                                              ci != c->ci);
        if (layout_changed) {
            c->pattern_ok = false;
            ++c->pattern_gen;
            c->n = n;
            c->b = b;
            c->p = p;
            c->nnzb = nnzb;
            c->rp.swap(rp);
            c->ci.swap(ci);
            c->diag_pos.assign(n, -1);
            for (int i = 0; i < n; ++i)
                for (int k = c->rp[i]; k < c->rp[i + 1]; ++k)
                    if (c->ci[k] == i) c->diag_pos[i] = k;
            c->pattern_sym = pattern_symmetric(n, c->rp.data(), c->ci.data());
            build_layout_A(c);
        }
        c->pattern_ok = true;
        const double ti = now_ms();
        c->info.phase_ms[0] = ti - t0;
        c->clear_flag();
        HIPCHK(launch_ingest_bsr(b, p, c->SA.lay.slot_lanes, c->SA.src, vals, c->valA, c->pcol32,
                                 c->flag, c->stream));
        if (c->read_flag()) fail(MSP_ERR_NONFINITE);
        c->info.phase_ms[1] = now_ms() - ti;
        c->haveA = true;
        // adaptive SETUP (Sec. 3.2)
        const bool rebuild = !c->hasB || c->Bn != n || c->Bb != b || c->Bp != p ||
                             c->it_prev < 0 || c->it_prev > c->opt.mu;
        c->info.rebuilt = rebuild ? 1 : 0;
        c->info.rebuild_ms = 0.0;
        if (rebuild) {
            const double t1 = now_ms();
            rebuild_B(c, vals);
            c->info.rebuild_ms = now_ms() - t1;
        }
        return MSP_OK;
    });
    if (st != MSP_OK) {
        try {
            release_B(c);
        } catch (...) {
        }
    }
    c->info.status = st;
    c->info.setup_ms = now_ms() - t0;
    c->info.setup_calls = c->setup_calls;
    c->info.n_levels = (int)c->lev.size();
    for (int l = 0; l < MSP_MAX_LEVELS; ++l) {
        c->info.level_rows[l] = l < (int)c->lev.size() ? c->lev[l].n : 0;
        c->info.n_colors[l] = l < (int)c->lev.size() ? c->lev[l].g : 0;
    }
    c->info.bilu_levels_fwd = c->hasB && !c->bilu.fwd_ptr.empty() ? (int)c->bilu.fwd_ptr.size() - 1 : 0;
    c->info.bilu_levels_bwd = c->hasB && !c->bilu.bwd_ptr.empty() ? (int)c->bilu.bwd_ptr.size() - 1 : 0;
    return st;
}

int msp_solve(msp_ctx *c, const double *rhs, double *x, double rtol, msp_info *info)
{
    if (!c || !rhs || !x || !(rtol > 0.0)) return MSP_ERR_ARG;
    if (!c->hasB || !c->haveA) return MSP_ERR_STATE;
    const int st = guarded([&]() {
        ensure_workspace(c);
        return MSP_OK;
    });
    if (st != MSP_OK) return st;
    std::vector<Fgmres> runs{make_run(c, c->kw, true, rhs, x, rtol)};
    run_solves(runs);
    return record_solve(runs[0], info);
}

int msp_solve_noalloc(msp_ctx *c, const double *rhs, double *x, double rtol, msp_info *info)
{
    if (!c || !rhs || !x || !(rtol > 0.0)) return MSP_ERR_ARG;
    if (!c->hasB || !c->haveA) return MSP_ERR_STATE;
    const long long N = (long long)c->n * c->b;
    if (krylov_bytes(N, c->opt.restart) > kScratchBytes) return MSP_ERR_SCRATCH;
    double *base = scratch_ptr(c->device);
    if (!base) return MSP_ERR_HIP;
    std::vector<Fgmres> runs{make_run(c, krylov_carve(base, N, c->opt.restart), false, rhs, x,
                                      rtol)};
    run_solves(runs);
    return record_solve(runs[0], info);
}

int msp_solve_batch(msp_ctx *const *ctx, int k, const double *const *rhs, double *const *x,
                    double rtol, msp_info *infos)
{
    if (!ctx || !rhs || !x || k < 1 || !(rtol > 0.0)) return MSP_ERR_ARG;
    for (int i = 0; i < k; ++i) {
        if (!ctx[i] || !rhs[i] || !x[i]) return MSP_ERR_ARG;
        for (int q = 0; q < i; ++q)
            if (ctx[q] == ctx[i]) return MSP_ERR_ARG;  // one solve per context
    }
    for (int i = 0; i < k; ++i)
        if (!ctx[i]->hasB || !ctx[i]->haveA) return MSP_ERR_STATE;
    std::vector<Fgmres> runs;
    runs.reserve(k);
    for (int i = 0; i < k; ++i) {
        msp_ctx *c = ctx[i];
        const int st = guarded([&]() {
            ensure_workspace(c);
            return MSP_OK;
        });
        if (st != MSP_OK) return st;
        runs.push_back(make_run(c, c->kw, true, rhs[i], x[i], rtol));
    }
    run_solves(runs);
    int worst = MSP_OK;
    for (int i = 0; i < k; ++i) {
        const int st = record_solve(runs[i], infos ? infos + i : nullptr);
        if (st < 0 && worst >= 0) worst = st;
        if (st == MSP_NOT_CONVERGED && worst == MSP_OK) worst = st;
    }
    return worst;
}

int msp_get_info(msp_ctx *c, msp_info *info)
{
    if (!c || !info) return MSP_ERR_ARG;
    *info = c->info;
    return MSP_OK;
}

int msp_footprint(int n, long long nnzb, int b, const msp_options *opt, size_t *bytes)
{
    if (!bytes || n < 1 || b < 1 || b > 8 || nnzb < n) return MSP_ERR_ARG;
    msp_options o;
    msp_default_options(&o);
    if (opt) o = *opt;
    const double E = (double)b * b;
    const double slots = (double)nnzb * 1.15 + 64.0 * 64;  // slice padding bound
    const double ts = o.precond_fp32 ? 4.0 : 8.0;
    double A = slots * (E * 8 + 8) + (double)n * 8 + (o.precond_fp32 ? slots * b * 4 : 0);
    double amg = 2.0 * ((double)nnzb * 1.15 * (8 + ts + 8)) + 8.0 * n * (3 * ts + 16);
    double coarse = 2 * 8.0 * (double)o.max_coarse * o.max_coarse + 8.0 * o.max_coarse;
    double bilu = (double)nnzb * E * 8 + (double)n * E * 8 + 2 * slots * (E * ts + 8) +
                  (double)n * (E * ts + 24);
    double vecs = (double)n * b * (8 + 2 * ts) + (double)n * 8 * b;
    double krylov = 8.0 * (double)n * b * (2.0 * o.restart + 4) + 8.0 * kDotBlocks * (o.restart + 2);
    double setup_tmp = 8.0 * nnzb + 8.0 * (double)dense_inverse_work(o.max_coarse) +
                       8.0 * (double)dense_inverse_lband(o.max_coarse, nullptr);
    if (o.host_chain == 0 && n > o.max_coarse) setup_tmp += (double)device_chain_bytes(n, nnzb);
    *bytes = (size_t)(A + amg + coarse + bilu + vecs + krylov + setup_tmp + (1 << 20));
    return MSP_OK;
}

const char *msp_status_string(int s)
{
    switch (s) {
    case MSP_OK: return "ok";
    case MSP_ERR_ARG: return "invalid argument";
    case MSP_ERR_PATTERN: return "invalid sparsity pattern";
    case MSP_ERR_SINGULAR: return "singular block, pivot or diagonal";
    case MSP_ERR_NONFINITE: return "non-finite value";
    case MSP_ERR_NOMEM: return "out of memory";
    case MSP_ERR_HIP: return "HIP runtime error";
    case MSP_ERR_NO_DEVICE: return "no GPU device";
    case MSP_ERR_STATE: return "no preconditioner: call msp_setup first";
    case MSP_ERR_COARSE: return "coarsest level exceeds the dense limit";
    case MSP_ERR_SCRATCH:
        return "the solve needs more than the fixed scratch of msp_solve_noalloc";
    case MSP_NOT_CONVERGED: return "not converged within max_iter";
    default: return "unknown status";
    }
}

// ---------------------------- stage entry points --------------------------
int msp_stage_spmv(msp_ctx *c, const double *x, double *y)
{
    if (!c || !x || !y) return MSP_ERR_ARG;
    if (!c->haveA) return MSP_ERR_STATE;
    return guarded([&]() {
        spmv(c, x, nullptr, y);
        c->sync();
        return MSP_OK;
    });
}

int msp_stage_precond(msp_ctx *c, const double *v, double *z)
{
    if (!c || !v || !z) return MSP_ERR_ARG;
    if (!c->hasB || !c->haveA) return MSP_ERR_STATE;
    return guarded([&]() {
        apply(c, v, z);
        c->sync();
        return MSP_OK;
    });
}


int msp_stage_vcycle(msp_ctx *c, const double *f, double *e)
{
    if (!c || !f || !e) return MSP_ERR_ARG;
    if (!c->hasB) return MSP_ERR_STATE;
    return guarded([&]() {
        if (c->fp32())
            stage_vcycle_T<float>(c, f, e);
        else
            stage_vcycle_T<double>(c, f, e);
        c->sync();
        return MSP_OK;
    });
}


int msp_stage_smooth(msp_ctx *c, int level, const double *f, double *x, int forward)
{
    if (!c || !f || !x) return MSP_ERR_ARG;
    if (!c->hasB) return MSP_ERR_STATE;
    if (level < 0 || level >= (int)c->lev.size() - 1) return MSP_ERR_ARG;
    return guarded([&]() {
        if (c->fp32())
            stage_smooth_T<float>(c, level, f, x, forward);
        else
            stage_smooth_T<double>(c, level, f, x, forward);
        c->sync();
        return MSP_OK;
    });
}


int msp_stage_bilu(msp_ctx *c, const double *r, double *z)
{
    if (!c || !r || !z) return MSP_ERR_ARG;
    if (!c->hasB) return MSP_ERR_STATE;
    return guarded([&]() {
        if (c->fp32())
            stage_bilu_T<float>(c, r, z);
        else
            stage_bilu_T<double>(c, r, z);
        c->sync();
        return MSP_OK;
    });
}

int msp_stage_level_info(msp_ctx *c, int level, int *n, long long *nnz, int *ncolors,
                         int *n_next)
{
    if (!c) return MSP_ERR_ARG;
    if (!c->hasB) return MSP_ERR_STATE;
    if (level < 0 || level >= (int)c->lev.size()) return MSP_ERR_ARG;
    const Level &L = c->lev[level];
    if (n) *n = L.n;
    if (nnz) *nnz = L.A.nnz();
    if (ncolors) *ncolors = L.g;
    if (n_next) *n_next = level + 1 < (int)c->lev.size() ? c->lev[level + 1].n : 0;
    return MSP_OK;
}

int msp_stage_get_level(msp_ctx *c, int level, int *row_ptr, int *col_ind, double *val,
                        int *color, int *agg)
{
    if (!c) return MSP_ERR_ARG;
    if (!c->hasB) return MSP_ERR_STATE;
    if (level < 0 || level >= (int)c->lev.size()) return MSP_ERR_ARG;
    const Level &L = c->lev[level];
    const bool last = level == (int)c->lev.size() - 1;
    if (row_ptr) std::memcpy(row_ptr, L.A.rp.data(), sizeof(int) * (L.n + 1));
    if (col_ind) std::memcpy(col_ind, L.A.ci.data(), sizeof(int) * L.A.ci.size());
    if (val) std::memcpy(val, L.A.val.data(), sizeof(double) * L.A.val.size());
    if (!last) {
        if (color) std::memcpy(color, L.color.data(), sizeof(int) * L.n);
        if (agg) std::memcpy(agg, L.agg.data(), sizeof(int) * L.n);
    }
    return MSP_OK;
}

int msp_stage_get_level_f32(msp_ctx *c, int level, float *val)
{
    if (!c || !val) return MSP_ERR_ARG;
    if (!c->hasB || !c->fp32()) return MSP_ERR_STATE;
    if (level < 0 || level >= (int)c->lev.size() - 1) return MSP_ERR_ARG;
    return guarded([&]() {
        const Level &L = c->lev[level];
        // off-diagonal entries from the device layout, diagonal from the device array
        ungather<float>(c, L.S, L.val32, 1, val);
        std::vector<float> d(L.n);
        HIPCHK(hipMemcpyAsync(d.data(), L.diag32, sizeof(float) * L.n, hipMemcpyDeviceToHost,
                              c->stream));
        c->sync();
        for (int t = 0; t < L.n; ++t) {
            int i = L.iperm[t];
            for (int k = L.A.rp[i]; k < L.A.rp[i + 1]; ++k)
                if (L.A.ci[k] == i) val[k] = d[t];
        }
        return MSP_OK;
    });
}

int msp_stage_get_omega(msp_ctx *c, double *omega)
{
    if (!c || !omega) return MSP_ERR_ARG;
    if (!c->hasB) return MSP_ERR_STATE;
    return guarded([&]() {
        HIPCHK(hipMemcpyAsync(omega, c->omega, sizeof(double) * (size_t)c->Bn * c->Bb,
                              hipMemcpyDeviceToHost, c->stream));
        c->sync();
        return MSP_OK;
    });
}

int msp_stage_get_bilu(msp_ctx *c, double *F, double *Dinv)
{
    if (!c) return MSP_ERR_ARG;
    if (!c->hasB) return MSP_ERR_STATE;
    return guarded([&]() {
        const long long E = (long long)c->Bb * c->Bb;
        if (F && c->bilu.F)
            HIPCHK(hipMemcpyAsync(F, c->bilu.F, sizeof(double) * c->Bnnzb * E,
                                  hipMemcpyDeviceToHost, c->stream));
        if (Dinv)
            HIPCHK(hipMemcpyAsync(Dinv, c->bilu.Dinv, sizeof(double) * (size_t)c->Bn * E,
                                  hipMemcpyDeviceToHost, c->stream));
        c->sync();
        return MSP_OK;
    });
}

int msp_stage_get_nstage(msp_ctx *c, double *Dn, double *Ann)
{
    if (!c) return MSP_ERR_ARG;
    if (!c->hasB || !c->ns.on) return MSP_ERR_STATE;
    return guarded([&]() {
        const long long m = c->Bb - 1;
        if (Dn)
            HIPCHK(hipMemcpyAsync(Dn, c->ns.Dn64, sizeof(double) * (size_t)(c->Bn * m * c->Bb),
                                  hipMemcpyDeviceToHost, c->stream));
        if (Ann)
            HIPCHK(hipMemcpyAsync(Ann, c->ns.Ann64, sizeof(double) * (size_t)(c->Bnnzb * m * m),
                                  hipMemcpyDeviceToHost, c->stream));
        c->sync();
        return MSP_OK;
    });
}

int msp_stage_get_bilu_f32(msp_ctx *c, float *F, float *Dinv)
{
    if (!c) return MSP_ERR_ARG;
    if (!c->hasB || !c->fp32()) return MSP_ERR_STATE;
    return guarded([&]() {
        const long long E = (long long)c->Bb * c->Bb;
        BiluData &D = c->bilu;
        if (c->opt.full_smoother == 1) {  // block Jacobi: natural-order inverses only
            if (Dinv)
                HIPCHK(hipMemcpyAsync(Dinv, D.D32, sizeof(float) * (size_t)c->Bn * E,
                                      hipMemcpyDeviceToHost, c->stream));
            c->sync();
            return MSP_OK;
        }
        if (F) {
            // diagonal slots are not stored in the FP32 layouts; fill them from FP64 F
            std::vector<double> F64((size_t)(c->Bnnzb * E));
            HIPCHK(hipMemcpyAsync(F64.data(), D.F, sizeof(double) * c->Bnnzb * E,
                                  hipMemcpyDeviceToHost, c->stream));
            c->sync();
            for (long long q = 0; q < c->Bnnzb * E; ++q) F[q] = (float)F64[q];
            ungather<float>(c, D.L, D.L32, E, F);
            ungather<float>(c, D.U, D.U32, E, F);
        }
        if (Dinv) {
            const long long dsl = (long long)D.U.lay.slice_row0.size() * 64;
            std::vector<float> h((size_t)(dsl * E));
            HIPCHK(hipMemcpyAsync(h.data(), D.D32, sizeof(float) * dsl * E, hipMemcpyDeviceToHost,
                                  c->stream));
            c->sync();
            for (size_t s = 0; s < D.U.lay.slice_row0.size(); ++s)
                for (int l = 0; l < D.U.lay.slice_rows[s]; ++l) {
                    int i = D.bwd_rows[D.U.lay.slice_row0[s] + l];
                    for (long long e = 0; e < E; ++e)
                        Dinv[(long long)i * E + e] = h[s * 64 * E + e * 64 + l];
                }
        }
        return MSP_OK;
    });
}

int msp_stage_repeat(msp_ctx *c, int stage, int reps, const double *in, double *out)
{
    if (!c || reps < 1 || stage < 0 || stage > 6) return MSP_ERR_ARG;
    if ((stage == MSP_STAGE_SPMV || stage == MSP_STAGE_PRECOND) && (!in || !out))
        return MSP_ERR_ARG;
    if (!c->haveA || (stage != MSP_STAGE_SPMV && !c->hasB)) return MSP_ERR_STATE;
    if (stage == MSP_STAGE_GS0 && c->lev.size() < 2) return MSP_ERR_STATE;
    return guarded([&]() {
        const bool f32 = c->fp32();
        if (stage == MSP_STAGE_TRI_SWEEP) {
            // the largest step of the triangular-inverse sweeps of the
            // coarsest solver, W's last block column: C = -A B with A
            // (J P) x k and B k x P, J = the last block, k the depth of U's
            // band there, on scratch operands made on first use and kept
            // with B (P the block size); C is overwritten, so every
            // repetition does the same work
            constexpr int P = kLuBlock;
            const int m = c->nL, kd = std::max(c->sweepK, 1);
            const int mr = std::max((m - 1) / P * P, 1);
            if (!c->tC) {
                c->tC = (double *)c->dalloc(sizeof(double) * (size_t)mr * P, c->allocB);
                c->tA = (double *)c->dalloc(sizeof(double) * (size_t)mr * kd, c->allocB);
                c->tB = (double *)c->dalloc(sizeof(double) * (size_t)kd * P, c->allocB);
                HIPCHK(launch_fill((long long)mr * kd, 1e-3, c->tA, c->stream));
                HIPCHK(launch_fill((long long)kd * P, 1e-3, c->tB, c->stream));
                c->sync();
            }
            for (int r = 0; r < reps; ++r)
                HIPCHK(launch_dgemm(mr, P, kd, c->tA, kd, c->tB, P, c->tC, P, -1.0, 0.0,
                                    c->stream));
            c->sync();
            return MSP_OK;
        }
        for (int r = 0; r < reps; ++r) {
            switch (stage) {
            case MSP_STAGE_SPMV: spmv(c, in, nullptr, out); break;
            case MSP_STAGE_GS0:
                if (f32) smooth<float>(c, c->lev[0], true, false, 1);
                else smooth<double>(c, c->lev[0], true, false, 1);
                break;
            case MSP_STAGE_PRECOND: apply(c, in, out); break;
            case MSP_STAGE_BILU:
                if (f32) bilu_solve<float>(c, (float *)c->ybuf);
                else bilu_solve<double>(c, (double *)c->ybuf);
                break;
            case MSP_STAGE_VCYCLE:
                if (f32) vcycle<float>(c, 0);
                else vcycle<double>(c, 0);
                break;
            case MSP_STAGE_COARSE: {
                Level &L = c->lev.back();
                if (f32)
                    HIPCHK(launch_coarse_solve<float>(L.n, c->ldL, kLuBlock, c->cY, c->cinv,
                                                      (const float *)L.f, c->ct, (float *)L.x,
                                                      c->stream));
                else
                    HIPCHK(launch_coarse_solve<double>(L.n, c->ldL, kLuBlock, c->cY, c->cinv,
                                                       (const double *)L.f, c->ct,
                                                       (double *)L.x, c->stream));
                break;
            }
            }
        }
        c->sync();
        return MSP_OK;
    });
}

}  // extern "C"

int msp_stage_set_timing(msp_ctx *c, int on)
{
    if (!c) return MSP_ERR_ARG;
    return guarded([&] {
        if (on && !c->tev[0])
            for (auto &e : c->tev) HIPCHK(hipEventCreate(&e));
        c->timing = on != 0;
        return MSP_OK;
    });
}

int msp_stage_get_timing(msp_ctx *c, double *ms, int *calls)
{
    if (!c || !ms || !calls) return MSP_ERR_ARG;
    for (int q = 0; q < kTimedParts; ++q) {
        ms[q] = c->t_ms[q];
        calls[q] = c->t_calls[q];
    }
    return MSP_OK;
}
