// Host-side setup of libmsp: pattern checks, the adjacency-graph grouping of
// Alg. 4.1/4.2, pairwise aggregation, Galerkin products, block-ILU(0)
// dependency levels and the sliced-ELL device layout.  Plain C++, no HIP.
#pragma once

#include <cstdint>
#include <functional>
#include <thread>
#include <memory>
#include <utility>
#include <vector>

namespace msp {

// Threads for the host setup loops: min(hardware threads, 8).
int host_threads();
// host_threads() for levels of at least 16384 rows, else 1.
int host_parts(int n);
// Runs f(lo, hi, t) over nparts contiguous, ordered chunks of [0, n) on
// worker threads (chunk t on thread t); results that each chunk keeps apart
// and the caller joins in chunk order are identical to a sequential pass.
template <class F>
void for_chunks(int n, int nparts, F f)
{
    if (nparts <= 1 || n < 2 * nparts) {
        f(0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(nparts - 1);
    for (int t = 1; t < nparts; ++t)
        th.emplace_back([&, t]() {
            f((int)((long long)n * t / nparts), (int)((long long)n * (t + 1) / nparts), t);
        });
    f(0, (int)((long long)n / nparts), 0);
    for (auto &x : th) x.join();
}

// Allocator that leaves scalars uninitialised on resize: a large host array
// is then first touched by the (parallel) code that fills it, instead of by
// one thread zeroing it page by page.
template <typename T>
struct UninitAlloc : std::allocator<T> {
    template <typename U>
    struct rebind {
        using other = UninitAlloc<U>;
    };
    UninitAlloc() = default;
    template <typename U>
    UninitAlloc(const UninitAlloc<U> &) noexcept
    {
    }
    template <typename U>
    void construct(U *p) noexcept
    {
        ::new ((void *)p) U;
    }
    template <typename U, typename... A>
    void construct(U *p, A &&...a)
    {
        ::new ((void *)p) U(std::forward<A>(a)...);
    }
};
using IVecU = std::vector<int, UninitAlloc<int>>;

// Scalar CSR matrix (one AMG level).
struct Csr {
    int n = 0;
    std::vector<int> rp, ci;
    std::vector<double> val;
    long long nnz() const { return rp.empty() ? 0 : rp[n]; }
};

// Returns 0, or -2 (pattern error) for a BSR/CSR pattern that is not
// monotone / in range / strictly ascending per row / holding every diagonal.
int check_pattern(int n, const int *rp, const int *ci, long long nnz);

// Symmetrised off-diagonal adjacency (Sec. 4.1 with A and A^T together),
// sorted neighbour lists.
struct Adjacency {
    int n = 0;
    std::vector<int> ptr, nbr;
    int degree(int i) const { return ptr[i + 1] - ptr[i]; }
};
// known_symmetric skips the symmetry test (pattern_symmetric) when the caller
// already knows the answer.
Adjacency build_adjacency(int n, const int *rp, const int *ci, bool known_symmetric = false);
// True if every stored (i, j) has a stored (j, i).
bool pattern_symmetric(int n, const int *rp, const int *ci);

// Alg. 4.2 (VerticesGrouping) around Alg. 4.1 (VerticesSplitting): color[i]
// in 1..g, returns g.  Largest static degree first, lowest index on ties,
// second-ring candidates before the rest.
int vertices_grouping(const Adjacency &G, std::vector<int> &color);
// The same groups for a structurally symmetric pattern (row_ptr, col_ind),
// read without building the adjacency first.  *diag_once (if given) is set
// when every row was found to hold its diagonal exactly once (always false
// on the fallback path, which does not check).
int vertices_grouping_symmetric(int n, const int *rp, const int *ci, std::vector<int> &color,
                                bool *diag_once = nullptr);

// One pairwise-matching pass; agg[i] in [0, nc), returns nc.
int pairwise_pass(const Csr &A, std::vector<int> &agg);

// Stalled coarsening (the two pairwise passes of a level kept more than 90%
// of its rows): every eligible row alone in its aggregate joins the aggregate
// of its strongest neighbour with s_ij >= 0.25 max_k s_ik among neighbours in
// aggregates of two or more rows (sizes before any move, lowest index among
// equals).  Emptied aggregates are dropped, the rest keep their order; agg is
// renumbered in place and the new count returned.
int absorb_singletons(const Csr &A, std::vector<int> &agg, int nc);

// Galerkin product P^T A P for a piecewise-constant P given by agg; entries
// summed in (fine row, fine column) ascending order, structural pattern.
Csr galerkin(const Csr &A, const std::vector<int> &agg, int nc);

// AMG hierarchy (Sec. 5): levels[0] = A0, ..., levels.back() = coarsest;
// colors/aggs for every non-coarsest level.  Returns 0 or a negative code
// (-3: zero diagonal on a smoothed level, -9: coarsest level too large).
struct Hierarchy {
    std::vector<Csr> A;
    std::vector<std::vector<int>> color, agg;
    std::vector<int> ncolors;
};
// with_colors = false leaves color/ncolors empty (the groups can then be
// computed per level with color_level, e.g. on other threads); on_smoothed
// (if set) is called with (l, n, row_ptr, col_ind) as soon as level l is
// known to be a smoothed level and its pattern is on the host (its values may
// still be on their way).  The pointed-to arrays stay valid until the setup
// that builds H has returned (they may be a copy of H.A[l]'s, e.g. in a
// staging buffer); H.A grows meanwhile, so a callee must not keep a
// reference to the Csr itself.
using LevelCallback = std::function<void(int, int, const int *, const int *)>;
int build_hierarchy(Csr A0, int max_coarse, int max_levels, int max_dense, Hierarchy &H,
                    bool with_colors = true, const LevelCallback &on_smoothed = nullptr);
// The final checks of build_hierarchy: 0, -3 (zero diagonal on a smoothed
// level) or -9 (coarsest level above max_dense rows).
int check_hierarchy(const Hierarchy &H, int max_dense);
// Its first part: 0, or -3 for a zero diagonal on a smoothed level.
int check_diagonals(const Hierarchy &H);
// groups of Alg. 4.2 on one level: fills color, returns g
int color_level(const Csr &A, std::vector<int> &color);

// Dependency levels of a block triangular solve restricted to the stored
// pattern: lower = true gives level(i) = 1 + max level(k) over stored k < i
// in the order `ord` (ord[t] = block row at position t of the elimination
// order); upper = reverse.  Returns the positions sorted by level (stable) and
// the level boundaries.
void triangular_levels(int n, const int *rp, const int *ci, const std::vector<int> &ord,
                       bool lower, std::vector<int> &rows_by_level, std::vector<int> &level_ptr);
// The same levels for an order made of independent groups (no stored entry
// joins two rows of one group): ord holds group k at positions
// [grp[k], grp[k+1]).  The rows of a group are then levelled in parallel,
// group after group.  Returns false, with nothing written, if some stored
// entry joins two rows of one group.
bool triangular_levels_groups(int n, const int *rp, const int *ci, const std::vector<int> &ord,
                              const std::vector<int> &grp, bool lower,
                              std::vector<int> &rows_by_level, std::vector<int> &level_ptr);

// Sliced ELL with 64-row slices that never straddle a segment boundary.
struct SellLayout {
    int nrows = 0;                    // positions
    std::vector<int> seg_slice;       // nseg+1 slice boundaries
    std::vector<int> slice_row0, slice_rows, slice_width, slice_off;  // off in slot-lanes
    long long slot_lanes = 0;         // sum of width*64
    std::vector<int> col;             // [slot_lanes], -1 = padding
    std::vector<int> src;             // [slot_lanes], source entry id or -1
};
// seg_row: segment boundaries over positions (size nseg+1); per position t its
// entries ent_ptr[t]..ent_ptr[t+1] with columns ent_col and source ids ent_src.
// The slice table alone (slice_* arrays, seg_slice, slot_lanes; col and src
// left empty) for positions holding cnt[t] entries each.
void sell_slices(int nrows, const std::vector<int> &seg_row, const std::vector<int> &cnt,
                 SellLayout &L);
void build_sell(int nrows, const std::vector<int> &seg_row, const std::vector<int> &ent_ptr,
                const std::vector<int> &ent_col, const std::vector<int> &ent_src,
                SellLayout &L);

}  // namespace msp
