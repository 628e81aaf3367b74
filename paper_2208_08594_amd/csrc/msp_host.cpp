// Host-side setup of libmsp (see msp_host.h).  Compiled with -ffp-contract=off:
// the aggregation decisions and Galerkin sums must round exactly as written.
#include "msp_host.h"

#include <algorithm>
#include <memory>
#include <numeric>
#include <queue>
#include <thread>

namespace msp {

int host_threads()
{
    unsigned hc = std::thread::hardware_concurrency();
    return (int)std::min(hc ? hc : 1u, 8u);
}

int host_parts(int n)
{
    // worth splitting only for large levels; a few threads are enough
    return n >= 16384 ? host_threads() : 1;
}

int check_pattern(int n, const int *rp, const int *ci, long long nnz)
{
    if (rp[0] != 0 || (long long)rp[n] != nnz) return -2;
    for (int i = 0; i < n; ++i) {
        int a = rp[i], b = rp[i + 1];
        if (b <= a) return -2;
        bool diag = false;
        for (int k = a; k < b; ++k) {
            int j = ci[k];
            if (j < 0 || j >= n) return -2;
            if (k > a && j <= ci[k - 1]) return -2;
            diag |= (j == i);
        }
        if (!diag) return -2;
    }
    return 0;
}

bool pattern_symmetric(int n, const int *rp, const int *ci)
{
    const int parts = host_parts(n);
    std::vector<unsigned char> miss(parts, 0);
    for_chunks(n, parts, [&](int lo, int hi, int t) {
        for (int i = lo; i < hi && !miss[t]; ++i)
            for (int k = rp[i]; k < rp[i + 1]; ++k) {
                const int j = ci[k];
                if (!std::binary_search(ci + rp[j], ci + rp[j + 1], i)) {
                    miss[t] = 1;
                    break;
                }
            }
    });
    for (unsigned char m : miss)
        if (m) return false;
    return true;
}

Adjacency build_adjacency(int n, const int *rp, const int *ci, bool known_symmetric)
{
    // A structurally symmetric pattern is its own symmetrisation: the
    // neighbours of i are row i without the diagonal (already ascending),
    // copied by row chunks in parallel.
    if (known_symmetric || pattern_symmetric(n, rp, ci)) {
        Adjacency G;
        G.n = n;
        G.ptr.assign(n + 1, 0);
        const int parts = host_parts(n);
        for_chunks(n, parts, [&](int lo, int hi, int) {
            for (int i = lo; i < hi; ++i) {
                int m = 0;
                for (int k = rp[i]; k < rp[i + 1]; ++k) m += ci[k] != i;
                G.ptr[i + 1] = m;
            }
        });
        for (int i = 0; i < n; ++i) G.ptr[i + 1] += G.ptr[i];
        G.nbr.resize(G.ptr[n]);
        for_chunks(n, parts, [&](int lo, int hi, int) {
            for (int i = lo; i < hi; ++i) {
                int o = G.ptr[i];
                for (int k = rp[i]; k < rp[i + 1]; ++k)
                    if (ci[k] != i) G.nbr[o++] = ci[k];
            }
        });
        return G;
    }
    // otherwise count both directions of every off-diagonal entry, then sort
    // and drop duplicates
    std::vector<int> cnt(n + 1, 0);
    for (int i = 0; i < n; ++i)
        for (int k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] != i) { ++cnt[i + 1]; ++cnt[ci[k] + 1]; }
    for (int i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    std::vector<int> buf(cnt[n]);
    std::vector<int> fill(cnt.begin(), cnt.end() - 1);
    for (int i = 0; i < n; ++i)
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            int j = ci[k];
            if (j == i) continue;
            buf[fill[i]++] = j;
            buf[fill[j]++] = i;
        }
    Adjacency G;
    G.n = n;
    G.ptr.assign(n + 1, 0);
    G.nbr.reserve(buf.size());
    for (int i = 0; i < n; ++i) {
        auto b0 = buf.begin() + cnt[i], b1 = buf.begin() + cnt[i + 1];
        std::sort(b0, b1);
        auto e = std::unique(b0, b1);
        G.nbr.insert(G.nbr.end(), b0, e);
        G.ptr[i + 1] = (int)G.nbr.size();
    }
    return G;
}

// Alg. 4.2 on a bipartite graph, in closed form.  Let C be a connected
// component with an edge, A its side holding its best vertex (largest
// degree, lowest index), B the other side.  Group 1 is the union of the A
// sides and of the isolated vertices, group 2 the union of the B sides:
//  - a new seed is taken only when no second-ring candidate is open, and it
//    is the best open vertex; a component is untouched until its first
//    seed, so that seed is its best vertex, on side A;
//  - the second ring of a vertex of A lies in A, so every later pick of
//    the component is in A (by induction), and a vertex of A, never adjacent
//    to another, leaves V only by being picked;
//  - every unpicked vertex a of A is a second-ring candidate of an earlier
//    pick: on a path from the seed to a alternating between the sides, the
//    first unpicked vertex of A is in the second ring of the vertex of A
//    before it.  So the component's A is picked whole before the next seed;
//    each vertex of B then has a picked neighbour and has left V;
//  - in group 2 the remaining vertices (the B sides) are independent, so
//    all of them are picked.
// An isolated vertex is picked in group 1 as a seed.  Returns false (and
// leaves color alone) when G has an odd cycle; sets g = 2, or 1 when G has
// no edges.
static bool bipartite_groups(const Adjacency &G, std::vector<int> &color, int &g)
{
    // 2-colouring by a union-find over the edges in natural order (which
    // reads the neighbour lists sequentially): side[v] is v's parity relative
    // to its parent; every root is the lowest vertex of its set
    const int n = G.n;
    std::vector<int> parent(n);
    std::vector<unsigned char> side(n, 0);
    std::iota(parent.begin(), parent.end(), 0);
    auto find = [&](int v, unsigned char &par) {
        unsigned char p = 0;
        int r = v;
        while (parent[r] != r) {
            p ^= side[r];
            r = parent[r];
        }
        // compress: every vertex on the path points at the root
        unsigned char q = p;
        while (parent[v] != r) {
            const int nx = parent[v];
            const unsigned char s = side[v];
            parent[v] = r;
            side[v] = q;
            q ^= s;
            v = nx;
        }
        par = p;
        return r;
    };
    bool edges = false;
    for (int u = 0; u < n; ++u) {
        const int q0 = G.ptr[u], q1 = G.ptr[u + 1];
        if (q0 == q1 || G.nbr[q0] >= u) continue;  // no lower neighbour
        edges = true;
        unsigned char pu;
        int ru = find(u, pu);  // kept current as u's set is merged below
        for (int q = q0; q < q1; ++q) {
            const int w = G.nbr[q];
            if (w >= u) break;  // neighbour lists ascend: each edge once
            unsigned char pw;
            const int rw = find(w, pw);
            if (ru == rw) {
                if (pu == pw) return false;  // odd cycle
            } else if (ru < rw) {
                parent[rw] = ru;
                side[rw] = pu ^ pw ^ 1;
            } else {
                parent[ru] = rw;
                side[ru] = pu ^ pw ^ 1;
                pu ^= side[ru];
                ru = rw;
            }
        }
    }
    // best vertex (largest degree, lowest index) of every component, and
    // its parity
    std::vector<int> best(n, -1);
    std::vector<unsigned char> par(n);
    for (int v = 0; v < n; ++v) {
        const int r = find(v, par[v]);
        const int b = best[r];
        if (b < 0 || G.degree(v) > G.degree(b)) best[r] = v;  // v ascends: ties keep b
    }
    color.assign(n, 0);
    for (int v = 0; v < n; ++v) {
        const int r = parent[v];  // compressed above: the root
        color[v] = par[v] == par[best[r]] ? 1 : 2;
    }
    g = edges ? 2 : 1;
    return true;
}

// The greedy of Alg. 4.2 over the neighbour lists nb[ptr[u] .. ptr[u+1]):
// with REL each entry holds w - u (16 bits: the arrays the greedy reads at
// random then take about half the cache, which keeps it fast while other
// host threads stream through memory), else w.  Cnt holds the counts of
// uncoloured neighbours (at least the largest degree).
template <bool REL, typename Off, typename Cnt>
static int greedy_groups(int n, const int *ptr, const Off *nb, int dmax, std::vector<int> &color)
{
    auto degree = [ptr](int i) { return ptr[i + 1] - ptr[i]; };
    color.assign(n, 0);
    // Static priority: larger |S_i| first, smaller index on ties (Alg. 4.1 picks
    // any vertex of maximal |S_i|; the lowest index makes the choice unique).
    // (a counting sort by degree: buckets from the largest degree down,
    // ascending indices inside a bucket)
    std::vector<int> order(n);
    {
        std::vector<int> start(dmax + 2, 0);
        for (int i = 0; i < n; ++i) ++start[dmax - degree(i) + 1];
        for (int d = 0; d <= dmax; ++d) start[d + 1] += start[d];
        for (int i = 0; i < n; ++i) order[start[dmax - degree(i)]++] = i;
    }
    // Candidates W^ are taken in the same priority, i.e. smallest position in
    // `order` first: a two-level bit set over positions (words of 64
    // positions and a summary bit per word) gives that position quickly.
    std::vector<int> pos(n);
    for (int q = 0; q < n; ++q) pos[order[q]] = q;
    const int nw = (n + 63) / 64, ns = (nw + 63) / 64;
    std::vector<unsigned long long> bits(nw, 0ull), summ(ns, 0ull);
    int nqueued = 0;
    int s_lo = ns;  // no summary word below s_lo is set
    auto hat_push = [&](int v) {
        const int q = pos[v];
        bits[q >> 6] |= 1ull << (q & 63);
        summ[q >> 12] |= 1ull << ((q >> 6) & 63);
        s_lo = std::min(s_lo, q >> 12);
        ++nqueued;
    };
    auto hat_pop = [&]() -> int {  // requires nqueued > 0
        int s = s_lo;
        while (summ[s] == 0ull) ++s;
        s_lo = s;
        const int w = (s << 6) + __builtin_ctzll(summ[s]);
        const int b = __builtin_ctzll(bits[w]);
        bits[w] &= bits[w] - 1;
        if (bits[w] == 0ull) summ[s] &= ~(1ull << (w & 63));
        --nqueued;
        return order[(w << 6) + b];
    };
    // per vertex: kOpen (in V), kQueued (already a second-ring candidate of this
    // group), kScanned (neighbourhood already enumerated for this group), in
    // one byte so that each visit touches one cache line.  A vertex never
    // re-enters V inside a group, so enumerating a neighbourhood a second time
    // cannot add a candidate: each neighbourhood is scanned at most once per
    // group.
    constexpr unsigned char kOpen = 1, kQueued = 2, kScanned = 4;
    std::vector<unsigned char> fl(n);
    // unc[u]: neighbours of u not yet in any group; a vertex with none has
    // nothing left to add to a second ring, so its neighbourhood is skipped
    std::vector<Cnt> unc(n);
    for (int u = 0; u < n; ++u) unc[u] = (Cnt)degree(u);
    // second-ring vertices newly queued for one chosen vertex (each vertex is
    // queued at most once per group)
    std::vector<int> fresh((size_t)std::min<long long>((long long)dmax * dmax, n) + 1);
    unsigned char *F = fl.data();
    auto at = [nb](int u, int q) { return REL ? u + (int)nb[q] : (int)nb[q]; };
    int left = n, g = 0;
    while (left > 0) {
        ++g;  // one call of VerticesSplitting builds group g
        int avail = 0;
        for (int i = 0; i < n; ++i) {
            F[i] = color[i] == 0 ? kOpen : 0;  // V: undetermined vertices
            avail += F[i];
        }
        std::fill(bits.begin(), bits.end(), 0ull);
        std::fill(summ.begin(), summ.end(), 0ull);
        nqueued = 0;
        s_lo = ns;
        size_t cursor = 0;
        while (avail > 0) {
            int v = -1;
            while (nqueued > 0) {  // second-ring candidates W^ that are still in V
                int t = hat_pop();
                if (F[t] & kOpen) { v = t; break; }
            }
            if (v < 0) {
                while (!(F[order[cursor]] & kOpen)) ++cursor;
                v = order[cursor];
            }
            color[v] = g;  // v joins W
            F[v] &= (unsigned char)~kOpen;
            --avail;
            --left;
            const int p0 = ptr[v], p1 = ptr[v + 1];
            for (int q = p0; q < p1; ++q) {  // S_v leaves V (W-bar)
                const int u = at(v, q);
                __builtin_prefetch(&nb[ptr[u]]);  // read by the second ring below
                --unc[u];
                const unsigned char f = F[u];
                avail -= f & kOpen;
                F[u] = f & (unsigned char)~kOpen;
            }
            // second ring enters W^.  Whether a vertex is open is close to
            // random here: the flags are updated without a branch and the
            // newly queued vertices collected, then pushed together.
            int k = 0;
            for (int q = p0; q < p1; ++q) {
                const int u = at(v, q);
                if ((F[u] & kScanned) || unc[u] == 0) continue;
                F[u] |= kScanned;
                const int e = ptr[u + 1];
                for (int t = ptr[u]; t < e; ++t) {
                    const int w = at(u, t);
                    const unsigned char f = F[w];
                    const int take = (f & (kOpen | kQueued)) == kOpen;
                    F[w] = (unsigned char)(f | take * kQueued);
                    fresh[k] = w;
                    k += take;
                }
            }
            for (int i = 0; i < k; ++i) hat_push(fresh[i]);
        }
    }
    return g;
}

int vertices_grouping(const Adjacency &G, std::vector<int> &color)
{
    const int n = G.n;
    int g_bip = 0;
    if (bipartite_groups(G, color, g_bip)) return g_bip;
    int dmax = 0;
    for (int i = 0; i < n; ++i) dmax = std::max(dmax, G.degree(i));
    // 16-bit neighbour offsets where every one fits (levels built from a mesh
    // numbering: neighbours lie within a few planes)
    const long long nnz = (long long)G.nbr.size();
    std::unique_ptr<short[]> nb16(new short[std::max<long long>(nnz, 1)]);
    const int parts = host_parts(n);
    std::vector<unsigned char> fits(parts, 1);
    for_chunks(n, parts, [&](int lo, int hi, int t) {
        for (int u = lo; u < hi && fits[t]; ++u)
            for (int q = G.ptr[u]; q < G.ptr[u + 1]; ++q) {
                const int d = G.nbr[q] - u;
                if (d < -32768 || d > 32767) {
                    fits[t] = 0;
                    break;
                }
                nb16[q] = (short)d;
            }
    });
    const bool rel = dmax <= 65535 &&
                     std::all_of(fits.begin(), fits.end(), [](unsigned char f) { return f != 0; });
    if (rel)
        return greedy_groups<true, short, unsigned short>(n, G.ptr.data(), nb16.get(), dmax, color);
    nb16.reset();
    return greedy_groups<false, int, int>(n, G.ptr.data(), G.nbr.data(), dmax, color);
}

int vertices_grouping_symmetric(int n, const int *rp, const int *ci, std::vector<int> &color,
                                bool *diag_once)
{
    if (diag_once) *diag_once = false;
    // Off-diagonal lists straight from the pattern: when every row stores its
    // diagonal exactly once, row u's neighbours go to [rp[u] - u,
    // rp[u+1] - u - 1), ranges that are disjoint and cover [0, nnz - n).
    // The groups of a bipartite graph come out of the greedy itself here (the
    // closed form gives the same groups, only faster).
    if (n <= 0) return vertices_grouping(build_adjacency(n, rp, ci, true), color);
    const int parts = host_parts(n);
    std::vector<unsigned char> ok(parts, 1);
    std::vector<int> dpart(parts, 0);
    for_chunks(n, parts, [&](int lo, int hi, int t) {
        int dm = 0;
        for (int u = lo; u < hi && ok[t]; ++u) {
            int diag = 0;
            for (int e = rp[u]; e < rp[u + 1]; ++e) {
                const int d = ci[e] - u;
                diag += d == 0;
                if (d < -32768 || d > 32767) ok[t] = 0;
            }
            if (diag != 1) ok[t] = 0;
            dm = std::max(dm, rp[u + 1] - rp[u] - 1);
        }
        dpart[t] = dm;
    });
    const int dmax = *std::max_element(dpart.begin(), dpart.end());
    if (!std::all_of(ok.begin(), ok.end(), [](unsigned char f) { return f != 0; }) ||
        dmax > 65535)
        return vertices_grouping(build_adjacency(n, rp, ci, true), color);
    if (diag_once) *diag_once = true;
    const long long nadj = (long long)rp[n] - n;
    std::unique_ptr<int[]> aptr(new int[(size_t)n + 1]);
    std::unique_ptr<short[]> nb16(new short[(size_t)std::max<long long>(nadj, 1)]);
    for_chunks(n, parts, [&](int lo, int hi, int) {
        for (int u = lo; u < hi; ++u) {
            int q = rp[u] - u;
            aptr[u] = q;
            for (int e = rp[u]; e < rp[u + 1]; ++e)
                if (ci[e] != u) nb16[q++] = (short)(ci[e] - u);
        }
    });
    aptr[n] = (int)nadj;
    return greedy_groups<true, short, unsigned short>(n, aptr.get(), nb16.get(), dmax, color);
}

static inline double entry(const Csr &A, int i, int j)
{
    auto b = A.ci.begin() + A.rp[i], e = A.ci.begin() + A.rp[i + 1];
    auto it = std::lower_bound(b, e, j);
    return (it != e && *it == j) ? A.val[it - A.ci.begin()] : 0.0;
}

int pairwise_pass(const Csr &A, std::vector<int> &agg)
{
    const int n = A.n;
    const int parts = host_parts(n);
    // transpose with values: A^T row j lists (i, a_ij) for stored (i, j), i
    // ascending.  For a structurally symmetric pattern row j of A^T has the
    // columns of row j of A, so only the values are gathered (through the
    // mirror position of each entry, in parallel); otherwise a counting sort
    // over row chunks (per-chunk column counts, offsets in (column, chunk)
    // order, each chunk scattering its rows in order).
    std::vector<int> tp;
    std::unique_ptr<int[]> ti_own;
    const int *ti = A.ci.data();
    std::unique_ptr<double[]> tv(new double[A.ci.size() + 1]);
    bool symmetric = true;
    {
        std::vector<unsigned char> miss(parts, 0);
        for_chunks(n, parts, [&](int lo, int hi, int t) {
            for (int i = lo; i < hi && !miss[t]; ++i)
                for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
                    // rows are short: a forward scan finds the mirror entry
                    const int j = A.ci[k];
                    int q = A.rp[j];
                    const int qe = A.rp[j + 1];
                    while (q < qe && A.ci[q] < i) ++q;
                    if (q == qe || A.ci[q] != i) {
                        miss[t] = 1;
                        break;
                    }
                    tv[k] = A.val[q];
                }
        });
        for (unsigned char m : miss) symmetric = symmetric && !m;
    }
    if (symmetric) {
        tp = A.rp;
    } else {
        tp.assign(n + 1, 0);
        ti_own.reset(new int[A.ci.size() + 1]);
        std::vector<int> hist((size_t)n * parts, 0);  // [column][chunk]
        for_chunks(n, parts, [&](int lo, int hi, int t) {
            for (int k = A.rp[lo]; k < A.rp[hi]; ++k) ++hist[(size_t)A.ci[k] * parts + t];
        });
        int run = 0;
        for (int c = 0; c < n; ++c) {
            tp[c] = run;
            int *h = &hist[(size_t)c * parts];
            for (int t = 0; t < parts; ++t) {
                const int v = h[t];
                h[t] = run;
                run += v;
            }
        }
        tp[n] = run;
        for_chunks(n, parts, [&](int lo, int hi, int t) {
            for (int i = lo; i < hi; ++i)
                for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
                    const int q = hist[(size_t)A.ci[k] * parts + t]++;
                    ti_own[q] = i;
                    tv[q] = A.val[k];
                }
        });
        ti = ti_own.get();
    }
    // symmetrised neighbours of i = merge of row i of A and row i of A^T
    // (both ascending), with s_ij = -(a_ij + a_ji)/2, built per row chunk at
    // the bound offset start[i] = rp[i] + tp[i] (a row has at most
    // rowlen(A) + rowlen(A^T) neighbours)
    std::vector<double> smax(n, 0.0);
    std::vector<unsigned char> eligible(n, 0);
    const size_t bound = (size_t)A.rp[n] + (size_t)tp[n];
    std::unique_ptr<int[]> nbr(new int[bound + 1]);
    std::unique_ptr<double[]> s(new double[bound + 1]);
    std::vector<int> cnt(n, 0);
    for_chunks(n, parts, [&](int lo, int hi, int) {
        for (int i = lo; i < hi; ++i) {
            int a = A.rp[i], ae = A.rp[i + 1], q = tp[i], te = tp[i + 1];
            bool coupled = false, any = false;
            double mx = 0.0;
            size_t o = (size_t)A.rp[i] + (size_t)tp[i];
            const size_t before = o;
            while (a < ae || q < te) {
                int ja = a < ae ? A.ci[a] : n, jt = q < te ? ti[q] : n;
                int j = ja < jt ? ja : jt;
                double aij = 0.0, aji = 0.0;
                if (ja == j) { aij = A.val[a]; ++a; }
                if (jt == j) { aji = tv[q]; ++q; }
                if (j == i) continue;
                if (ja == j && aij != 0.0) coupled = true;
                double sij = -(aij + aji) / 2.0;
                nbr[o] = j;
                s[o] = sij;
                ++o;
                if (!any || sij > mx) mx = sij;
                any = true;
            }
            cnt[i] = (int)(o - before);
            smax[i] = mx;
            eligible[i] = coupled && any && mx > 0.0;
        }
    });
    // Candidates of each eligible row: eligible neighbours j with
    // s_ij >= 0.25 max_k s_ik, ordered by s_ij descending, then j ascending.
    // The first one still free is then the strongest free eligible partner
    // (lowest index among equals), exactly what a scan of the row picks.
    std::vector<int> ncand(n, 0);
    for_chunks(n, parts, [&](int lo, int hi, int) {
        for (int i = lo; i < hi; ++i) {
            if (!eligible[i]) continue;
            const double thr = 0.25 * smax[i];
            const size_t b0 = (size_t)A.rp[i] + (size_t)tp[i];
            int m = 0;
            for (int q = 0; q < cnt[i]; ++q) {
                const int j = nbr[b0 + q];
                const double sj = s[b0 + q];
                if (!eligible[j] || !(sj >= thr)) continue;
                // insertion into the sorted prefix [b0, b0 + m)
                int r = m;
                while (r > 0 && (s[b0 + r - 1] < sj || (s[b0 + r - 1] == sj && nbr[b0 + r - 1] > j))) {
                    nbr[b0 + r] = nbr[b0 + r - 1];
                    s[b0 + r] = s[b0 + r - 1];
                    --r;
                }
                nbr[b0 + r] = j;
                s[b0 + r] = sj;
                ++m;
            }
            ncand[i] = m;
        }
    });
    agg.assign(n, -1);
    int nc = 0;
    for (int i = 0; i < n; ++i) {
        if (agg[i] >= 0) continue;
        int best = -1;
        const int *cb = nbr.get() + (size_t)A.rp[i] + (size_t)tp[i];
        for (int q = 0; q < ncand[i]; ++q)
            if (agg[cb[q]] < 0) {
                best = cb[q];
                break;
            }
        agg[i] = nc;
        if (best >= 0) agg[best] = nc;
        ++nc;
    }
    return nc;
}

Csr galerkin(const Csr &A, const std::vector<int> &agg, int nc)
{
    const int n = A.n;
    std::vector<int> mptr(nc + 1, 0), mem(n);
    for (int i = 0; i < n; ++i) ++mptr[agg[i] + 1];
    for (int I = 0; I < nc; ++I) mptr[I + 1] += mptr[I];
    {
        std::vector<int> f(mptr.begin(), mptr.end() - 1);
        for (int i = 0; i < n; ++i) mem[f[agg[i]]++] = i;  // ascending fine index
    }
    // Coarse rows in ordered chunks, each with its own accumulator.  Row I has
    // at most as many entries as its member rows hold together, so a chunk
    // writes from that bound offset into memory allocated here; the chunks
    // are then packed in order.
    const int parts = host_parts(n);
    std::vector<long long> bnd(nc + 1, 0);
    for (int I = 0; I < nc; ++I) {
        long long w = 0;
        for (int m = mptr[I]; m < mptr[I + 1]; ++m) w += A.rp[mem[m] + 1] - A.rp[mem[m]];
        bnd[I + 1] = bnd[I] + w;
    }
    Csr C;
    C.n = nc;
    C.ci.resize(bnd[nc]);
    C.val.resize(bnd[nc]);
    std::vector<int> rowlen(nc, 0), chunk_lo(parts + 1, nc);
    for_chunks(nc, parts, [&](int lo, int hi, int t) {
        chunk_lo[t] = lo;
        std::vector<int> slot(nc, -1), cols, idx;
        std::vector<double> vals;
        long long o = bnd[lo];
        for (int I = lo; I < hi; ++I) {
            cols.clear();
            vals.clear();
            for (int m = mptr[I]; m < mptr[I + 1]; ++m) {
                int i = mem[m];
                for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
                    int J = agg[A.ci[k]];
                    if (slot[J] < 0) {
                        slot[J] = (int)cols.size();
                        cols.push_back(J);
                        vals.push_back(A.val[k]);
                    } else {
                        vals[slot[J]] = vals[slot[J]] + A.val[k];
                    }
                }
            }
            idx.resize(cols.size());
            std::iota(idx.begin(), idx.end(), 0);
            std::sort(idx.begin(), idx.end(), [&](int a, int b) { return cols[a] < cols[b]; });
            for (int q : idx) {
                C.ci[o] = cols[q];
                C.val[o] = vals[q];
                ++o;
                slot[cols[q]] = -1;
            }
            rowlen[I] = (int)cols.size();
        }
    });
    C.rp.assign(nc + 1, 0);
    for (int I = 0; I < nc; ++I) C.rp[I + 1] = C.rp[I] + rowlen[I];
    for (int t = 0; t < parts && chunk_lo[t] < nc; ++t) {
        const int lo = chunk_lo[t], hi = chunk_lo[t + 1];
        const long long from = bnd[lo], len = C.rp[hi] - C.rp[lo];
        if (from != C.rp[lo] && len) {
            std::copy(C.ci.begin() + from, C.ci.begin() + from + len, C.ci.begin() + C.rp[lo]);
            std::copy(C.val.begin() + from, C.val.begin() + from + len, C.val.begin() + C.rp[lo]);
        }
    }
    C.ci.resize(C.rp[nc]);
    C.val.resize(C.rp[nc]);
    return C;
}

int absorb_singletons(const Csr &A, std::vector<int> &agg, int nc)
{
    const int n = A.n;
    const size_t nnz = A.ci.size();
    // A^T with values (counting sort), for the symmetrised strengths
    std::vector<int> tp(n + 1, 0), ti(nnz);
    std::vector<double> tv(nnz);
    for (size_t k = 0; k < nnz; ++k) ++tp[A.ci[k] + 1];
    for (int j = 0; j < n; ++j) tp[j + 1] += tp[j];
    {
        std::vector<int> f(tp.begin(), tp.end() - 1);
        for (int i = 0; i < n; ++i)
            for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
                const int q = f[A.ci[k]]++;
                ti[q] = i;
                tv[q] = A.val[k];
            }
    }
    std::vector<int> size(nc, 0), target(agg);
    for (int i = 0; i < n; ++i) ++size[agg[i]];
    std::vector<int> nb;
    std::vector<double> sv;
    for (int i = 0; i < n; ++i) {
        if (size[agg[i]] != 1) continue;
        // neighbours of i in the symmetrised pattern, ascending, with s_ij
        nb.clear();
        sv.clear();
        bool coupled = false, any = false;
        double mx = 0.0;
        int a = A.rp[i], ae = A.rp[i + 1], q = tp[i], te = tp[i + 1];
        while (a < ae || q < te) {
            const int ja = a < ae ? A.ci[a] : n, jt = q < te ? ti[q] : n;
            const int j = ja < jt ? ja : jt;
            double aij = 0.0, aji = 0.0;
            if (ja == j) { aij = A.val[a]; ++a; }
            if (jt == j) { aji = tv[q]; ++q; }
            if (j == i) continue;
            if (ja == j && aij != 0.0) coupled = true;
            const double sij = -(aij + aji) / 2.0;
            nb.push_back(j);
            sv.push_back(sij);
            if (!any || sij > mx) mx = sij;
            any = true;
        }
        if (!(coupled && any && mx > 0.0)) continue;
        int best = -1;
        double bs = 0.0;
        for (size_t t = 0; t < nb.size(); ++t) {
            if (size[agg[nb[t]]] < 2) continue;
            if (sv[t] >= 0.25 * mx && (best < 0 || sv[t] > bs)) {
                best = nb[t];
                bs = sv[t];
            }
        }
        if (best >= 0) target[i] = agg[best];
    }
    std::vector<int> map(nc, -1);
    for (int i = 0; i < n; ++i) map[target[i]] = 0;
    int k = 0;
    for (int c = 0; c < nc; ++c)
        if (map[c] == 0) map[c] = k++;
    for (int i = 0; i < n; ++i) agg[i] = map[target[i]];
    return k;
}

int color_level(const Csr &A, std::vector<int> &color)
{
    Adjacency G = build_adjacency(A.n, A.rp.data(), A.ci.data());
    return vertices_grouping(G, color);
}

int build_hierarchy(Csr A0, int max_coarse, int max_levels, int max_dense, Hierarchy &H,
                    bool with_colors, const LevelCallback &on_smoothed)
{
    H = Hierarchy();
    H.A.push_back(std::move(A0));
    for (int l = 0;; ++l) {
        const Csr &cur = H.A[l];
        bool last = cur.n <= max_coarse || l == max_levels - 1 ||
                    (l > 0 && (double)cur.n > 0.9 * (double)H.A[l - 1].n);
        if (last) break;
        if (on_smoothed) on_smoothed(l, cur.n, cur.rp.data(), cur.ci.data());
        if (with_colors) {
            std::vector<int> color;
            H.ncolors.push_back(color_level(cur, color));
            H.color.push_back(std::move(color));
        }
        std::vector<int> a1, a2;
        int nc1 = pairwise_pass(cur, a1);
        Csr M1 = galerkin(cur, a1, nc1);
        int nc2 = pairwise_pass(M1, a2);
        Csr Cn = galerkin(M1, a2, nc2);
        std::vector<int> agg(cur.n);
        for (int i = 0; i < cur.n; ++i) agg[i] = a2[a1[i]];
        if ((double)nc2 > 0.9 * (double)cur.n) {
            // stalled: absorb singletons, then one Galerkin product on A_l
            const int nc3 = absorb_singletons(cur, agg, nc2);
            if (nc3 < nc2) Cn = galerkin(cur, agg, nc3);
        }
        H.agg.push_back(std::move(agg));
        H.A.push_back(std::move(Cn));
    }
    return check_hierarchy(H, max_dense);
}

int check_diagonals(const Hierarchy &H)
{
    for (size_t l = 0; l + 1 < H.A.size(); ++l) {
        const Csr &A = H.A[l];
        const int parts = host_parts(A.n);
        std::vector<unsigned char> zero(parts, 0);
        for_chunks(A.n, parts, [&](int lo, int hi, int t) {
            for (int i = lo; i < hi; ++i)
                if (entry(A, i, i) == 0.0) {
                    zero[t] = 1;
                    break;
                }
        });
        for (unsigned char z : zero)
            if (z) return -3;
    }
    return 0;
}

int check_hierarchy(const Hierarchy &H, int max_dense)
{
    const int st = check_diagonals(H);
    if (st) return st;
    if (H.A.back().n > max_dense) return -9;
    return 0;
}

void triangular_levels(int n, const int *rp, const int *ci, const std::vector<int> &ord,
                       bool lower, std::vector<int> &rows_by_level, std::vector<int> &level_ptr)
{
    std::vector<int> pos(n), lev(n, 0);
    for (int t = 0; t < n; ++t) pos[ord[t]] = t;
    int maxlev = 0;
    for (int s = 0; s < n; ++s) {
        int t = lower ? s : n - 1 - s;
        int i = ord[t];
        int l = 0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            int j = ci[k];
            bool dep = lower ? pos[j] < t : pos[j] > t;
            if (dep) l = std::max(l, lev[j] + 1);
        }
        lev[i] = l;
        maxlev = std::max(maxlev, l);
    }
    level_ptr.assign(maxlev + 2, 0);
    for (int i = 0; i < n; ++i) ++level_ptr[lev[i] + 1];
    for (int l = 0; l <= maxlev; ++l) level_ptr[l + 1] += level_ptr[l];
    rows_by_level.assign(n, 0);
    std::vector<int> f(level_ptr.begin(), level_ptr.end() - 1);
    for (int s = 0; s < n; ++s) {
        int i = ord[lower ? s : n - 1 - s];
        rows_by_level[f[lev[i]]++] = i;
    }
}

bool triangular_levels_groups(int n, const int *rp, const int *ci, const std::vector<int> &ord,
                              const std::vector<int> &grp, bool lower,
                              std::vector<int> &rows_by_level, std::vector<int> &level_ptr)
{
    const int g = (int)grp.size() - 1;
    std::vector<int> pos(n), lev(n, 0);
    for_chunks(n, host_parts(n), [&](int lo, int hi, int) {
        for (int t = lo; t < hi; ++t) pos[ord[t]] = t;
    });
    const int parts = host_parts(n);
    std::vector<int> pmax(parts, 0);
    std::vector<char> pbad(parts, 0);
    for (int q = 0; q < g; ++q) {
        const int k = lower ? q : g - 1 - q;
        const int g0 = grp[k], g1 = grp[k + 1];
        // every dependency of the group lies in groups already levelled
        for_chunks(g1 - g0, parts, [&](int lo, int hi, int w) {
            int mx = pmax[w];
            bool bad = false;
            for (int t = g0 + lo; t < g0 + hi; ++t) {
                const int i = ord[t];
                int l = 0;
                for (int e = rp[i]; e < rp[i + 1]; ++e) {
                    const int pj = pos[ci[e]];
                    if (lower ? pj < t : pj > t) {
                        if (pj >= g0 && pj < g1) {
                            bad = true;
                            continue;
                        }
                        l = std::max(l, lev[ci[e]] + 1);
                    }
                }
                lev[i] = l;
                mx = std::max(mx, l);
            }
            pmax[w] = mx;
            if (bad) pbad[w] = 1;
        });
        for (char b : pbad)
            if (b) return false;
    }
    int maxlev = 0;
    for (int m : pmax) maxlev = std::max(maxlev, m);
    level_ptr.assign(maxlev + 2, 0);
    for (int i = 0; i < n; ++i) ++level_ptr[lev[i] + 1];
    for (int l = 0; l <= maxlev; ++l) level_ptr[l + 1] += level_ptr[l];
    rows_by_level.assign(n, 0);
    std::vector<int> f(level_ptr.begin(), level_ptr.end() - 1);
    for (int s = 0; s < n; ++s) {
        int i = ord[lower ? s : n - 1 - s];
        rows_by_level[f[lev[i]]++] = i;
    }
    return true;
}

void sell_slices(int nrows, const std::vector<int> &seg_row, const std::vector<int> &cnt,
                 SellLayout &L)
{
    L = SellLayout();
    L.nrows = nrows;
    const int nseg = (int)seg_row.size() - 1;
    L.seg_slice.assign(nseg + 1, 0);
    int off = 0;
    for (int s = 0; s < nseg; ++s) {
        L.seg_slice[s] = (int)L.slice_row0.size();
        for (int r0 = seg_row[s]; r0 < seg_row[s + 1]; r0 += 64) {
            int rows = std::min(64, seg_row[s + 1] - r0);
            int w = 0;
            for (int t = r0; t < r0 + rows; ++t) w = std::max(w, cnt[t]);
            L.slice_row0.push_back(r0);
            L.slice_rows.push_back(rows);
            L.slice_width.push_back(w);
            L.slice_off.push_back(off);
            off += w * 64;
        }
    }
    L.seg_slice[nseg] = (int)L.slice_row0.size();
    L.slot_lanes = off;
}

void build_sell(int nrows, const std::vector<int> &seg_row, const std::vector<int> &ent_ptr,
                const std::vector<int> &ent_col, const std::vector<int> &ent_src, SellLayout &L)
{
    std::vector<int> cnt(nrows);
    for (int t = 0; t < nrows; ++t) cnt[t] = ent_ptr[t + 1] - ent_ptr[t];
    sell_slices(nrows, seg_row, cnt, L);
    const long long off = L.slot_lanes;
    L.col.assign(off, -1);
    L.src.assign(off, -1);
    const int nsl = (int)L.slice_row0.size();
    for_chunks(nsl, host_parts(nrows), [&](int lo, int hi, int) {
        for (int s = lo; s < hi; ++s) {
            for (int l = 0; l < L.slice_rows[s]; ++l) {
                int t = L.slice_row0[s] + l;
                for (int k = ent_ptr[t]; k < ent_ptr[t + 1]; ++k) {
                    int slot = k - ent_ptr[t];
                    long q = (long)L.slice_off[s] + slot * 64 + l;
                    L.col[q] = ent_col[k];
                    L.src[q] = ent_src[k];
                }
            }
        }
    });
}

}  // namespace msp
