// Test-only C shim over the library's host setup code (msp_host.cpp), so the
// CPU suite can compare its grouping, matching and Galerkin products with the
// oracle without a GPU.
#include <cstring>
#include <vector>

#include "msp_host.h"

extern "C" {

int shim_color(int n, const int *rp, const int *ci, int *color)
{
    msp::Adjacency G = msp::build_adjacency(n, rp, ci);
    std::vector<int> c;
    int g = msp::vertices_grouping(G, c);
    std::memcpy(color, c.data(), sizeof(int) * n);
    return g;
}

int shim_color_sym(int n, const int *rp, const int *ci, int *color, int *diag_once)
{
    std::vector<int> c;
    bool d = false;
    int g = msp::vertices_grouping_symmetric(n, rp, ci, c, &d);
    std::memcpy(color, c.data(), sizeof(int) * n);
    *diag_once = d ? 1 : 0;
    return g;
}

static msp::Csr make(int n, const int *rp, const int *ci, const double *val)
{
    msp::Csr A;
    A.n = n;
    A.rp.assign(rp, rp + n + 1);
    A.ci.assign(ci, ci + rp[n]);
    A.val.assign(val, val + rp[n]);
    return A;
}

int shim_pair(int n, const int *rp, const int *ci, const double *val, int *agg)
{
    std::vector<int> a;
    int nc = msp::pairwise_pass(make(n, rp, ci, val), a);
    std::memcpy(agg, a.data(), sizeof(int) * n);
    return nc;
}

long long shim_galerkin(int n, const int *rp, const int *ci, const double *val, const int *agg,
                        int nc, int *crp, int *cci, double *cval)
{
    std::vector<int> a(agg, agg + n);
    msp::Csr C = msp::galerkin(make(n, rp, ci, val), a, nc);
    std::memcpy(crp, C.rp.data(), sizeof(int) * (nc + 1));
    std::memcpy(cci, C.ci.data(), sizeof(int) * C.ci.size());
    std::memcpy(cval, C.val.data(), sizeof(double) * C.val.size());
    return (long long)C.ci.size();
}

// The library's whole aggregation chain (no groups): returns the number of
// levels; sizes[l] = rows of level l; aggs = the fine-to-coarse maps of the
// non-coarsest levels, concatenated; the coarsest level's CSR is copied to
// crp/cci/cval (capacity nnz of the input).
int shim_hierarchy(int n, const int *rp, const int *ci, const double *val, int max_coarse,
                   int *sizes, int *aggs, int *crp, int *cci, double *cval)
{
    msp::Hierarchy H;
    int st = msp::build_hierarchy(make(n, rp, ci, val), max_coarse, 25, 1 << 30, H, false);
    if (st != 0) return st;
    long long off = 0;
    for (size_t l = 0; l < H.A.size(); ++l) {
        sizes[l] = H.A[l].n;
        if (l + 1 < H.A.size()) {
            std::memcpy(aggs + off, H.agg[l].data(), sizeof(int) * H.A[l].n);
            off += H.A[l].n;
        }
    }
    const msp::Csr &C = H.A.back();
    std::memcpy(crp, C.rp.data(), sizeof(int) * (C.n + 1));
    std::memcpy(cci, C.ci.data(), sizeof(int) * C.ci.size());
    std::memcpy(cval, C.val.data(), sizeof(double) * C.val.size());
    return (int)H.A.size();
}

int shim_pattern(int n, const int *rp, const int *ci, long long nnz)
{
    return msp::check_pattern(n, rp, ci, nnz);
}

// levels of a triangular solve in natural order; returns the number of levels
// dependency levels in a given elimination order: sequential pass, and the
// group-parallel pass for an order made of groups (-1 when it declines)
int shim_levels_ord(int n, const int *rp, const int *ci, const int *ord_in, int lower, int *rows,
                    int *ptr)
{
    std::vector<int> ord(ord_in, ord_in + n), r, p;
    msp::triangular_levels(n, rp, ci, ord, lower != 0, r, p);
    std::memcpy(rows, r.data(), sizeof(int) * n);
    std::memcpy(ptr, p.data(), sizeof(int) * p.size());
    return (int)p.size() - 1;
}

int shim_levels_groups(int n, const int *rp, const int *ci, const int *ord_in, int ng,
                       const int *grp_in, int lower, int *rows, int *ptr)
{
    std::vector<int> ord(ord_in, ord_in + n), grp(grp_in, grp_in + ng + 1), r, p;
    if (!msp::triangular_levels_groups(n, rp, ci, ord, grp, lower != 0, r, p)) return -1;
    std::memcpy(rows, r.data(), sizeof(int) * n);
    std::memcpy(ptr, p.data(), sizeof(int) * p.size());
    return (int)p.size() - 1;
}

int shim_levels(int n, const int *rp, const int *ci, int lower, int *rows_by_level)
{
    std::vector<int> ord(n), rows, ptr;
    for (int i = 0; i < n; ++i) ord[i] = i;
    msp::triangular_levels(n, rp, ci, ord, lower != 0, rows, ptr);
    std::memcpy(rows_by_level, rows.data(), sizeof(int) * n);
    return (int)ptr.size() - 1;
}
}
