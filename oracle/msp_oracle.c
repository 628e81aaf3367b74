/*
 * msp_oracle.c -- plain, sequential FP64 reference for the multi-stage
 * (CPR-type) preconditioned FGMRES solve of a block-sparse reservoir Jacobian,
 * after L. Zhao, C.-S. Zhang, C.-S. Feng, S. Shu, "An Improved Multi-Stage
 * Preconditioner on GPUs for Compositional Reservoir Simulation" (2022).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or constant with the GPU library; the product path
 * never calls it.
 *
 * Everything is written in the order the method states it, one row / one
 * entry at a time, with no blocking, fusion or reordering.  Sums run over
 * ascending indices.  The dense coarsest-level factorisation is a library
 * primitive (LAPACK getrf, called from the Python wrapper); this file only
 * applies its factors.
 *
 * Where the paper is silent the readings used here are:
 *   - decoupling: alternate block factorisation (ABF), the weights of cell c
 *     are row p of the inverse diagonal block, obtained by Gaussian
 *     elimination with partial pivoting on the transposed block;
 *   - adjacency: the structural off-diagonal pattern of A and A^T together;
 *     vertex degrees are static; ties go to the lowest index;
 *   - aggregation: two passes of pairwise matching (a concrete form of the
 *     nonsymmetric pairwise aggregation the paper names, not claimed identical
 *     to the cited method);
 *   - block ILU(0) in natural block order, pivot blocks inverted;
 *   - stages P then R of the multiplicative preconditioner, initial guess 0;
 *   - right-preconditioned flexible GMRES(m) with modified Gram-Schmidt.
 *
 * "parity unpinned" items: the aggregation rule is the builder's reading and
 * is pinned only by invariants (partition, pair sizes, strength), not against
 * the cited method.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_ARG (-1)
#define OR_ERR_PATTERN (-2)
#define OR_ERR_SINGULAR (-3)
#define OR_ERR_NONFINITE (-4)
#define OR_ERR_NOMEM (-5)
#define OR_ERR_STATE (-8)
#define OR_ERR_COARSE (-9)
#define OR_NOT_CONVERGED 1

#define OR_MAXB 16
#define OR_MAX_LEVELS 25
#define OR_MAX_DENSE 16384

/* ------------------------------------------------------------------------ */
/* O1  Input validation (the block system of Sec. 2.3: block rows of n_c+1    */
/*     equations, every block row holds its diagonal block).                  */
/* ------------------------------------------------------------------------ */
int or_validate(int n, int b, int p, const int *rp, const int *ci, const double *vals, long nnzb)
{
    if (n < 1 || b < 1 || b > OR_MAXB || p < 0 || p >= b || !rp || !ci || !vals || nnzb < n)
        return OR_ERR_ARG;
    if (rp[0] != 0 || (long)rp[n] != nnzb)
        return OR_ERR_PATTERN;
    for (int c = 0; c < n; ++c) {
        if (rp[c + 1] <= rp[c])
            return OR_ERR_PATTERN;
        int has_diag = 0;
        for (int k = rp[c]; k < rp[c + 1]; ++k) {
            if (ci[k] < 0 || ci[k] >= n)
                return OR_ERR_PATTERN;
            if (k > rp[c] && ci[k] <= ci[k - 1])
                return OR_ERR_PATTERN;
            if (ci[k] == c)
                has_diag = 1;
        }
        if (!has_diag)
            return OR_ERR_PATTERN;
    }
    for (long q = 0; q < nnzb * (long)b * b; ++q)
        if (!isfinite(vals[q]))
            return OR_ERR_NONFINITE;
    return OR_OK;
}

static int find_col(const int *rp, const int *ci, int row, int col)
{
    for (int k = rp[row]; k < rp[row + 1]; ++k)
        if (ci[k] == col)
            return k;
    return -1;
}

/* ------------------------------------------------------------------------ */
/* O2  Decoupling and pressure extraction (the pressure stage of eq. MSP     */
/*     acts on Pi_P^T of the decoupled system).  w_c solves D_c^T w = e_p,   */
/*     i.e. w_c^T = e_p^T D_c^{-1}; A_P[c,d] = sum_k w_c[k] A_cd[k][p].       */
/* ------------------------------------------------------------------------ */
static int abf_weights(int b, int p, const double *D, double *w)
{
    double T[OR_MAXB * OR_MAXB], y[OR_MAXB];
    for (int r = 0; r < b; ++r)
        for (int s = 0; s < b; ++s)
            T[r * b + s] = D[s * b + r];
    for (int r = 0; r < b; ++r)
        y[r] = (r == p) ? 1.0 : 0.0;
    for (int k = 0; k < b; ++k) {
        int piv = k;
        double best = fabs(T[k * b + k]);
        for (int r = k + 1; r < b; ++r)
            if (fabs(T[r * b + k]) > best) {
                best = fabs(T[r * b + k]);
                piv = r;
            }
        if (best == 0.0)
            return OR_ERR_SINGULAR;
        if (piv != k) {
            for (int s = 0; s < b; ++s) {
                double t = T[k * b + s];
                T[k * b + s] = T[piv * b + s];
                T[piv * b + s] = t;
            }
            double t = y[k];
            y[k] = y[piv];
            y[piv] = t;
        }
        for (int r = k + 1; r < b; ++r) {
            double m = T[r * b + k] / T[k * b + k];
            for (int s = k + 1; s < b; ++s)
                T[r * b + s] = T[r * b + s] - m * T[k * b + s];
            y[r] = y[r] - m * y[k];
        }
    }
    for (int r = b - 1; r >= 0; --r) {
        double acc = y[r];
        for (int s = r + 1; s < b; ++s)
            acc = acc - T[r * b + s] * w[s];
        w[r] = acc / T[r * b + r];
    }
    return OR_OK;
}

int or_decouple(int n, int b, int p, const int *rp, const int *ci, const double *vals,
                double *omega, double *ap_vals)
{
    const int bb = b * b;
    for (int c = 0; c < n; ++c) {
        int kd = find_col(rp, ci, c, c);
        if (kd < 0)
            return OR_ERR_PATTERN;
        int st = abf_weights(b, p, vals + (long)kd * bb, omega + (long)c * b);
        if (st != OR_OK)
            return st;
        for (int k = rp[c]; k < rp[c + 1]; ++k) {
            const double *blk = vals + (long)k * bb;
            double acc = 0.0;
            for (int r = 0; r < b; ++r)
                acc = acc + omega[(long)c * b + r] * blk[r * b + p];
            ap_vals[k] = acc;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Adjacency graph G_A (Sec. 4.1, eq. for S): S_ij = 1 iff i != j and a_ij   */
/* is stored; for a nonsymmetric pattern S is taken over A and A^T so that   */
/* principle (iii) (a_ij = a_ji = 0 inside a group) holds.                    */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    int *ptr;
    int *adj;
} or_graph;

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

static int build_sym_graph(int n, const int *rp, const int *ci, or_graph *G)
{
    long nnz = rp[n];
    int *cnt = (int *)calloc((size_t)n + 1, sizeof(int));
    int *tmp = (int *)malloc(sizeof(int) * (size_t)(2 * nnz + 1));
    int *fill = (int *)calloc((size_t)n, sizeof(int));
    if (!cnt || !tmp || !fill) {
        free(cnt); free(tmp); free(fill);
        return OR_ERR_NOMEM;
    }
    for (int i = 0; i < n; ++i)
        for (int k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] != i) {
                cnt[i + 1]++;
                cnt[ci[k] + 1]++;
            }
    for (int i = 0; i < n; ++i)
        cnt[i + 1] += cnt[i];
    for (int i = 0; i < n; ++i)
        for (int k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] != i) {
                int j = ci[k];
                tmp[cnt[i] + fill[i]++] = j;
                tmp[cnt[j] + fill[j]++] = i;
            }
    G->n = n;
    G->ptr = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    G->adj = (int *)malloc(sizeof(int) * (size_t)(2 * nnz + 1));
    if (!G->ptr || !G->adj) {
        free(cnt); free(tmp); free(fill);
        return OR_ERR_NOMEM;
    }
    G->ptr[0] = 0;
    for (int i = 0; i < n; ++i) {
        int len = cnt[i + 1] - cnt[i];
        qsort(tmp + cnt[i], (size_t)len, sizeof(int), cmp_int);
        int out = G->ptr[i];
        for (int q = 0; q < len; ++q)
            if (q == 0 || tmp[cnt[i] + q] != tmp[cnt[i] + q - 1])
                G->adj[out++] = tmp[cnt[i] + q];
        G->ptr[i + 1] = out;
    }
    free(cnt); free(tmp); free(fill);
    return OR_OK;
}

static void free_graph(or_graph *G)
{
    free(G->ptr);
    free(G->adj);
}

/* ------------------------------------------------------------------------ */
/* O4  VerticesGrouping (Alg. 4.2) around VerticesSplitting (Alg. 4.1).      */
/*                                                                            */
/* One call of Alg. 4.1 builds one group W from the undetermined set V:      */
/* the next vertex is the one of largest |S_i| among the second-ring          */
/* candidates W^ that are still undetermined, else among V (ties: lowest      */
/* index); it joins W, its neighbours S_i leave V (they form W-bar), and the */
/* undetermined vertices of its second ring enter W^.  With a symmetric S a   */
/* vertex still in V is never adjacent to W, so the test of Alg. 4.1 always  */
/* passes for it; candidates of W^ that have left V are dropped, which is     */
/* what the else-branch of Alg. 4.1 does with them.  Alg. 4.2 repeats on      */
/* W-bar until nothing is left.  Colors are 1..g.                             */
/* ------------------------------------------------------------------------ */
static const int *g_deg; /* degree array used by the orderings below */

static int higher_priority(int a, int b)
{
    /* larger |S| first, then smaller index */
    if (g_deg[a] != g_deg[b])
        return g_deg[a] > g_deg[b];
    return a < b;
}

static int cmp_priority(const void *pa, const void *pb)
{
    int a = *(const int *)pa, b = *(const int *)pb;
    if (a == b)
        return 0;
    return higher_priority(a, b) ? -1 : 1;
}

typedef struct {
    int *a;
    int size;
} or_heap;

static void heap_push(or_heap *h, int v)
{
    int i = h->size++;
    h->a[i] = v;
    while (i > 0) {
        int par = (i - 1) / 2;
        if (!higher_priority(h->a[i], h->a[par]))
            break;
        int t = h->a[i]; h->a[i] = h->a[par]; h->a[par] = t;
        i = par;
    }
}

static int heap_pop(or_heap *h)
{
    int top = h->a[0];
    h->a[0] = h->a[--h->size];
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = l + 1, best = i;
        if (l < h->size && higher_priority(h->a[l], h->a[best]))
            best = l;
        if (r < h->size && higher_priority(h->a[r], h->a[best]))
            best = r;
        if (best == i)
            break;
        int t = h->a[i]; h->a[i] = h->a[best]; h->a[best] = t;
        i = best;
    }
    return top;
}

int or_color(int n, const int *rp, const int *ci, int *color)
{
    or_graph G;
    int st = build_sym_graph(n, rp, ci, &G);
    if (st != OR_OK)
        return st;
    int *deg = (int *)malloc(sizeof(int) * (size_t)n);
    int *order = (int *)malloc(sizeof(int) * (size_t)n);
    char *inV = (char *)calloc((size_t)n, 1);
    char *inH = (char *)calloc((size_t)n, 1);
    or_heap h;
    h.a = (int *)malloc(sizeof(int) * (size_t)n + 4);
    h.size = 0;
    if (!deg || !order || !inV || !inH || !h.a) {
        free(deg); free(order); free(inV); free(inH); free(h.a); free_graph(&G);
        return OR_ERR_NOMEM;
    }
    for (int i = 0; i < n; ++i) {
        deg[i] = G.ptr[i + 1] - G.ptr[i];
        order[i] = i;
        color[i] = 0;
    }
    g_deg = deg;
    qsort(order, (size_t)n, sizeof(int), cmp_priority);

    int uncolored = n, g = 0;
    while (uncolored > 0) {
        ++g;
        int remaining = 0;
        for (int i = 0; i < n; ++i) {
            inV[i] = (color[i] == 0);
            inH[i] = 0;
            remaining += inV[i];
        }
        h.size = 0;
        int cursor = 0;
        while (remaining > 0) {
            int v = -1;
            while (h.size > 0) {
                int t = heap_pop(&h);
                if (inV[t]) {
                    v = t;
                    break;
                }
            }
            if (v < 0) {
                while (!inV[order[cursor]])
                    ++cursor;
                v = order[cursor];
            }
            color[v] = g;
            inV[v] = 0;
            --remaining;
            --uncolored;
            for (int q = G.ptr[v]; q < G.ptr[v + 1]; ++q) {
                int u = G.adj[q];
                if (inV[u]) {
                    inV[u] = 0;
                    --remaining;
                }
            }
            for (int q = G.ptr[v]; q < G.ptr[v + 1]; ++q) {
                int u = G.adj[q];
                for (int t = G.ptr[u]; t < G.ptr[u + 1]; ++t) {
                    int w = G.adj[t];
                    if (inV[w] && !inH[w]) {
                        inH[w] = 1;
                        heap_push(&h, w);
                    }
                }
            }
        }
    }
    free(deg); free(order); free(inV); free(inH); free(h.a); free_graph(&G);
    return g;
}

/* ------------------------------------------------------------------------ */
/* O5  One pass of pairwise matching (the paper's UA-AMG uses nonsymmetric   */
/*     pairwise aggregation, Sec. 5).  Builder's concrete rule:              */
/*     s_ij = -(m_ij + m_ji)/2 over the symmetrised neighbours; strong set   */
/*     {j : s_ij >= 0.25 max_k s_ik} when that max is positive; rows whose     */
/*     stored off-diagonal values are all zero, or with no positive s, stay   */
/*     single and are never chosen as partners; vertices are visited in       */
/*     ascending order and take the strongest free eligible strong neighbour  */
/*     (ties: lowest index).  Aggregates are numbered in order of creation.  */
/* ------------------------------------------------------------------------ */
static double csr_value(const int *rp, const int *ci, const double *val, int i, int j)
{
    int lo = rp[i], hi = rp[i + 1] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (ci[mid] == j)
            return val[mid];
        if (ci[mid] < j)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return 0.0;
}

int or_npair_pass(int n, const int *rp, const int *ci, const double *val, int *agg)
{
    or_graph G;
    int st = build_sym_graph(n, rp, ci, &G);
    if (st != OR_OK)
        return st;
    char *elig = (char *)calloc((size_t)n, 1);
    double *smax = (double *)calloc((size_t)n, sizeof(double));
    if (!elig || !smax) {
        free(elig); free(smax); free_graph(&G);
        return OR_ERR_NOMEM;
    }
    for (int i = 0; i < n; ++i) {
        int offdiag_nonzero = 0;
        for (int k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] != i && val[k] != 0.0)
                offdiag_nonzero = 1;
        int has = 0;
        double mx = 0.0;
        for (int q = G.ptr[i]; q < G.ptr[i + 1]; ++q) {
            int j = G.adj[q];
            double s = -(csr_value(rp, ci, val, i, j) + csr_value(rp, ci, val, j, i)) / 2.0;
            if (!has || s > mx)
                mx = s;
            has = 1;
        }
        smax[i] = mx;
        elig[i] = (char)(offdiag_nonzero && has && mx > 0.0);
    }
    int nc = 0;
    for (int i = 0; i < n; ++i)
        agg[i] = -1;
    for (int i = 0; i < n; ++i) {
        if (agg[i] >= 0)
            continue;
        int best = -1;
        double bs = 0.0;
        if (elig[i]) {
            for (int q = G.ptr[i]; q < G.ptr[i + 1]; ++q) {
                int j = G.adj[q];
                if (agg[j] >= 0 || !elig[j])
                    continue;
                double s = -(csr_value(rp, ci, val, i, j) + csr_value(rp, ci, val, j, i)) / 2.0;
                if (s >= 0.25 * smax[i] && (best < 0 || s > bs)) {
                    best = j;
                    bs = s;
                }
            }
        }
        agg[i] = nc;
        if (best >= 0)
            agg[best] = nc;
        ++nc;
    }
    free(elig); free(smax); free_graph(&G);
    return nc;
}

/* Stalled coarsening (the two pairwise passes of a level kept more than    */
/* 90% of its rows): every eligible row alone in its aggregate joins the     */
/* aggregate of its strongest neighbour j with s_ij >= 0.25 max_k s_ik among  */
/* the neighbours in aggregates of two or more rows (sizes before any move,  */
/* lowest j among equals; the strengths and eligibility of the pairwise      */
/* pass).  Aggregates left empty are dropped, the others keep their order.   */
/* Returns the new number of aggregates.                                      */
int or_absorb_singletons(int n, const int *rp, const int *ci, const double *val, int *agg,
                         int nc)
{
    or_graph G;
    int st = build_sym_graph(n, rp, ci, &G);
    if (st != OR_OK)
        return st;
    int *size = (int *)calloc((size_t)nc, sizeof(int));
    int *target = (int *)malloc(sizeof(int) * (size_t)n);
    int *map = (int *)malloc(sizeof(int) * (size_t)nc);
    if (!size || !target || !map) {
        free(size); free(target); free(map); free_graph(&G);
        return OR_ERR_NOMEM;
    }
    for (int i = 0; i < n; ++i)
        size[agg[i]]++;
    for (int i = 0; i < n; ++i) {
        target[i] = agg[i];
        if (size[agg[i]] != 1)
            continue;
        int offdiag_nonzero = 0;
        for (int k = rp[i]; k < rp[i + 1]; ++k)
            if (ci[k] != i && val[k] != 0.0)
                offdiag_nonzero = 1;
        int has = 0;
        double mx = 0.0;
        for (int q = G.ptr[i]; q < G.ptr[i + 1]; ++q) {
            int j = G.adj[q];
            double s = -(csr_value(rp, ci, val, i, j) + csr_value(rp, ci, val, j, i)) / 2.0;
            if (!has || s > mx)
                mx = s;
            has = 1;
        }
        if (!(offdiag_nonzero && has && mx > 0.0))
            continue;
        int best = -1;
        double bs = 0.0;
        for (int q = G.ptr[i]; q < G.ptr[i + 1]; ++q) {
            int j = G.adj[q];
            if (size[agg[j]] < 2)
                continue;
            double s = -(csr_value(rp, ci, val, i, j) + csr_value(rp, ci, val, j, i)) / 2.0;
            if (s >= 0.25 * mx && (best < 0 || s > bs)) {
                best = j;
                bs = s;
            }
        }
        if (best >= 0)
            target[i] = agg[best];
    }
    for (int a = 0; a < nc; ++a)
        map[a] = -1;
    for (int i = 0; i < n; ++i)
        map[target[i]] = 0;
    int k = 0;
    for (int a = 0; a < nc; ++a)
        if (map[a] == 0)
            map[a] = k++;
    for (int i = 0; i < n; ++i)
        agg[i] = map[target[i]];
    free(size); free(target); free(map); free_graph(&G);
    return k;
}

/* ------------------------------------------------------------------------ */
/* O6  Galerkin coarse operator A_c = P^T A P for piecewise-constant P       */
/*     (unsmoothed aggregation, Sec. 5): A_c[agg(i), agg(j)] accumulates     */
/*     a_ij over fine rows i ascending and, within a row, j ascending.        */
/*     The pattern is structural (exact zeros stay); columns sorted.          */
/*     Output capacity: at most nnz(A) entries.  Returns nnz(A_c).            */
/* ------------------------------------------------------------------------ */
long or_galerkin(int n, const int *rp, const int *ci, const double *val, const int *agg, int nc,
                 int *crp, int *cci, double *cval)
{
    /* per coarse row: a list with capacity = sum of member row lengths */
    long *cap = (long *)calloc((size_t)nc + 1, sizeof(long));
    int *len = (int *)calloc((size_t)nc, sizeof(int));
    if (!cap || !len) {
        free(cap); free(len);
        return OR_ERR_NOMEM;
    }
    for (int i = 0; i < n; ++i)
        cap[agg[i] + 1] += rp[i + 1] - rp[i];
    for (int I = 0; I < nc; ++I)
        cap[I + 1] += cap[I];
    int *lc = (int *)malloc(sizeof(int) * (size_t)(cap[nc] + 1));
    double *lv = (double *)malloc(sizeof(double) * (size_t)(cap[nc] + 1));
    if (!lc || !lv) {
        free(cap); free(len); free(lc); free(lv);
        return OR_ERR_NOMEM;
    }
    for (int i = 0; i < n; ++i) {
        int I = agg[i];
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            int J = agg[ci[k]];
            long base = cap[I];
            int q;
            for (q = 0; q < len[I]; ++q)
                if (lc[base + q] == J)
                    break;
            if (q == len[I]) {
                lc[base + q] = J;
                lv[base + q] = val[k];
                len[I]++;
            } else {
                lv[base + q] = lv[base + q] + val[k];
            }
        }
    }
    long out = 0;
    crp[0] = 0;
    for (int I = 0; I < nc; ++I) {
        long base = cap[I];
        /* insertion sort by column (stable, carries values) */
        for (int a = 1; a < len[I]; ++a) {
            int c = lc[base + a];
            double v = lv[base + a];
            int q = a - 1;
            while (q >= 0 && lc[base + q] > c) {
                lc[base + q + 1] = lc[base + q];
                lv[base + q + 1] = lv[base + q];
                --q;
            }
            lc[base + q + 1] = c;
            lv[base + q + 1] = v;
        }
        for (int a = 0; a < len[I]; ++a) {
            cci[out] = lc[base + a];
            cval[out] = lv[base + a];
            ++out;
        }
        crp[I + 1] = (int)out;
    }
    free(cap); free(len); free(lc); free(lv);
    return out;
}

/* ------------------------------------------------------------------------ */
/* Small dense block helpers (b x b, row-major).                              */
/* ------------------------------------------------------------------------ */
/* X = M^{-1} by Gaussian elimination with partial pivoting (first largest). */
static int block_inverse(int b, const double *M, double *X)
{
    double LU[OR_MAXB * OR_MAXB];
    int perm[OR_MAXB];
    memcpy(LU, M, sizeof(double) * (size_t)(b * b));
    for (int r = 0; r < b; ++r)
        perm[r] = r;
    for (int k = 0; k < b; ++k) {
        int piv = k;
        double best = fabs(LU[k * b + k]);
        for (int r = k + 1; r < b; ++r)
            if (fabs(LU[r * b + k]) > best) {
                best = fabs(LU[r * b + k]);
                piv = r;
            }
        if (best == 0.0)
            return OR_ERR_SINGULAR;
        if (piv != k) {
            for (int s = 0; s < b; ++s) {
                double t = LU[k * b + s];
                LU[k * b + s] = LU[piv * b + s];
                LU[piv * b + s] = t;
            }
            int t = perm[k]; perm[k] = perm[piv]; perm[piv] = t;
        }
        for (int r = k + 1; r < b; ++r) {
            LU[r * b + k] = LU[r * b + k] / LU[k * b + k];
            for (int s = k + 1; s < b; ++s)
                LU[r * b + s] = LU[r * b + s] - LU[r * b + k] * LU[k * b + s];
        }
    }
    for (int e = 0; e < b; ++e) {
        double y[OR_MAXB];
        for (int r = 0; r < b; ++r) {
            double acc = (perm[r] == e) ? 1.0 : 0.0;
            for (int s = 0; s < r; ++s)
                acc = acc - LU[r * b + s] * y[s];
            y[r] = acc;
        }
        for (int r = b - 1; r >= 0; --r) {
            double acc = y[r];
            for (int s = r + 1; s < b; ++s)
                acc = acc - LU[r * b + s] * y[s];
            y[r] = acc / LU[r * b + r];
        }
        for (int r = 0; r < b; ++r)
            X[r * b + e] = y[r];
    }
    return OR_OK;
}

/* C = A B */
static void block_mul(int b, const double *A, const double *B, double *C)
{
    for (int r = 0; r < b; ++r)
        for (int s = 0; s < b; ++s) {
            double acc = 0.0;
            for (int t = 0; t < b; ++t)
                acc = acc + A[r * b + t] * B[t * b + s];
            C[r * b + s] = acc;
        }
}

/* ------------------------------------------------------------------------ */
/* O7  Block ILU(0) of the whole system (the relaxation R of eq. MSP), IKJ   */
/*     form in a given elimination order ord (ord[t] = block row eliminated   */
/*     t-th; natural order is ord[t] = t): for each block row i in that order */
/*     and each stored k eliminated before i (in elimination order):          */
/*     F_ik <- F_ik F_kk^{-1}; F_ij <- F_ij - F_ik F_kj for stored j          */
/*     eliminated after k with (k,j) stored.  Pivot blocks are kept inverted. */
/* ------------------------------------------------------------------------ */
/* entries of block row i whose column is eliminated before (lower != 0) or  */
/* after (lower == 0) row i, in elimination order; returns their count       */
static int ordered_entries(const int *rp, const int *ci, const int *pos, int i, int lower,
                           int *out)
{
    int m = 0;
    for (int q = rp[i]; q < rp[i + 1]; ++q) {
        int j = ci[q];
        if (lower ? pos[j] < pos[i] : pos[j] > pos[i]) {
            int a = m++;
            while (a > 0 && pos[ci[out[a - 1]]] > pos[j]) {
                out[a] = out[a - 1];
                --a;
            }
            out[a] = q;
        }
    }
    return m;
}

static int max_row_len(int n, const int *rp)
{
    int w = 1;
    for (int i = 0; i < n; ++i)
        if (rp[i + 1] - rp[i] > w)
            w = rp[i + 1] - rp[i];
    return w;
}

int or_bilu0_factor_ordered(int n, int b, const int *rp, const int *ci, const double *A,
                            const int *ord, double *F, double *Dinv)
{
    const int bb = b * b;
    long nnzb = rp[n];
    memcpy(F, A, sizeof(double) * (size_t)(nnzb * bb));
    int *pos = (int *)malloc(sizeof(int) * (size_t)n);
    int *low = (int *)malloc(sizeof(int) * (size_t)max_row_len(n, rp));
    if (!pos || !low) { free(pos); free(low); return OR_ERR_NOMEM; }
    for (int t = 0; t < n; ++t)
        pos[ord[t]] = t;
    double tmp[OR_MAXB * OR_MAXB], prod[OR_MAXB * OR_MAXB];
    int st = OR_OK;
    for (int t = 0; t < n && st == OR_OK; ++t) {
        int i = ord[t];
        int m = ordered_entries(rp, ci, pos, i, 1, low);
        for (int a = 0; a < m; ++a) {
            int kk = low[a], k = ci[kk];
            block_mul(b, F + (long)kk * bb, Dinv + (long)k * bb, tmp);
            memcpy(F + (long)kk * bb, tmp, sizeof(double) * (size_t)bb);
            for (int jj = rp[i]; jj < rp[i + 1]; ++jj) {
                int j = ci[jj];
                if (pos[j] <= pos[k])
                    continue;
                int kj = find_col(rp, ci, k, j);
                if (kj < 0)
                    continue;
                block_mul(b, F + (long)kk * bb, F + (long)kj * bb, prod);
                double *Fij = F + (long)jj * bb;
                for (int q = 0; q < bb; ++q)
                    Fij[q] = Fij[q] - prod[q];
            }
        }
        int kd = find_col(rp, ci, i, i);
        if (kd < 0)
            st = OR_ERR_PATTERN;
        else
            st = block_inverse(b, F + (long)kd * bb, Dinv + (long)i * bb);
    }
    free(pos);
    free(low);
    return st;
}

int or_bilu0_factor(int n, int b, const int *rp, const int *ci, const double *A, double *F,
                    double *Dinv)
{
    int *ord = (int *)malloc(sizeof(int) * (size_t)n);
    if (!ord)
        return OR_ERR_NOMEM;
    for (int t = 0; t < n; ++t)
        ord[t] = t;
    int st = or_bilu0_factor_ordered(n, b, rp, ci, A, ord, F, Dinv);
    free(ord);
    return st;
}

/* Multi-color elimination order of the block adjacency graph: the groups of */
/* Alg. 4.2 one after another, ascending index inside a group.               */
int or_multicolor_order(int n, const int *rp, const int *ci, int *ord)
{
    int *col = (int *)malloc(sizeof(int) * (size_t)n);
    if (!col)
        return OR_ERR_NOMEM;
    int g = or_color(n, rp, ci, col);
    if (g < 0) { free(col); return g; }
    int t = 0;
    for (int l = 1; l <= g; ++l)
        for (int i = 0; i < n; ++i)
            if (col[i] == l)
                ord[t++] = i;
    free(col);
    return g;
}

/* ------------------------------------------------------------------------ */
/* Precision-generic apply routines (double, and float for the FP32         */
/* preconditioner): included twice.                                           */
/* ------------------------------------------------------------------------ */
#define REAL double
#define SFX(name) name##_f64
#include "oracle_apply.inc"
#undef REAL
#undef SFX
#define REAL float
#define SFX(name) name##_f32
#include "oracle_apply.inc"
#undef REAL
#undef SFX

/* Exported double-precision stage functions (pins and per-kernel parity). */
void or_bilu0_solve_ordered(int n, int b, const int *rp, const int *ci, const double *F,
                            const double *Dinv, const int *ord, const double *r, double *z)
{
    bilu0_solve_f64(n, b, rp, ci, F, Dinv, ord, r, z);
}

void or_bilu0_solve(int n, int b, const int *rp, const int *ci, const double *F,
                    const double *Dinv, const double *r, double *z)
{
    int *ord = (int *)malloc(sizeof(int) * (size_t)n);
    if (!ord)
        return;
    for (int t = 0; t < n; ++t)
        ord[t] = t;
    bilu0_solve_f64(n, b, rp, ci, F, Dinv, ord, r, z);
    free(ord);
}

/* One weighted point-Jacobi sweep x_out = x + w D^{-1} (f - A x): every row */
/* reads only the incoming x.                                                 */
int or_jacobi_sweep(int n, const int *rp, const int *ci, const double *val, double w,
                    const double *f, const double *x, double *x_out)
{
    return jacobi_sweep_f64(n, rp, ci, val, w, f, x, x_out);
}

void or_gs_sweep(int n, const int *rp, const int *ci, const double *val, const int *color, int g,
                 const double *f, double *x, int forward)
{
    for (int t = 0; t < g; ++t) {
        int col = forward ? t + 1 : g - t;
        for (int i = 0; i < n; ++i)
            if (color[i] == col)
                gs_row_f64(rp, ci, val, i, f, x);
    }
}

/* ------------------------------------------------------------------------ */
/* Oracle context: a Newton sequence of systems with the adaptive SETUP of   */
/* Sec. 3.2.                                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int n;
    int *rp, *ci;
    double *val;
    float *val32;
    int *color; /* 1..g */
    int g;
    int *agg; /* fine -> next level (NULL on the coarsest) */
    int nc;
} or_level;

typedef struct {
    /* options */
    int mu, restart, max_iter, max_coarse, precond_fp32, bilu_order;
    int smoother;          /* 0: PGS-MC (Alg. 4.3), 1: point Jacobi, 2: natural-order
                              sequential Gauss-Seidel (comparison reference) */
    double jacobi_weight;  /* weight of the Jacobi correction */
    int nu_pre, nu_post;   /* smoothing sweeps before / after the coarse correction */
    int full_smoother;     /* R stage: 0 block ILU(0), 1 block Jacobi */
    int n_stage;           /* 1: the concentration stage B_N runs first (Alg. 3.1) */
    /* current matrix (used by the Krylov SpMV and the pressure-column residual) */
    int n, b, p;
    long nnzb;
    int *rp, *ci;
    double *A;
    float *A32;
    /* preconditioner B (rebuilt or reused) */
    int has_B, Bn, Bb, Bp;
    long Bnnzb;
    double *omega;
    int nlev;
    or_level lev[OR_MAX_LEVELS];
    double *coarse_dense, *LU;
    int *piv;
    int have_lu;
    int *Brp, *Bci, *Bord;
    double *F, *Dinv;
    float *F32, *Dinv32;
    double *Djac;  /* block Jacobi: inverses of the diagonal blocks A_cc */
    float *Djac32;
    /* N stage: groups of the block graph, rows N of D_c^-1 ((b-1) x b per   */
    /* cell) and the N-N part of every decoupled block D_c^-1 A_cd             */
    int *ncolor, ng;
    double *Dn, *Ann;
    float *Dn32, *Ann32;
    /* adaptive state */
    int it_prev, setup_calls, solves;
} or_ctx;

or_ctx *or_create(int mu, int restart, int max_iter, int max_coarse, int precond_fp32,
                  int bilu_order, int smoother, double jacobi_weight, int nu_pre, int nu_post,
                  int full_smoother, int n_stage)
{
    or_ctx *c = (or_ctx *)calloc(1, sizeof(or_ctx));
    if (!c)
        return NULL;
    c->n_stage = n_stage;
    c->smoother = smoother;
    c->jacobi_weight = jacobi_weight;
    c->nu_pre = nu_pre;
    c->nu_post = nu_post;
    c->full_smoother = full_smoother;
    c->mu = mu;
    c->restart = restart;
    c->max_iter = max_iter;
    c->max_coarse = max_coarse;
    c->precond_fp32 = precond_fp32;
    c->bilu_order = bilu_order;
    c->it_prev = -1;
    return c;
}

static void free_B(or_ctx *c)
{
    free(c->omega);
    for (int l = 0; l < c->nlev; ++l) {
        free(c->lev[l].rp); free(c->lev[l].ci); free(c->lev[l].val); free(c->lev[l].val32);
        free(c->lev[l].color); free(c->lev[l].agg);
    }
    memset(c->lev, 0, sizeof(c->lev));
    c->nlev = 0;
    free(c->coarse_dense); free(c->LU); free(c->piv);
    free(c->Brp); free(c->Bci); free(c->Bord); free(c->F); free(c->Dinv); free(c->F32); free(c->Dinv32);
    free(c->Djac); free(c->Djac32);
    free(c->ncolor); free(c->Dn); free(c->Ann); free(c->Dn32); free(c->Ann32);
    c->ncolor = NULL; c->Dn = NULL; c->Ann = NULL; c->Dn32 = NULL; c->Ann32 = NULL;
    c->omega = NULL; c->coarse_dense = NULL; c->LU = NULL; c->piv = NULL;
    c->Brp = NULL; c->Bci = NULL; c->Bord = NULL; c->F = NULL; c->Dinv = NULL; c->F32 = NULL; c->Dinv32 = NULL;
    c->Djac = NULL; c->Djac32 = NULL;
    c->have_lu = 0;
    c->has_B = 0;
}

void or_destroy(or_ctx *c)
{
    if (!c)
        return;
    free_B(c);
    free(c->rp); free(c->ci); free(c->A); free(c->A32);
    free(c);
}

static float *round_f32(const double *x, long m)
{
    float *y = (float *)malloc(sizeof(float) * (size_t)(m > 0 ? m : 1));
    if (y)
        for (long q = 0; q < m; ++q)
            y[q] = (float)x[q];
    return y;
}

/* N stage (the concentration stage of eq. MSP, B_N = one block Gauss-      */
/* Seidel sweep): on the decoupled system W A (W = blockdiag(D_c^-1)) the    */
/* concentration block has N-N blocks (D_c^-1 A_cd)[N, N] and identity       */
/* diagonal blocks; its right-hand side is (D_c^-1 v_c)[N].  The sweep runs  */
/* in the order of the block graph's groups (Alg. 4.2).  N = the unknowns    */
/* other than p, ascending.                                                  */
static int setup_n_stage(or_ctx *c, int n, int b, int p, const int *rp, const int *ci,
                         const double *vals, long nnzb)
{
    const int m = b - 1, bb = b * b;
    c->ncolor = (int *)malloc(sizeof(int) * (size_t)n);
    c->Dn = (double *)calloc((size_t)n * (size_t)(m > 0 ? m * b : 1), sizeof(double));
    c->Ann = (double *)calloc((size_t)nnzb * (size_t)(m > 0 ? m * m : 1), sizeof(double));
    if (!c->ncolor || !c->Dn || !c->Ann)
        return OR_ERR_NOMEM;
    int g = or_color(n, rp, ci, c->ncolor);
    if (g < 0)
        return g;
    c->ng = g;
    double Dinv[OR_MAXB * OR_MAXB], P[OR_MAXB * OR_MAXB];
    for (int cc = 0; cc < n; ++cc) {
        int kd = find_col(rp, ci, cc, cc);
        int st = block_inverse(b, vals + (long)kd * bb, Dinv);
        if (st != OR_OK)
            return st;
        for (int a = 0, ra = 0; a < b; ++a) {
            if (a == p) continue;
            for (int s2 = 0; s2 < b; ++s2)
                c->Dn[((long)cc * m + ra) * b + s2] = Dinv[a * b + s2];
            ++ra;
        }
        for (int q = rp[cc]; q < rp[cc + 1]; ++q) {
            double *out = c->Ann + (long)q * m * m;
            if (ci[q] == cc) {
                for (int a = 0; a < m; ++a)
                    out[a * m + a] = 1.0;
                continue;
            }
            block_mul(b, Dinv, vals + (long)q * bb, P);
            for (int a = 0, ra = 0; a < b; ++a) {
                if (a == p) continue;
                for (int t = 0, rt = 0; t < b; ++t) {
                    if (t == p) continue;
                    out[ra * m + rt] = P[a * b + t];
                    ++rt;
                }
                ++ra;
            }
        }
    }
    return OR_OK;
}

/* O3  Hierarchy: A_0 = A_P; while n_l > max_coarse, color A_l, aggregate in */
/*     two pairwise passes and form A_{l+1}; stop at max_coarse rows, at 25   */
/*     levels, or when a coarsening keeps more than 90% of the rows.          */
static int build_hierarchy(or_ctx *c, int *rp0, int *ci0, double *val0, int n0)
{
    or_level *L = c->lev;
    L[0].n = n0; L[0].rp = rp0; L[0].ci = ci0; L[0].val = val0;
    int l = 0;
    for (;;) {
        or_level *cur = &L[l];
        int last = (cur->n <= c->max_coarse) || (l == OR_MAX_LEVELS - 1) ||
                   (l > 0 && (double)cur->n > 0.9 * (double)L[l - 1].n);
        if (last)
            break;
        cur->color = (int *)malloc(sizeof(int) * (size_t)cur->n);
        if (!cur->color) return OR_ERR_NOMEM;
        int g = or_color(cur->n, cur->rp, cur->ci, cur->color);
        if (g < 0) return g;
        cur->g = g;
        /* pass 1 */
        int *agg1 = (int *)malloc(sizeof(int) * (size_t)cur->n);
        if (!agg1) return OR_ERR_NOMEM;
        int nc1 = or_npair_pass(cur->n, cur->rp, cur->ci, cur->val, agg1);
        if (nc1 < 0) { free(agg1); return nc1; }
        long nnz = cur->rp[cur->n];
        int *m_rp = (int *)malloc(sizeof(int) * ((size_t)nc1 + 1));
        int *m_ci = (int *)malloc(sizeof(int) * (size_t)(nnz + 1));
        double *m_val = (double *)malloc(sizeof(double) * (size_t)(nnz + 1));
        if (!m_rp || !m_ci || !m_val) { free(agg1); return OR_ERR_NOMEM; }
        long mnnz = or_galerkin(cur->n, cur->rp, cur->ci, cur->val, agg1, nc1, m_rp, m_ci, m_val);
        if (mnnz < 0) { free(agg1); return (int)mnnz; }
        /* pass 2 on M_1 = P_1^T A_l P_1 */
        int *agg2 = (int *)malloc(sizeof(int) * (size_t)nc1);
        if (!agg2) return OR_ERR_NOMEM;
        int nc2 = or_npair_pass(nc1, m_rp, m_ci, m_val, agg2);
        if (nc2 < 0) return nc2;
        int *c_rp = (int *)malloc(sizeof(int) * ((size_t)nc2 + 1));
        int *c_ci = (int *)malloc(sizeof(int) * (size_t)(mnnz + 1));
        double *c_val = (double *)malloc(sizeof(double) * (size_t)(mnnz + 1));
        if (!c_rp || !c_ci || !c_val) return OR_ERR_NOMEM;
        long cnnz = or_galerkin(nc1, m_rp, m_ci, m_val, agg2, nc2, c_rp, c_ci, c_val);
        if (cnnz < 0) return (int)cnnz;
        cur->agg = (int *)malloc(sizeof(int) * (size_t)cur->n);
        if (!cur->agg) return OR_ERR_NOMEM;
        for (int i = 0; i < cur->n; ++i)
            cur->agg[i] = agg2[agg1[i]];
        if ((double)nc2 > 0.9 * (double)cur->n) {
            /* stalled: absorb singletons, then one Galerkin product on A_l */
            int nc3 = or_absorb_singletons(cur->n, cur->rp, cur->ci, cur->val, cur->agg, nc2);
            if (nc3 < 0) return nc3;
            if (nc3 < nc2) {
                cnnz = or_galerkin(cur->n, cur->rp, cur->ci, cur->val, cur->agg, nc3, c_rp, c_ci,
                                   c_val);
                if (cnnz < 0) return (int)cnnz;
                nc2 = nc3;
            }
        }
        cur->nc = nc2;
        free(agg1); free(agg2); free(m_rp); free(m_ci); free(m_val);
        ++l;
        L[l].n = nc2; L[l].rp = c_rp; L[l].ci = c_ci; L[l].val = c_val;
        c->nlev = l + 1;
    }
    c->nlev = l + 1;
    /* every level needs a nonzero diagonal for Gauss-Seidel */
    for (int q = 0; q < c->nlev - 1; ++q) {
        or_level *cur = &L[q];
        for (int i = 0; i < cur->n; ++i) {
            int kd = find_col(cur->rp, cur->ci, i, i);
            if (kd < 0 || cur->val[kd] == 0.0)
                return OR_ERR_SINGULAR;
        }
    }
    int nL = L[c->nlev - 1].n;
    if (nL > OR_MAX_DENSE)
        return OR_ERR_COARSE;
    c->coarse_dense = (double *)calloc((size_t)nL * (size_t)nL, sizeof(double));
    if (!c->coarse_dense) return OR_ERR_NOMEM;
    or_level *cl = &L[c->nlev - 1];
    for (int i = 0; i < nL; ++i)
        for (int k = cl->rp[i]; k < cl->rp[i + 1]; ++k)
            c->coarse_dense[(long)i * nL + cl->ci[k]] = cl->val[k];
    return OR_OK;
}

static int store_matrix(or_ctx *c, int n, int b, int p, const int *rp, const int *ci,
                        const double *vals, long nnzb)
{
    free(c->rp); free(c->ci); free(c->A); free(c->A32);
    c->A32 = NULL;
    c->rp = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    c->ci = (int *)malloc(sizeof(int) * (size_t)nnzb);
    c->A = (double *)malloc(sizeof(double) * (size_t)(nnzb * b * b));
    if (!c->rp || !c->ci || !c->A)
        return OR_ERR_NOMEM;
    memcpy(c->rp, rp, sizeof(int) * ((size_t)n + 1));
    memcpy(c->ci, ci, sizeof(int) * (size_t)nnzb);
    memcpy(c->A, vals, sizeof(double) * (size_t)(nnzb * b * b));
    if (c->precond_fp32) {
        /* FP32 copy of the pressure columns A_cd[:,p] (RNE), one per setup */
        c->A32 = (float *)malloc(sizeof(float) * (size_t)(nnzb * b));
        if (!c->A32)
            return OR_ERR_NOMEM;
        for (long k = 0; k < nnzb; ++k)
            for (int r = 0; r < b; ++r)
                c->A32[k * b + r] = (float)vals[k * b * b + r * b + p];
    }
    c->n = n; c->b = b; c->p = p; c->nnzb = nnzb;
    return OR_OK;
}

/* A2  Adaptive SETUP (Sec. 3.2): the preconditioner is regenerated on the    */
/*     first system, when the previous solve took more than mu iterations,   */
/*     or when the size changed (Remark after the two cases); otherwise       */
/*     B^(i-1) is reused as B^(i).  The current A is always taken for the     */
/*     Krylov products and the residual steps of the preconditioner.          */
int or_setup(or_ctx *c, int n, int b, int p, const int *rp, const int *ci, const double *vals,
             long nnzb, int *rebuilt)
{
    int st = or_validate(n, b, p, rp, ci, vals, nnzb);
    if (st != OR_OK)
        return st;
    st = store_matrix(c, n, b, p, rp, ci, vals, nnzb);
    if (st != OR_OK)
        return st;
    int rebuild = !c->has_B || c->Bn != n || c->Bb != b || c->Bp != p || c->it_prev < 0 ||
                  c->it_prev > c->mu;
    *rebuilt = rebuild;
    if (!rebuild)
        return OR_OK;
    free_B(c);
    c->omega = (double *)malloc(sizeof(double) * (size_t)n * b);
    double *ap = (double *)malloc(sizeof(double) * (size_t)nnzb);
    int *rp0 = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    int *ci0 = (int *)malloc(sizeof(int) * (size_t)nnzb);
    if (!c->omega || !ap || !rp0 || !ci0)
        return OR_ERR_NOMEM;
    st = or_decouple(n, b, p, rp, ci, vals, c->omega, ap);
    if (st != OR_OK) { free(ap); free(rp0); free(ci0); return st; }
    memcpy(rp0, rp, sizeof(int) * ((size_t)n + 1));
    memcpy(ci0, ci, sizeof(int) * (size_t)nnzb);
    st = build_hierarchy(c, rp0, ci0, ap, n);
    if (st != OR_OK)
        return st;
    c->Brp = (int *)malloc(sizeof(int) * ((size_t)n + 1));
    c->Bci = (int *)malloc(sizeof(int) * (size_t)nnzb);
    c->F = (double *)malloc(sizeof(double) * (size_t)(nnzb * b * b));
    c->Dinv = (double *)malloc(sizeof(double) * (size_t)n * b * b);
    if (!c->Brp || !c->Bci || !c->F || !c->Dinv)
        return OR_ERR_NOMEM;
    memcpy(c->Brp, rp, sizeof(int) * ((size_t)n + 1));
    memcpy(c->Bci, ci, sizeof(int) * (size_t)nnzb);
    c->Bord = (int *)malloc(sizeof(int) * (size_t)n);
    if (!c->Bord)
        return OR_ERR_NOMEM;
    if (c->bilu_order == 1) {
        st = or_multicolor_order(n, rp, ci, c->Bord);
        if (st < 0)
            return st;
    } else {
        for (int t = 0; t < n; ++t)
            c->Bord[t] = t;
    }
    if (c->full_smoother == 1) {
        /* block Jacobi: the inverse of every diagonal block, as in the block */
        /* ILU(0) pivot inversions                                           */
        c->Djac = (double *)malloc(sizeof(double) * (size_t)n * b * b);
        if (!c->Djac)
            return OR_ERR_NOMEM;
        for (int cc = 0; cc < n; ++cc) {
            int kd = find_col(rp, ci, cc, cc);
            st = block_inverse(b, vals + (long)kd * b * b, c->Djac + (long)cc * b * b);
            if (st != OR_OK)
                return st;
        }
    } else {
        st = or_bilu0_factor_ordered(n, b, rp, ci, vals, c->Bord, c->F, c->Dinv);
        if (st != OR_OK)
            return st;
    }
    if (c->n_stage) {
        st = setup_n_stage(c, n, b, p, rp, ci, vals, nnzb);
        if (st != OR_OK)
            return st;
    }
    if (c->precond_fp32) {
        /* O13: FP32 copies by IEEE round-to-nearest-even of the FP64 setup */
        for (int l = 0; l < c->nlev; ++l) {
            or_level *L = &c->lev[l];
            L->val32 = round_f32(L->val, L->rp[L->n]);
            if (!L->val32) return OR_ERR_NOMEM;
        }
        if (c->n_stage) {
            c->Dn32 = round_f32(c->Dn, (long)n * (b - 1) * b);
            c->Ann32 = round_f32(c->Ann, nnzb * (b - 1) * (b - 1));
            if (!c->Dn32 || !c->Ann32) return OR_ERR_NOMEM;
        }
        if (c->full_smoother == 1) {
            c->Djac32 = round_f32(c->Djac, (long)n * b * b);
            if (!c->Djac32) return OR_ERR_NOMEM;
        } else {
            c->F32 = round_f32(c->F, nnzb * b * b);
            c->Dinv32 = round_f32(c->Dinv, (long)n * b * b);
            if (!c->F32 || !c->Dinv32) return OR_ERR_NOMEM;
        }
    }
    c->Bn = n; c->Bb = b; c->Bp = p; c->Bnnzb = nnzb;
    c->has_B = 1;
    c->setup_calls++;
    return OR_OK;
}

int or_coarse_n(const or_ctx *c) { return c->nlev > 0 ? c->lev[c->nlev - 1].n : 0; }

void or_get_coarse_dense(const or_ctx *c, double *out)
{
    long m = (long)or_coarse_n(c);
    memcpy(out, c->coarse_dense, sizeof(double) * (size_t)(m * m));
}

/* O8  the coarsest level is solved directly: LU factors with row            */
/*     interchanges as returned by LAPACK getrf (0-based pivots).            */
int or_set_coarse_lu(or_ctx *c, const double *lu, const int *piv)
{
    long m = (long)or_coarse_n(c);
    free(c->LU); free(c->piv);
    c->LU = (double *)malloc(sizeof(double) * (size_t)(m * m));
    c->piv = (int *)malloc(sizeof(int) * (size_t)m);
    if (!c->LU || !c->piv)
        return OR_ERR_NOMEM;
    memcpy(c->LU, lu, sizeof(double) * (size_t)(m * m));
    memcpy(c->piv, piv, sizeof(int) * (size_t)m);
    for (long i = 0; i < m; ++i)
        if (c->LU[i * m + i] == 0.0)
            return OR_ERR_SINGULAR;
    c->have_lu = 1;
    return OR_OK;
}

void or_lu_solve(int m, const double *LU, const int *piv, const double *f, double *x)
{
    for (int i = 0; i < m; ++i)
        x[i] = f[i];
    for (int i = 0; i < m; ++i) {
        int j = piv[i];
        if (j != i) {
            double t = x[i]; x[i] = x[j]; x[j] = t;
        }
    }
    for (int i = 0; i < m; ++i) {
        double acc = 0.0;
        for (int j = 0; j < i; ++j)
            acc = acc + LU[(long)i * m + j] * x[j];
        x[i] = x[i] - acc;
    }
    for (int i = m - 1; i >= 0; --i) {
        double acc = 0.0;
        for (int j = i + 1; j < m; ++j)
            acc = acc + LU[(long)i * m + j] * x[j];
        x[i] = (x[i] - acc) / LU[(long)i * m + i];
    }
}

/* O10 V-cycle and O9 preconditioner apply, in the chosen precision. */
#define REAL double
#define SFX(name) name##_f64
#define LEVVAL(L) ((L)->val)
#define APCOL(c, q, k) ((c)->A[(long)(q) * (c)->b * (c)->b + (long)(k) * (c)->b + (c)->p])
#define BILU_F(c) ((c)->F)
#define BILU_D(c) ((c)->Dinv)
#define DJAC(c) ((c)->Djac)
#define DN(c) ((c)->Dn)
#define ANN(c) ((c)->Ann)
#include "oracle_cycle.inc"
#undef REAL
#undef SFX
#undef LEVVAL
#undef APCOL
#undef BILU_F
#undef BILU_D
#undef DJAC
#undef DN
#undef ANN
#define REAL float
#define SFX(name) name##_f32
#define LEVVAL(L) ((L)->val32)
#define APCOL(c, q, k) ((c)->A32[(long)(q) * (c)->b + (k)])
#define BILU_F(c) ((c)->F32)
#define BILU_D(c) ((c)->Dinv32)
#define DJAC(c) ((c)->Djac32)
#define DN(c) ((c)->Dn32)
#define ANN(c) ((c)->Ann32)
#include "oracle_cycle.inc"
#undef REAL
#undef SFX
#undef LEVVAL
#undef APCOL
#undef BILU_F
#undef BILU_D
#undef DJAC
#undef DN
#undef ANN

/* z = B v, the multiplicative two-stage preconditioner (Alg. 3.1, stages P  */
/* then R, initial w = 0) in the reduced form                                  */
/*   g_P = w . v;  e = Vcycle(g_P);  r = v - A Pi_P e;  z = Pi_P e + (LU)^-1 r */
/* which equals Alg. 3.1 on the decoupled system (W A, W v), W = blockdiag    */
/* (D_c^{-1}), because ILU(0)(W A) = W ILU(0)(A).                              */
int or_apply(or_ctx *c, const double *v, double *z)
{
    if (!c->has_B || !c->have_lu)
        return OR_ERR_STATE;
    if (c->precond_fp32)
        return msp_apply_f32(c, v, z);
    return msp_apply_f64(c, v, z);
}

int or_vcycle(or_ctx *c, const double *f, double *x)
{
    if (!c->has_B || !c->have_lu)
        return OR_ERR_STATE;
    return vcycle_f64(c, 0, f, x);
}

/* The R stage on its own (FP64): z = (LU)^{-1} r for block ILU(0), or       */
/* z_c = A_cc^{-1} r_c for block Jacobi.                                       */
int or_bilu_apply(or_ctx *c, const double *r, double *z)
{
    if (!c->has_B)
        return OR_ERR_STATE;
    if (c->full_smoother == 1)
        block_jacobi_f64(c->Bn, c->Bb, c->Djac, r, z);
    else
        bilu0_solve_f64(c->Bn, c->Bb, c->Brp, c->Bci, c->F, c->Dinv, c->Bord, r, z);
    return OR_OK;
}

/* Block SpMV y = A x with the current matrix. */
void or_spmv(const or_ctx *c, const double *x, double *y)
{
    bsr_spmv_f64(c->n, c->b, c->rp, c->ci, c->A, x, y);
}

static double dot(long N, const double *a, const double *b)
{
    double s = 0.0;
    for (long i = 0; i < N; ++i)
        s = s + a[i] * b[i];
    return s;
}

/* ------------------------------------------------------------------------ */
/* O11 Restarted flexible GMRES(m), right preconditioned, modified           */
/*     Gram-Schmidt Arnoldi, Givens rotations; the paper's GMRES(m) with      */
/*     m = 30 and a relative-residual stopping test.  One iteration is one    */
/*     Arnoldi step (one preconditioner application), counted over restarts.  */
/*     Stopping: |g_{j+1}| <= rtol ||b|| ends a cycle; the true residual        */
/*     ||b - A x|| <= rtol ||b|| ends the solve; max_iter caps the total.     */
/* ------------------------------------------------------------------------ */
int or_solve(or_ctx *c, const double *rhs, double *x, double rtol, int *iters, double *relres)
{
    if (!c->has_B || !c->have_lu)
        return OR_ERR_STATE;
    const long N = (long)c->n * c->b;
    const int m = c->restart;
    for (long i = 0; i < N; ++i)
        if (!isfinite(rhs[i]))
            return OR_ERR_NONFINITE;
    double *V = (double *)malloc(sizeof(double) * (size_t)(N * (m + 1)));
    double *Z = (double *)malloc(sizeof(double) * (size_t)(N * m));
    double *w = (double *)malloc(sizeof(double) * (size_t)N);
    double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = (double *)malloc(sizeof(double) * (size_t)m);
    double *sn = (double *)malloc(sizeof(double) * (size_t)m);
    double *g = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    double *y = (double *)malloc(sizeof(double) * (size_t)m);
    if (!V || !Z || !w || !H || !cs || !sn || !g || !y) {
        free(V); free(Z); free(w); free(H); free(cs); free(sn); free(g); free(y);
        return OR_ERR_NOMEM;
    }
    int it = 0, status = OR_OK;
    double bnorm = sqrt(dot(N, rhs, rhs));
    double tol = rtol * bnorm;
    double beta;
    *relres = 0.0;
    if (bnorm == 0.0) {
        for (long i = 0; i < N; ++i)
            x[i] = 0.0;
        goto done;
    }
    /* r = b - A x */
    or_spmv(c, x, w);
    for (long i = 0; i < N; ++i)
        w[i] = rhs[i] - w[i];
    beta = sqrt(dot(N, w, w));
    while (beta > tol) {
        if (it >= c->max_iter) {
            status = OR_NOT_CONVERGED;
            break;
        }
        for (long i = 0; i < N; ++i)
            V[i] = w[i] / beta;
        for (int q = 0; q <= m; ++q)
            g[q] = 0.0;
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m; ++j) {
            int st = or_apply(c, V + (long)j * N, Z + (long)j * N);
            if (st != OR_OK) { status = st; goto done; }
            or_spmv(c, Z + (long)j * N, w);
            for (int i = 0; i <= j; ++i) {
                double h = dot(N, w, V + (long)i * N);
                H[i * m + j] = h;
                for (long q = 0; q < N; ++q)
                    w[q] = w[q] - h * V[(long)i * N + q];
            }
            double hn = sqrt(dot(N, w, w));
            H[(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                double a = H[i * m + j], bq = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * bq;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * bq;
            }
            double a = H[j * m + j], bq = H[(j + 1) * m + j];
            double d = hypot(a, bq);
            cs[j] = a / d;
            sn[j] = bq / d;
            H[j * m + j] = d;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++it;
            k = j + 1;
            if (hn == 0.0 || fabs(g[j + 1]) <= tol || it >= c->max_iter)
                break;
            for (long q = 0; q < N; ++q)
                V[(long)(j + 1) * N + q] = w[q] / hn;
        }
        /* y = H_k^{-1} g_k (upper triangular), x += Z_k y */
        for (int i = k - 1; i >= 0; --i) {
            double acc = g[i];
            for (int q = i + 1; q < k; ++q)
                acc = acc - H[i * m + q] * y[q];
            y[i] = acc / H[i * m + i];
        }
        for (int i = 0; i < k; ++i)
            for (long q = 0; q < N; ++q)
                x[q] = x[q] + y[i] * Z[(long)i * N + q];
        or_spmv(c, x, w);
        for (long i = 0; i < N; ++i)
            w[i] = rhs[i] - w[i];
        beta = sqrt(dot(N, w, w));
    }
    *relres = (bnorm > 0.0) ? beta / bnorm : 0.0;
done:
    *iters = it;
    c->it_prev = it;
    c->solves++;
    free(V); free(Z); free(w); free(H); free(cs); free(sn); free(g); free(y);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Getters (tests compare these bit for bit with the GPU library).           */
/* ------------------------------------------------------------------------ */
int or_nlevels(const or_ctx *c) { return c->nlev; }
int or_setup_calls(const or_ctx *c) { return c->setup_calls; }
int or_level_n(const or_ctx *c, int l) { return c->lev[l].n; }
long or_level_nnz(const or_ctx *c, int l) { return c->lev[l].rp[c->lev[l].n]; }
int or_level_ncolors(const or_ctx *c, int l) { return c->lev[l].g; }
int or_level_nc(const or_ctx *c, int l) { return c->lev[l].nc; }

void or_get_level(const or_ctx *c, int l, int *rp, int *ci, double *val, int *color, int *agg)
{
    const or_level *L = &c->lev[l];
    long nnz = L->rp[L->n];
    if (rp) memcpy(rp, L->rp, sizeof(int) * ((size_t)L->n + 1));
    if (ci) memcpy(ci, L->ci, sizeof(int) * (size_t)nnz);
    if (val) memcpy(val, L->val, sizeof(double) * (size_t)nnz);
    if (color && L->color) memcpy(color, L->color, sizeof(int) * (size_t)L->n);
    if (agg && L->agg) memcpy(agg, L->agg, sizeof(int) * (size_t)L->n);
}

void or_get_omega(const or_ctx *c, double *out)
{
    memcpy(out, c->omega, sizeof(double) * (size_t)c->Bn * c->Bb);
}

/* N-stage data (n_stage = 1): Dn (n x (b-1) x b) and Ann (nnzb x (b-1)^2). */
int or_get_nstage(const or_ctx *c, double *Dn, double *Ann)
{
    if (!c->has_B || !c->n_stage || !c->Dn)
        return OR_ERR_STATE;
    const long m = c->Bb - 1;
    if (Dn) memcpy(Dn, c->Dn, sizeof(double) * (size_t)(c->Bn * m * c->Bb));
    if (Ann) memcpy(Ann, c->Ann, sizeof(double) * (size_t)(c->Bnnzb * m * m));
    return OR_OK;
}

/* R-stage data: block ILU(0) factors F and pivot inverses, or (block Jacobi) */
/* no F and the diagonal-block inverses in Dinv.                              */
void or_get_bilu(const or_ctx *c, double *F, double *Dinv)
{
    if (F && c->F) memcpy(F, c->F, sizeof(double) * (size_t)(c->Bnnzb * c->Bb * c->Bb));
    const double *D = c->full_smoother == 1 ? c->Djac : c->Dinv;
    if (Dinv && D) memcpy(Dinv, D, sizeof(double) * (size_t)c->Bn * c->Bb * c->Bb);
}
