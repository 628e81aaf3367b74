"""Element-wise checks shared by the GPU parity tests.

Every check bounds each entry on its own, never a norm of the whole vector, so
one wrong row cannot hide behind the size of the others:

* `assert_entrywise`: |g_i - o_i| <= tol * scale_i for a given scale vector;
* `spmv_scale`: (|A| |x|)_i, the natural scale of one row of a sparse product;
* `gs_local_residual`: a Gauss-Seidel sweep's output satisfies its own row
  equations (each row against the values its neighbours had when it was
  updated), relative to the size of the terms of that row;
* `bilu_backward_error`: z = (LU)^-1 r satisfies L U z = r row by row,
  relative to (|L| |U| |z| + |r|)_i;
* `dense_backward_error`: a direct solve satisfies A x = f row by row,
  relative to (|A| |x| + |f|)_i.

They use the oracle's matrices (natural order) and plain numpy/scipy
products; none of them runs any of the library's code.
"""
import numpy as np
import scipy.sparse as sp


def assert_entrywise(g, o, tol, scale, what):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    scale = np.broadcast_to(np.asarray(scale, dtype=np.float64), o.shape)
    err = np.abs(g - o)
    bound = tol * scale
    bad = ~(err <= bound)
    if bad.any():
        ratio = np.where(bound > 0, err / np.maximum(bound, 1e-300), np.inf)
        i = int(np.argmax(ratio))
        raise AssertionError(f"{what}: {int(bad.sum())} of {o.size} entries beyond "
                             f"{tol:g} * scale; worst entry {i}: gpu {g[i]!r} oracle {o[i]!r} "
                             f"err {err[i]:.3e} scale {scale[i]:.3e}")
    return float(np.max(err / np.maximum(scale, 1e-300))) if o.size else 0.0


def close(g, o, tol, what):
    """Entry by entry: |g_i - o_i| <= tol * max_j |o_j|."""
    return assert_entrywise(g, o, tol, inf_scale(o), what)


def blocks_close(g, o, tol, what):
    """Block arrays [k, b, b]: each block within tol of its largest oracle entry."""
    o = np.asarray(o)
    sc = np.abs(o).reshape(o.shape[0], -1).max(axis=1)
    return assert_entrywise(np.asarray(g).reshape(o.shape[0], -1),
                            o.reshape(o.shape[0], -1), tol, sc[:, None], what)


def coarse_tol_of(level):
    """kappa(A_L) * 1e-15, clipped to [1e-12, 1e-10]: the bar for stages that
    include the coarsest solve.  kappa_2 by SVD up to 2000 rows, above that
    the 1-norm estimate ||A||_1 ||A^-1||_1 (same order of magnitude)."""
    A = csr(level)
    m = level["n"]
    if m <= 2000:
        kappa = np.linalg.cond(A.toarray())
    else:
        import scipy.sparse.linalg as spla
        lu = spla.splu(A.tocsc())
        inv = spla.LinearOperator((m, m), matvec=lu.solve, rmatvec=lambda y: lu.solve(y, "T"))
        kappa = spla.norm(A, 1) * spla.onenormest(inv)
    return max(1e-12, min(1e-10, kappa * 1e-15))


def inf_scale(o):
    """Every entry measured against the largest |o_j|."""
    return np.full(np.shape(o), float(np.max(np.abs(o))) if np.size(o) else 0.0)


def bsr(sys_or_parts, b=None):
    """scipy BSR matrix of a system (or of (row_ptr, col_ind, vals[nnzb, b, b]))."""
    if isinstance(sys_or_parts, tuple):
        rp, ci, vals = sys_or_parts
    else:
        rp, ci, vals = sys_or_parts.row_ptr, sys_or_parts.col_ind, sys_or_parts.vals
    vals = np.asarray(vals, dtype=np.float64)
    b = vals.shape[1]
    n = len(rp) - 1
    return sp.bsr_matrix((vals, np.asarray(ci), np.asarray(rp)), shape=(n * b, n * b))


def csr(level):
    n = level["n"]
    return sp.csr_matrix((level["val"], level["col_ind"], level["row_ptr"]), shape=(n, n))


def spmv_scale(A, x):
    return abs(A) @ np.abs(x)


def gs_local_residual(level, f, x0, x, forward, tol, what):
    """One multi-color Gauss-Seidel sweep from x0 gave x: for every row i,
    a_ii x_i = f_i - sum_j a_ij xt_j, where xt_j is x_j for neighbours in
    colors swept before i's color and x0_j for the rest (no neighbour shares
    i's color).  Checked row by row against |a_ii x_i| + |f_i| + sum |a_ij xt_j|."""
    rp, ci, val, col = level["row_ptr"], level["col_ind"], level["val"], level["color"]
    n = level["n"]
    rows = np.repeat(np.arange(n), np.diff(rp))
    key = col if forward else -col
    diag = rows == ci
    assert not np.any((col[rows] == col[ci]) & ~diag), "a row shares its color with a neighbour"
    before = key[ci] < key[rows]
    xt = np.where(before, x[ci], x0[ci])
    off = np.where(diag, 0.0, val * xt)
    aii = np.zeros(n)
    aii[rows[diag]] = val[diag]
    lhs = aii * x - (f - np.bincount(rows, weights=off, minlength=n))
    scale = np.abs(aii * x) + np.abs(f) + np.bincount(rows, weights=np.abs(off), minlength=n)
    return assert_entrywise(lhs, np.zeros(n), tol, scale, what)


def bilu_factors(sys_, F, Dinv, order):
    """L (unit block-lower in the elimination order) and U (upper, with the
    factored pivot blocks on its diagonal) as scipy BSR matrices, from the
    oracle's factor array F (natural BSR order of the system's pattern)."""
    n, b = sys_.n, sys_.b
    rp, ci = sys_.row_ptr, sys_.col_ind
    pos = np.empty(n, dtype=np.int64)
    pos[np.asarray(order)] = np.arange(n)
    rows = np.repeat(np.arange(n), np.diff(rp))
    low = pos[ci] < pos[rows]
    Fl = np.where(low[:, None, None], F, 0.0)
    Fl[rows == ci] = np.eye(b)  # the unit diagonal of L
    Fu = np.where(low[:, None, None], 0.0, F)
    L = sp.bsr_matrix((Fl, ci, rp), shape=(n * b, n * b))
    U = sp.bsr_matrix((Fu, ci, rp), shape=(n * b, n * b))
    return L, U


def bilu_backward_error(L, U, r, z, tol, what):
    w = U @ z
    res = L @ w - r
    scale = abs(L) @ (abs(U) @ np.abs(z)) + np.abs(r)
    return assert_entrywise(res, np.zeros_like(res), tol, scale, what)


def dense_backward_error(A, x, f, tol, what):
    res = A @ x - f
    scale = abs(A) @ np.abs(x) + np.abs(f)
    return assert_entrywise(res, np.zeros_like(res), tol, scale, what)
