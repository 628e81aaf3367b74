"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a literal
transcription of the paper's set-based algorithm, a dense textbook operator,
a closed form, an exact rational solve or a library routine used on a
*different* formulation.  CPU only.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

from oracle import oracle as O
from paper_2208_08594_amd import synth


# --------------------------------------------------------------------------
# helpers
# --------------------------------------------------------------------------
def csr_from_dense_pattern(P):
    P = np.asarray(P, dtype=bool)
    n = P.shape[0]
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum(P.sum(1))
    ci = np.nonzero(P)[1].astype(np.int32)
    return rp, ci


def sym_adjacency(rp, ci):
    n = len(rp) - 1
    S = [set() for _ in range(n)]
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            j = int(ci[k])
            if j != i:
                S[i].add(j)
                S[j].add(i)
    return S


def literal_grouping(n, S):
    """Alg. 4.2 around Alg. 4.1 written with Python sets, line by line, with the
    paper's else-branch.  'Undetermined' = not yet placed in any group; the
    second-ring candidates therefore may include vertices already pushed to
    W-bar, which the else-branch discards."""
    deg = [len(S[i]) for i in range(n)]
    key = lambda v: (-deg[v], v)
    assigned = set()
    Vcur = set(range(n))
    groups = []
    while Vcur:
        Vin = set(Vcur)
        V = set(Vcur)
        W, Wbar, What = set(), set(), set()
        while V:
            i = min(What, key=key) if What else min(V, key=key)
            if not (S[i] & W):
                W.add(i)
                V.discard(i)
                What.discard(i)
                Wbar |= (S[i] & Vin)
                V -= S[i]
                second = set()
                for k in S[i]:
                    second |= S[k]
                second -= S[i] | {i}
                What |= {j for j in second if j not in assigned and j not in W}
            else:
                Wbar.add(i)
                V.discard(i)
                What.discard(i)
        groups.append(W)
        assigned |= W
        Vcur = Wbar - W
    return groups


def dense_from_csr(rp, ci, val, n=None):
    n = n or len(rp) - 1
    A = np.zeros((n, n))
    for i in range(len(rp) - 1):
        A[i, ci[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
    return A


def bsr_b1(rp, ci, val):
    return val.reshape(-1, 1, 1)


def random_pattern(n, density, seed, symmetric):
    rng = np.random.default_rng(seed)
    P = rng.random((n, n)) < density
    if symmetric:
        P = P | P.T
    np.fill_diagonal(P, True)
    return csr_from_dense_pattern(P)


# --------------------------------------------------------------------------
# generator
# --------------------------------------------------------------------------
def test_generator_is_seeded_and_well_formed():
    a = synth.config(0, seed=3)
    b = synth.config(0, seed=3)
    c = synth.config(0, seed=4)
    assert np.array_equal(a.vals, b.vals) and np.array_equal(a.rhs, b.rhs)
    assert not np.array_equal(a.vals, c.vals)
    assert a.n == 1000 and a.N == 4000 and a.nnzb == 6400
    assert O.validate(a.n, a.b, a.p, a.row_ptr, a.col_ind, a.vals) == 0
    for w in a.wells:
        blk = a.vals[a.diag_pos[w]]
        assert np.array_equal(blk[a.p], np.eye(a.b)[a.p])


# --------------------------------------------------------------------------
# O4: VerticesGrouping (Alg. 4.1/4.2) -- pins P2, P3, P4
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("symmetric", [True, False])
def test_coloring_matches_literal_algorithm(seed, symmetric):
    n = 20 + 7 * seed
    rp, ci = random_pattern(n, 0.08 + 0.01 * (seed % 4), seed, symmetric)
    col, g = O.color(rp, ci)
    groups = literal_grouping(n, sym_adjacency(rp, ci))
    lit = np.zeros(n, dtype=np.int32)
    for gi, W in enumerate(groups):
        for v in W:
            lit[v] = gi + 1
    assert g == len(groups)
    assert np.array_equal(col, lit)


@pytest.mark.parametrize("seed", range(8))
def test_coloring_principles(seed):
    """(i) cover, (ii) disjoint, (iii) no edge inside a group (a_ij = a_ji = 0),
    and every group is a maximal independent set of what was left."""
    n = 150
    rp, ci = random_pattern(n, 0.03, 100 + seed, symmetric=False)
    col, g = O.color(rp, ci)
    S = sym_adjacency(rp, ci)
    assert col.min() == 1 and col.max() == g
    for i in range(n):
        for j in S[i]:
            assert col[i] != col[j]
    for i in range(n):
        for earlier in range(1, col[i]):
            assert any(col[j] == earlier for j in S[i]), "group not maximal"


@pytest.mark.parametrize("shape", [(10, 10, 10), (7, 5, 3), (64, 1, 1), (6, 9, 1), (64, 64, 4)])
def test_coloring_seven_point_is_red_black(shape):
    nx, ny, nz = shape
    rp, ci, _ = synth.poisson_csr(shape)
    col, g = O.color(rp, ci)
    assert g == 2
    c = np.arange(nx * ny * nz)
    parity = (c % nx + (c // nx) % ny + c // (nx * ny)) % 2
    # both colors are parity classes: red-black GS is the g = 2 case
    assert len(set(zip(parity.tolist(), col.tolist()))) == 2


def test_coloring_complete_graph_is_classical_gs():
    n = 9
    rp, ci = csr_from_dense_pattern(np.ones((n, n), bool))
    col, g = O.color(rp, ci)
    assert g == n and sorted(col.tolist()) == list(range(1, n + 1))


@pytest.mark.parametrize("seed", range(4))
def test_color_submatrix_is_diagonal(seed):
    rp, ci = random_pattern(60, 0.07, 200 + seed, symmetric=False)
    col, g = O.color(rp, ci)
    A = dense_from_csr(rp, ci, np.ones(len(ci)))
    for l in range(1, g + 1):
        idx = np.nonzero(col == l)[0]
        sub = A[np.ix_(idx, idx)]
        assert np.count_nonzero(sub - np.diag(np.diag(sub))) == 0


# --------------------------------------------------------------------------
# O10 sweep -- pin P5
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(4))
def test_gs_sweep_is_dense_triangular_solve(seed):
    rng = np.random.default_rng(seed)
    n = 80
    rp, ci = random_pattern(n, 0.06, 300 + seed, symmetric=bool(seed % 2))
    val = rng.uniform(-1, 1, len(ci))
    rows = np.repeat(np.arange(n), np.diff(rp))
    val[rows == ci] = 8.0 + rng.random(n)
    col, g = O.color(rp, ci)
    A = dense_from_csr(rp, ci, val)
    f = rng.uniform(-1, 1, n)
    x0 = rng.uniform(-1, 1, n)
    perm = np.argsort(col, kind="stable")
    Ap = A[np.ix_(perm, perm)]
    L = np.tril(Ap, -1)
    U = np.triu(Ap, 1)
    D = np.diag(np.diag(Ap))
    fwd = scipy.linalg.solve_triangular(D + L, f[perm] - U @ x0[perm], lower=True)
    bwd = scipy.linalg.solve_triangular(D + U, f[perm] - L @ x0[perm], lower=False)
    xf = O.gs_sweep(rp, ci, val, col, g, f, x0, forward=True)
    xb = O.gs_sweep(rp, ci, val, col, g, f, x0, forward=False)
    np.testing.assert_allclose(xf[perm], fwd, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(xb[perm], bwd, rtol=1e-12, atol=1e-13)


def test_gs_sweep_rows_independent_inside_color():
    """Inside one color rows do not see each other (Alg. 4.3 runs them in
    parallel): updating all rows of a color at once from the values left by
    the previous colors gives the sequential sweep."""
    rng = np.random.default_rng(5)
    rp, ci = random_pattern(90, 0.05, 77, symmetric=False)
    n = len(rp) - 1
    val = rng.uniform(-1, 1, len(ci))
    rows = np.repeat(np.arange(n), np.diff(rp))
    val[rows == ci] = 6.0 + rng.random(n)
    col, g = O.color(rp, ci)
    A = dense_from_csr(rp, ci, val)
    f = rng.uniform(-1, 1, n)
    x0 = rng.uniform(-1, 1, n)
    d = np.diag(A)
    off = A - np.diag(d)
    x = x0.copy()
    for l in range(1, g + 1):
        idx = col == l
        x[idx] = (f[idx] - off[idx] @ x) / d[idx]
    np.testing.assert_allclose(O.gs_sweep(rp, ci, val, col, g, f, x0), x, rtol=1e-14, atol=1e-15)


# --------------------------------------------------------------------------
# O5/O6: aggregation and Galerkin -- pin P7 and invariants
# --------------------------------------------------------------------------
def _decoupled_level0(sys):
    om, ap = O.decouple(sys.n, sys.b, sys.p, sys.row_ptr, sys.col_ind, sys.vals)
    return sys.row_ptr, sys.col_ind, ap


@pytest.mark.parametrize("seed", range(3))
def test_npair_invariants(seed):
    sys = synth.lognormal_grid(9, 8, 5, 3, seed, 1.5, 0.1, "lateral4")
    rp, ci, ap = _decoupled_level0(sys)
    agg, nc = O.npair_pass(rp, ci, ap)
    n = sys.n
    sizes = np.bincount(agg, minlength=nc)
    assert sizes.min() >= 1 and sizes.max() <= 2 and sizes.sum() == n
    # aggregates numbered in order of creation = order of their first vertex
    first = np.array([np.min(np.nonzero(agg == a)[0]) for a in range(nc)])
    assert np.all(np.diff(first) > 0)
    A = dense_from_csr(rp, ci, ap)
    S = -(A + A.T) / 2
    np.fill_diagonal(S, -np.inf)
    for w in sys.wells:
        assert sizes[agg[w]] == 1, "Dirichlet rows stay single"
    for a in range(nc):
        mem = np.nonzero(agg == a)[0]
        if len(mem) == 2:
            i, j = mem
            smax = S[i][np.isfinite(S[i]) & (A[i] != 0) | (A[:, i] != 0)].max()
            assert S[i, j] > 0 and S[i, j] >= 0.25 * smax - 1e-15


@pytest.mark.parametrize("seed", range(3))
def test_galerkin_is_dense_ptap(seed):
    sys = synth.lognormal_grid(7, 6, 4, 4, seed, 1.0, 1.0, "corners2")
    rp, ci, ap = _decoupled_level0(sys)
    agg, nc = O.npair_pass(rp, ci, ap)
    crp, cci, cval = O.galerkin(rp, ci, ap, agg, nc)
    P = np.zeros((sys.n, nc))
    P[np.arange(sys.n), agg] = 1.0
    A = dense_from_csr(rp, ci, ap)
    Ac = P.T @ A @ P
    np.testing.assert_allclose(dense_from_csr(crp, cci, cval, nc), Ac, rtol=1e-13, atol=1e-14)
    # structural pattern: (I,J) stored iff some stored (i,j) maps onto it
    S0 = dense_from_csr(rp, ci, np.ones(len(ci)))
    pat = (P.T @ S0 @ P) > 0
    stored = dense_from_csr(crp, cci, np.ones(len(cci)), nc) > 0
    assert np.array_equal(pat, stored)
    for I in range(nc):
        assert np.all(np.diff(cci[crp[I]:crp[I + 1]]) > 0)


def test_stalled_level_absorbs_singletons_into_connected_aggregates():
    """A layered channelised grid whose coarsening stalls: the absorbed level
    still has compact aggregate ids, every aggregate is connected in the
    symmetrised pattern (an absorbed row joins a neighbour's aggregate), and
    the coarse matrix is the dense P^T A P of that level."""
    sys = synth.layered_grid(20, 44, 17, 4, 0)
    s = O.OracleSolver(max_coarse=60)
    s.setup(sys)
    sizes = [s.level(l)["n"] for l in range(s.nlevels)]
    jumps = [l for l in range(len(sizes) - 1) if sizes[l + 1] < sizes[l] / 5]
    assert jumps, sizes
    l = jumps[0]
    L = s.level(l)
    n, nc, agg = L["n"], L["nc"], L["agg"]
    assert sorted(set(agg.tolist())) == list(range(nc))
    S = sym_adjacency(L["row_ptr"], L["col_ind"])
    members = [[] for _ in range(nc)]
    for i in range(n):
        members[agg[i]].append(i)
    for mem in members:
        seen, stack = {mem[0]}, [mem[0]]
        ms = set(mem)
        while stack:
            u = stack.pop()
            for v in S[u]:
                if v in ms and v not in seen:
                    seen.add(v)
                    stack.append(v)
        assert seen == ms
    A = dense_from_csr(L["row_ptr"], L["col_ind"], L["val"])
    P = np.zeros((n, nc))
    P[np.arange(n), agg] = 1.0
    C = s.level(l + 1)
    np.testing.assert_allclose(dense_from_csr(C["row_ptr"], C["col_ind"], C["val"]), P.T @ A @ P,
                               rtol=1e-12, atol=1e-12 * np.abs(A).max())


def test_hierarchy_levels_and_coarsest():
    sys = synth.config(0)
    s = O.OracleSolver(max_coarse=64)
    s.setup(sys)
    ns = [s.level(l)["n"] for l in range(s.nlevels)]
    assert ns[0] == 1000 and ns[-1] <= 64 and all(a > b for a, b in zip(ns, ns[1:]))
    for l in range(s.nlevels - 1):
        L = s.level(l)
        sizes = np.bincount(L["agg"], minlength=ns[l + 1])
        assert sizes.min() >= 1 and sizes.max() <= 4


# --------------------------------------------------------------------------
# O2 decoupling -- pin P10
# --------------------------------------------------------------------------
@pytest.mark.parametrize("b", [3, 4, 7])
def test_abf_decoupling(b):
    sys = synth.lognormal_grid(5, 4, 3, b, 11, 1.0, 1.0, "corners2")
    om, ap = O.decouple(sys.n, sys.b, sys.p, sys.row_ptr, sys.col_ind, sys.vals)
    for c in range(sys.n):
        D = sys.vals[sys.diag_pos[c]]
        np.testing.assert_allclose(om[c], np.linalg.inv(D)[sys.p], rtol=1e-12, atol=1e-14)
        # w_c^T D_c = e_p^T: the decoupled diagonal block is the identity on row p
        np.testing.assert_allclose(om[c] @ D, np.eye(b)[sys.p], atol=1e-14)
    np.testing.assert_allclose(ap[sys.diag_pos], 1.0, rtol=1e-13)


def test_abf_singular_block_is_reported():
    sys = synth.lognormal_grid(3, 3, 1, 3, 0, 1.0, 1.0, "none")
    vals = sys.vals.copy()
    vals[sys.diag_pos[4]] = 0.0
    with pytest.raises(O.OracleError) as e:
        O.decouple(sys.n, sys.b, sys.p, sys.row_ptr, sys.col_ind, vals)
    assert e.value.code == -3


# --------------------------------------------------------------------------
# O7 block ILU(0) -- pin P8
# --------------------------------------------------------------------------
def _dense_lu_from_factors(sys_rp, sys_ci, F, D, n, b):
    L = np.eye(n * b)
    U = np.zeros((n * b, n * b))
    for i in range(n):
        for k in range(sys_rp[i], sys_rp[i + 1]):
            j = sys_ci[k]
            if j < i:
                L[i * b:(i + 1) * b, j * b:(j + 1) * b] = F[k]
            elif j > i:
                U[i * b:(i + 1) * b, j * b:(j + 1) * b] = F[k]
        U[i * b:(i + 1) * b, i * b:(i + 1) * b] = np.linalg.inv(D[i])
    return L, U


@pytest.mark.parametrize("b", [1, 3, 4])
def test_bilu0_defining_property(b):
    sys = synth.lognormal_grid(5, 4, 3, b, 21, 1.0, 1.0, "corners2")
    F, D = O.bilu0_factor(sys.n, b, sys.row_ptr, sys.col_ind, sys.vals)
    L, U = _dense_lu_from_factors(sys.row_ptr, sys.col_ind, F, D, sys.n, b)
    LU = L @ U
    A = sys.to_dense()
    for i in range(sys.n):
        for k in range(sys.row_ptr[i], sys.row_ptr[i + 1]):
            j = sys.col_ind[k]
            np.testing.assert_allclose(LU[i * b:(i + 1) * b, j * b:(j + 1) * b],
                                       A[i * b:(i + 1) * b, j * b:(j + 1) * b],
                                       rtol=1e-11, atol=1e-11)
    r = np.random.default_rng(0).uniform(-1, 1, sys.N)
    z = O.bilu0_solve(sys.n, b, sys.row_ptr, sys.col_ind, F, D, r)
    np.testing.assert_allclose(LU @ z, r, rtol=1e-10, atol=1e-12)


def test_bilu0_exact_on_block_tridiagonal_one_iteration():
    """1-D grid: ILU(0) has no dropped fill, so LU = A and the preconditioner is
    the exact inverse: FGMRES converges in one iteration (the paper's remark
    that one iteration means an exact inverse)."""
    sys = synth.lognormal_grid(40, 1, 1, 4, 2, 1.0, 1.0, "corners2")
    F, D = O.bilu0_factor(sys.n, sys.b, sys.row_ptr, sys.col_ind, sys.vals)
    L, U = _dense_lu_from_factors(sys.row_ptr, sys.col_ind, F, D, sys.n, sys.b)
    np.testing.assert_allclose(L @ U, sys.to_dense(), rtol=1e-12, atol=1e-10)
    s = O.OracleSolver(max_coarse=8, bilu_order=0)
    s.setup(sys)
    x, it, rr, st = s.solve(sys.rhs, 1e-10)
    assert it == 1 and rr <= 1e-10


# --------------------------------------------------------------------------
# O9 apply -- pins P1, P9 (Alg. 3.1 and eq. MSP)
# --------------------------------------------------------------------------
def _dense_operator(fn, n):
    return np.stack([fn(np.eye(n)[:, j]) for j in range(n)], axis=1)


@pytest.mark.parametrize("max_coarse,full_smoother,n_stage", [
    (10000, 0, 0), (4, 0, 0), (4, 1, 0), (4, 0, 1), (4, 1, 1), (10000, 0, 1)])
def test_reduced_apply_equals_literal_alg31(max_coarse, full_smoother, n_stage):
    sys = synth.lognormal_grid(3, 3, 2, 3, 7, 1.0, 1.0, [0])
    n, b, p, N = sys.n, sys.b, sys.p, sys.N
    s = O.OracleSolver(max_coarse=max_coarse, bilu_order=0, full_smoother=full_smoother,
                       n_stage=n_stage)
    s.setup(sys)
    A = sys.to_dense()
    W = np.zeros((N, N))
    for c in range(n):
        W[c * b:(c + 1) * b, c * b:(c + 1) * b] = np.linalg.inv(sys.vals[sys.diag_pos[c]])
    Ah = W @ A
    PiP = np.zeros((N, n))
    PiP[np.arange(n) * b + p, np.arange(n)] = 1.0
    # pressure block of the decoupled system is the oracle's level-0 matrix
    L0 = s.level(0)
    np.testing.assert_allclose(dense_from_csr(L0["row_ptr"], L0["col_ind"], L0["val"]),
                               PiP.T @ Ah @ PiP, rtol=1e-12, atol=1e-13)
    BP = _dense_operator(s.vcycle, n)
    if full_smoother == 0:
        # R = (ILU0(W A))^{-1}: factor the decoupled blocks (a different input)
        vals_hat = np.stack([np.linalg.inv(sys.vals[sys.diag_pos[c]]) @ sys.vals[k]
                             for c in range(n) for k in range(sys.row_ptr[c], sys.row_ptr[c + 1])])
        Fh, Dh = O.bilu0_factor(n, b, sys.row_ptr, sys.col_ind, vals_hat)
        Lh, Uh = _dense_lu_from_factors(sys.row_ptr, sys.col_ind, Fh, Dh, n, b)
        R = np.linalg.inv(Lh @ Uh)
    else:
        # block Jacobi on the decoupled system: its diagonal blocks are I
        np.testing.assert_allclose(np.stack([Ah[c * b:(c + 1) * b, c * b:(c + 1) * b]
                                             for c in range(n)]),
                                   np.broadcast_to(np.eye(b), (n, b, b)), atol=1e-13)
        R = np.eye(N)
    I = np.eye(N)
    if n_stage:
        # B_N: one block Gauss-Seidel sweep on the decoupled concentration
        # block, cells in the order of the block graph's groups
        keep = np.array([k for c in range(n) for k in range(c * b, (c + 1) * b) if k != c * b + p])
        PiN = np.zeros((N, len(keep)))
        PiN[keep, np.arange(len(keep))] = 1.0
        Ann = PiN.T @ Ah @ PiN
        col, _ = O.color(sys.row_ptr, sys.col_ind)
        m = b - 1
        order = np.argsort(col, kind="stable")
        perm = np.concatenate([np.arange(c * m, (c + 1) * m) for c in order])
        Ap = Ann[np.ix_(perm, perm)]
        lower = np.zeros_like(Ap)
        for bi in range(n):
            for bj in range(bi + 1):
                lower[bi * m:(bi + 1) * m, bj * m:(bj + 1) * m] = Ap[bi * m:(bi + 1) * m,
                                                                      bj * m:(bj + 1) * m]
        inv = np.argsort(perm)
        BN = np.linalg.inv(lower)[np.ix_(inv, inv)]
        # Alg. 3.1 with w = 0, stages N, P, R: the operator on g
        X1 = PiN @ BN @ PiN.T
        X2 = X1 + PiP @ BP @ PiP.T @ (I - Ah @ X1)
        Bg = X2 + R @ (I - Ah @ X2)
        # eq. MSP: I - B A = (I - R A)(I - Pi_P B_P Pi_P^T A)(I - Pi_N B_N Pi_N^T A)
        np.testing.assert_allclose(I - Bg @ Ah, (I - R @ Ah) @ (I - PiP @ BP @ PiP.T @ Ah)
                                   @ (I - X1 @ Ah), atol=1e-10)
    else:
        # Alg. 3.1 with w = 0, stages P then R: the operator on g
        Bg = PiP @ BP @ PiP.T + R @ (I - Ah @ PiP @ BP @ PiP.T)
        # eq. MSP: I - B A = (I - R A)(I - Pi_P B_P Pi_P^T A)
        np.testing.assert_allclose(I - Bg @ Ah, (I - R @ Ah) @ (I - PiP @ BP @ PiP.T @ Ah),
                                   atol=1e-10)
    Bor = _dense_operator(s.apply, N)
    np.testing.assert_allclose(Bor, Bg @ W, rtol=1e-9, atol=1e-11)
    if max_coarse >= n:
        # single level: B_P is the exact inverse of the pressure block
        np.testing.assert_allclose(BP @ (PiP.T @ Ah @ PiP), np.eye(n), atol=1e-11)


# --------------------------------------------------------------------------
# O10 V-cycle -- pin P6
# --------------------------------------------------------------------------
def _vcycle_dense(levels, l, coarse_inv, smoother=0, w=1.0, nu_pre=1, nu_post=1):
    """Textbook V-cycle operator: every smoothing sweep is the stationary step
    x <- x + S (f - A x) with S = (D + L_pi)^-1 / (D + U_pi)^-1 (Gauss-Seidel
    on the color-permuted matrix, forward / backward) or S = w D^-1 (Jacobi);
    nu_pre sweeps from x = 0, coarse correction, nu_post sweeps."""
    L = levels[l]
    n = L["n"]
    A = dense_from_csr(L["row_ptr"], L["col_ind"], L["val"])
    if L["color"] is None:
        return coarse_inv
    if smoother == 0:
        perm = np.argsort(L["color"], kind="stable")
        inv = np.argsort(perm)
        Ap = A[np.ix_(perm, perm)]
        # M^{-1} in natural numbering
        Sf = np.linalg.inv(np.tril(Ap))[np.ix_(inv, inv)]
        Sb = np.linalg.inv(np.triu(Ap))[np.ix_(inv, inv)]
    elif smoother == 2:
        Sf = np.linalg.inv(np.tril(A))
        Sb = np.linalg.inv(np.triu(A))
    else:
        Sf = Sb = w * np.diag(1.0 / np.diag(A))
    P = np.zeros((n, L["nc"]))
    P[np.arange(n), L["agg"]] = 1.0
    Bc = _vcycle_dense(levels, l + 1, coarse_inv, smoother, w, nu_pre, nu_post)
    I = np.eye(n)
    X = np.zeros((n, n))
    for _ in range(nu_pre):
        X = X + Sf @ (I - A @ X)
    X = X + P @ Bc @ P.T @ (I - A @ X)
    for _ in range(nu_post):
        X = X + Sb @ (I - A @ X)
    return X


@pytest.mark.parametrize("shape,max_coarse", [((64,), 20), ((64,), 4), ((8, 8, 8), 40), ((6, 6, 6), 10)])
def test_vcycle_is_textbook_multigrid(shape, max_coarse):
    rp, ci, val = synth.poisson_csr(shape)
    n = len(rp) - 1
    s = O.OracleSolver(max_coarse=max_coarse)
    s.setup(n=n, b=1, p=0, row_ptr=rp, col_ind=ci, vals=bsr_b1(rp, ci, val))
    levels = [s.level(l) for l in range(s.nlevels)]
    assert s.nlevels >= 2
    Lc = levels[-1]
    coarse_inv = np.linalg.inv(dense_from_csr(Lc["row_ptr"], Lc["col_ind"], Lc["val"]))
    Bd = _vcycle_dense(levels, 0, coarse_inv)
    Bo = _dense_operator(s.vcycle, n)
    np.testing.assert_allclose(Bo, Bd, rtol=1e-10, atol=1e-12)
    A0 = dense_from_csr(levels[0]["row_ptr"], levels[0]["col_ind"], levels[0]["val"])
    E = np.eye(n) - Bo @ A0
    rho = max(abs(np.linalg.eigvals(E)))
    assert rho < 1.0
    # the stationary iteration x <- x + V(f - A x) contracts at rate rho
    rng = np.random.default_rng(1)
    e = rng.uniform(-1, 1, n)
    for _ in range(60):
        e = E @ e
    e2 = E @ e
    rate = np.linalg.norm(e2) / np.linalg.norm(e)
    assert rate <= rho * 1.05 + 1e-12


@pytest.mark.parametrize("shape,max_coarse", [((64,), 4), ((6, 6, 6), 10)])
@pytest.mark.parametrize("smoother,w,nu_pre,nu_post", [
    (0, 1.0, 2, 1), (0, 1.0, 0, 2), (0, 1.0, 2, 2),
    (1, 2.0 / 3.0, 1, 1), (1, 2.0 / 3.0, 2, 2), (1, 1.0, 1, 1), (1, 0.8, 0, 3),
    (2, 1.0, 1, 1)])
def test_vcycle_smoothers_and_sweeps_are_textbook(shape, max_coarse, smoother, w, nu_pre,
                                                  nu_post):
    rp, ci, val = synth.poisson_csr(shape)
    n = len(rp) - 1
    s = O.OracleSolver(max_coarse=max_coarse, smoother=smoother, jacobi_weight=w,
                       nu_pre=nu_pre, nu_post=nu_post)
    s.setup(n=n, b=1, p=0, row_ptr=rp, col_ind=ci, vals=bsr_b1(rp, ci, val))
    levels = [s.level(l) for l in range(s.nlevels)]
    assert s.nlevels >= 2
    Lc = levels[-1]
    coarse_inv = np.linalg.inv(dense_from_csr(Lc["row_ptr"], Lc["col_ind"], Lc["val"]))
    Bd = _vcycle_dense(levels, 0, coarse_inv, smoother, w, nu_pre, nu_post)
    Bo = _dense_operator(s.vcycle, n)
    np.testing.assert_allclose(Bo, Bd, rtol=1e-10, atol=1e-12)
    if smoother == 1 and w <= 2.0 / 3.0 + 1e-12 and nu_pre + nu_post >= 2:
        # damped Jacobi on Poisson smooths every mode: the V-cycle contracts
        A0 = dense_from_csr(levels[0]["row_ptr"], levels[0]["col_ind"], levels[0]["val"])
        assert max(abs(np.linalg.eigvals(np.eye(n) - Bo @ A0))) < 1.0


def _diag_dominant(n, seed, density=0.05):
    rp, ci = random_pattern(n, density, seed, symmetric=False)
    rng = np.random.default_rng(seed + 1)
    val = rng.uniform(-1.0, 1.0, len(ci))
    rows = np.repeat(np.arange(n), np.diff(rp))
    d = rows == ci
    rowsum = np.zeros(n)
    np.add.at(rowsum, rows[~d], np.abs(val[~d]))
    val[d] = (1.5 + rng.random(n)) * (rowsum + 1.0)
    return rp, ci, val


@pytest.mark.parametrize("seed", range(3))
def test_jacobi_sweep_reads_only_the_old_iterate(seed):
    """Every row of a Jacobi sweep equals that row swept alone against the old
    iterate (bit for bit): a sweep that read values updated earlier in the
    same sweep (Gauss-Seidel-like) would differ."""
    n = 120
    rp, ci, val = _diag_dominant(n, seed)
    rng = np.random.default_rng(seed + 7)
    f = rng.uniform(-1, 1, n)
    x = rng.uniform(-1, 1, n)
    y = O.jacobi_sweep(rp, ci, val, 0.7, f, x)
    assert not np.array_equal(y, x)
    for i in range(n):
        cols = ci[rp[i]:rp[i + 1]]
        k = len(cols)
        di = int(np.nonzero(cols == i)[0][0])
        # local system: row di is row i (same stored order); the others are
        # unit rows that keep their old value
        rows = [np.arange(k, dtype=np.int32) if r == di else np.array([r], dtype=np.int32)
                for r in range(k)]
        prl = np.zeros(k + 1, dtype=np.int32)
        prl[1:] = np.cumsum([len(rr) for rr in rows])
        cil = np.concatenate(rows).astype(np.int32)
        vall = np.concatenate([val[rp[i]:rp[i + 1]] if r == di else np.array([1.0])
                               for r in range(k)])
        fl = x[cols].copy()
        fl[di] = f[i]
        yl = O.jacobi_sweep(prl, cil, vall, 0.7, fl, x[cols])
        assert yl[di] == y[i]


@pytest.mark.parametrize("b,p", [(3, 0), (4, 2), (7, 6)])
def test_n_stage_blocks_are_decoupled_concentration_blocks(b, p):
    """Dn = rows N of D_c^-1 and Ann = (D_c^-1 A_cd)[N, N] against numpy
    inverses, N = all unknowns but p, ascending."""
    n = 30
    rp, ci, vals = synth.random_bsr(n, b, 0.1, 40 + b)
    s = O.OracleSolver(max_coarse=10000, n_stage=1)
    s.setup(n=n, b=b, p=p, row_ptr=rp, col_ind=ci, vals=vals)
    Dn, Ann = s.nstage()
    N = [k for k in range(b) if k != p]
    for c in range(n):
        kd = rp[c] + int(np.nonzero(ci[rp[c]:rp[c + 1]] == c)[0][0])
        Di = np.linalg.inv(vals[kd])
        np.testing.assert_allclose(Dn[c], Di[N, :], rtol=1e-12, atol=1e-14)
        for q in range(rp[c], rp[c + 1]):
            ref = np.eye(b - 1) if ci[q] == c else (Di @ vals[q])[np.ix_(N, N)]
            np.testing.assert_allclose(Ann[q], ref, rtol=1e-11, atol=1e-13)


def test_jacobi_fixed_point_is_the_solution():
    n = 200
    rp, ci, val = _diag_dominant(n, 5)
    A = dense_from_csr(rp, ci, val)
    f = np.random.default_rng(6).uniform(-1, 1, n)
    x = np.zeros(n)
    for _ in range(400):
        x = O.jacobi_sweep(rp, ci, val, 1.0, f, x)
    np.testing.assert_allclose(x, np.linalg.solve(A, f), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("b", [1, 3, 7])
def test_block_jacobi_r_stage_is_blockwise_solve(b):
    n = 60
    rp, ci, vals = synth.random_bsr(n, b, 0.05, 21 + b)
    s = O.OracleSolver(max_coarse=10000, full_smoother=1)
    s.setup(n=n, b=b, p=0, row_ptr=rp, col_ind=ci, vals=vals)
    r = np.random.default_rng(3).uniform(-1, 1, n * b)
    z = s.bilu_apply(r)
    diag = [int(np.nonzero(ci[rp[c]:rp[c + 1]] == c)[0][0]) + rp[c] for c in range(n)]
    ref = np.concatenate([np.linalg.solve(vals[diag[c]], r[c * b:(c + 1) * b]) for c in range(n)])
    np.testing.assert_allclose(z, ref, rtol=1e-12, atol=1e-14)


def test_block_jacobi_exact_on_uncoupled_cells():
    """No couplings between cells: block Jacobi is the exact inverse, so the
    whole preconditioner is exact and FGMRES takes one iteration (cf. P8)."""
    n, b = 40, 4
    rp, ci, vals = synth.random_bsr(n, b, 0.0, 5)
    s = O.OracleSolver(max_coarse=8, full_smoother=1)
    s.setup(n=n, b=b, p=0, row_ptr=rp, col_ind=ci, vals=vals)
    rhs = np.random.default_rng(2).uniform(-1, 1, n * b)
    x, it, rr, st = s.solve(rhs, 1e-10)
    assert st == 0 and it == 1 and rr <= 1e-12


# --------------------------------------------------------------------------
# O8 coarse direct solve -- pin P11 (exact rational arithmetic)
# --------------------------------------------------------------------------
def _exact_solve(A, f):
    n = len(A)
    M = [[Fraction(int(A[i][j])) for j in range(n)] + [Fraction(int(f[i]))] for i in range(n)]
    for k in range(n):
        piv = next(r for r in range(k, n) if M[r][k] != 0)
        M[k], M[piv] = M[piv], M[k]
        for r in range(n):
            if r != k and M[r][k] != 0:
                fac = M[r][k] / M[k][k]
                M[r] = [a - fac * b for a, b in zip(M[r], M[k])]
    return [float(M[i][n] / M[i][i]) for i in range(n)]


@pytest.mark.parametrize("seed", range(5))
def test_coarse_lu_solve_exact(seed):
    rng = np.random.default_rng(seed)
    n = 7
    A = rng.integers(-9, 10, size=(n, n)).astype(float)
    A[0, 0] = 0.0  # forces a row interchange
    while abs(np.linalg.det(A)) < 1:
        A = rng.integers(-9, 10, size=(n, n)).astype(float)
    f = rng.integers(-9, 10, size=n).astype(float)
    lu, piv = O.lu_factor(A)
    x = O.lu_solve(lu, piv, f)
    np.testing.assert_allclose(x, _exact_solve(A, f), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("n,seed", [(130, 0), (517, 1), (1200, 2)])
def test_coarse_lu_solve_interchanges_at_coarse_sizes(n, seed):
    """Partial pivoting at coarse-level sizes: A = P T with T well conditioned
    and a small diagonal, and P a random row permutation, so nearly every
    elimination step interchanges rows.  The solve must give back a known
    x to within cond(A) eps (cond from the SVD) and a componentwise backward
    error of a few n eps; applying an interchange to the wrong row, in the
    wrong order or to the right-hand side twice gives O(1) errors."""
    rng = np.random.default_rng(seed)
    T = rng.uniform(-1.0, 1.0, size=(n, n)) / np.sqrt(n)
    T[np.arange(n), np.arange(n)] = 1e-3 * rng.uniform(0.5, 1.0, n)
    T += np.tril(rng.uniform(-1.0, 1.0, size=(n, n)), -1)
    A = T[rng.permutation(n)]
    x_true = rng.integers(-5, 6, size=n).astype(float)
    f = A @ x_true
    lu, piv = O.lu_factor(A)
    assert np.count_nonzero(piv != np.arange(n)) > n // 2
    x = O.lu_solve(lu, piv, f)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(x - x_true) / np.linalg.norm(x_true) <= 50 * kappa * np.finfo(float).eps
    berr = np.max(np.abs(f - A @ x) / (np.abs(A) @ np.abs(x) + np.abs(f)))
    assert berr <= 8 * n * np.finfo(float).eps


# --------------------------------------------------------------------------
# O11 FGMRES -- pins P12, P13
# --------------------------------------------------------------------------
@pytest.mark.parametrize("max_coarse", [10000, 64])
def test_fgmres_matches_dense_solve(max_coarse):
    sys = synth.config(0)
    s = O.OracleSolver(max_coarse=max_coarse)
    s.setup(sys)
    x, it, rr, st = s.solve(sys.rhs, 1e-6)
    A = sys.to_dense()
    xd = np.linalg.solve(A, sys.rhs)
    kappa = np.linalg.cond(A)
    assert st == 0 and 1 <= it <= 30
    true_rr = np.linalg.norm(sys.rhs - A @ x) / np.linalg.norm(sys.rhs)
    assert true_rr <= 1e-6 and abs(true_rr - rr) <= 1e-12
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= kappa * 1e-6


def test_exact_pressure_stage_one_iteration():
    """b = 1 and a single AMG level: the pressure stage is an exact solve and
    FGMRES stops after one iteration."""
    rp, ci, val = synth.poisson_csr((9, 7, 5))
    n = len(rp) - 1
    rhs = np.random.default_rng(2).uniform(-1, 1, n)
    s = O.OracleSolver(max_coarse=10000)
    s.setup(n=n, b=1, p=0, row_ptr=rp, col_ind=ci, vals=bsr_b1(rp, ci, val))
    x, it, rr, st = s.solve(rhs, 1e-10)
    assert it == 1 and rr < 1e-10


def test_zero_rhs_gives_zero_solution_without_iterations():
    sys = synth.config(0)
    s = O.OracleSolver()
    s.setup(sys)
    x, it, rr, st = s.solve(np.zeros(sys.N), 1e-6, x0=np.ones(sys.N))
    assert it == 0 and np.count_nonzero(x) == 0


def test_max_iter_reports_not_converged():
    sys = synth.config(0)
    s = O.OracleSolver(max_iter=2, max_coarse=64)
    s.setup(sys)
    x, it, rr, st = s.solve(sys.rhs, 1e-14)
    assert st == 1 and it == 2 and rr > 1e-14


def test_fp32_preconditioner_converges_like_fp64():
    sys = synth.config(0)
    r64 = O.OracleSolver(max_coarse=64)
    r64.setup(sys)
    x64, it64, rr64, _ = r64.solve(sys.rhs, 1e-6)
    r32 = O.OracleSolver(max_coarse=64, precond_fp32=True)
    r32.setup(sys)
    x32, it32, rr32, _ = r32.solve(sys.rhs, 1e-6)
    assert abs(it32 - it64) <= 1 and rr32 <= 1e-6
    v = np.random.default_rng(0).uniform(-1, 1, sys.N)
    z64, z32 = r64.apply(v), r32.apply(v)
    rel = np.linalg.norm(z64 - z32) / np.linalg.norm(z64)
    assert 1e-9 < rel < 1e-4  # FP32 rounding, not a different operator


# --------------------------------------------------------------------------
# O12 adaptive SETUP -- pin P14 (Sec. 3.2; mu = 0 is standard MSP)
# --------------------------------------------------------------------------
def _newton_sequence(sys, steps):
    out = [sys]
    for t in range(1, steps):
        out.append(synth.newton_step(sys, t, 77))
    return out


def test_adaptive_setup_rules():
    sys = synth.lognormal_grid(6, 6, 4, 3, 9, 1.0, 1.0, "corners2")
    seq = _newton_sequence(sys, 4)
    # mu = 0: every system regenerates the preconditioner (SetupCalls = NumNSteps)
    s0 = O.OracleSolver(mu=0, max_coarse=16)
    its = []
    for t, A in enumerate(seq):
        assert s0.setup(A) is True
        its.append(s0.solve(A.rhs, 1e-6)[1])
    assert s0.setup_calls == len(seq)
    # large mu: only the first system builds B; the others reuse it
    sb = O.OracleSolver(mu=1000, max_coarse=16)
    flags = []
    for A in seq:
        flags.append(sb.setup(A))
        x, it, rr, st = sb.solve(A.rhs, 1e-6)
        assert rr <= 1e-6
    assert flags == [True, False, False, False] and sb.setup_calls == 1
    # mu = It - 1 forces a rebuild, mu = It reuses
    it0 = its[0]
    for mu, expect in [(it0 - 1, True), (it0, False)]:
        s = O.OracleSolver(mu=mu, max_coarse=16)
        s.setup(seq[0])
        assert s.solve(seq[0].rhs, 1e-6)[1] == it0
        assert s.setup(seq[1]) is expect
    # a size change always regenerates (the remark of Sec. 3.2)
    s = O.OracleSolver(mu=1000, max_coarse=16)
    s.setup(seq[0])
    s.solve(seq[0].rhs, 1e-6)
    other = synth.lognormal_grid(5, 6, 4, 3, 9, 1.0, 1.0, "corners2")
    assert s.setup(other) is True and s.setup_calls == 2


def test_reuse_uses_current_matrix_for_krylov():
    """On reuse the old B is applied but the residual is that of the new A."""
    sys = synth.lognormal_grid(6, 5, 4, 3, 4, 1.0, 1.0, "corners2")
    nxt = synth.newton_step(sys, 1, 5)
    s = O.OracleSolver(mu=1000, max_coarse=16)
    s.setup(sys)
    s.solve(sys.rhs, 1e-6)
    assert s.setup(nxt) is False
    x, it, rr, st = s.solve(nxt.rhs, 1e-8)
    A = nxt.to_dense()
    assert np.linalg.norm(nxt.rhs - A @ x) / np.linalg.norm(nxt.rhs) <= 1e-8


# --------------------------------------------------------------------------
# O1 validation
# --------------------------------------------------------------------------
def test_validation_errors():
    sys = synth.config(0)
    n, b, p = sys.n, sys.b, sys.p
    rp, ci, v = sys.row_ptr, sys.col_ind, sys.vals
    assert O.validate(n, b, p, rp, ci, v) == 0
    assert O.validate(n, b, b, rp, ci, v) == -1
    assert O.validate(n, 0, 0, rp, ci, v) == -1
    bad = ci.copy()
    bad[1], bad[2] = bad[2], bad[1]
    assert O.validate(n, b, p, rp, bad, v) == -2
    bad = ci.copy()
    bad[0] = n
    assert O.validate(n, b, p, rp, bad, v) == -2
    vv = v.copy()
    vv[5, 1, 2] = np.nan
    assert O.validate(n, b, p, rp, ci, vv) == -4
    # a block row without its diagonal block
    rp2 = np.array([0, 1, 2], dtype=np.int32)
    ci2 = np.array([1, 0], dtype=np.int32)
    assert O.validate(2, 1, 0, rp2, ci2, np.ones((2, 1, 1))) == -2


@pytest.mark.parametrize("b", [1, 3])
def test_bilu0_multicolor_order_defining_property(b):
    """Block ILU(0) in the multi-color elimination order is ILU(0) of the
    symmetrically permuted matrix: (L U)_ij = (P A P^T)_ij on its pattern."""
    sys = synth.lognormal_grid(6, 5, 4, b, 31, 1.0, 1.0, "corners2")
    n = sys.n
    order = O.multicolor_order(sys.row_ptr, sys.col_ind)
    col, g = O.color(sys.row_ptr, sys.col_ind)
    assert g == 2 and np.all(np.diff(col[order]) >= 0)
    F, D = O.bilu0_factor(n, b, sys.row_ptr, sys.col_ind, sys.vals, order=order)
    pos = np.argsort(order)
    L = np.eye(n * b)
    U = np.zeros((n * b, n * b))
    for i in range(n):
        for k in range(sys.row_ptr[i], sys.row_ptr[i + 1]):
            j = sys.col_ind[k]
            pi, pj = pos[i], pos[j]
            blk = (slice(pi * b, (pi + 1) * b), slice(pj * b, (pj + 1) * b))
            if pj < pi:
                L[blk] = F[k]
            elif pj > pi:
                U[blk] = F[k]
        U[pos[i] * b:(pos[i] + 1) * b, pos[i] * b:(pos[i] + 1) * b] = np.linalg.inv(D[i])
    perm = (order[:, None] * b + np.arange(b)[None, :]).reshape(-1)
    PAPt = sys.to_dense()[np.ix_(perm, perm)]
    LU = L @ U
    for i in range(n):
        for k in range(sys.row_ptr[i], sys.row_ptr[i + 1]):
            pi, pj = pos[i], pos[sys.col_ind[k]]
            blk = (slice(pi * b, (pi + 1) * b), slice(pj * b, (pj + 1) * b))
            np.testing.assert_allclose(LU[blk], PAPt[blk], rtol=1e-11, atol=1e-11)
    r = np.random.default_rng(1).uniform(-1, 1, n * b)
    z = O.bilu0_solve(n, b, sys.row_ptr, sys.col_ind, F, D, r, order=order)
    np.testing.assert_allclose(LU @ z[perm], r[perm], rtol=1e-10, atol=1e-12)
