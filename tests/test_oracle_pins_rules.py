"""Pins of three oracle functions that invariants alone do not fix: the
pairwise matching pass of the aggregation (Sec. 5, NPAIR in the builder's
concrete reading: strength s_ij = -(a_ij + a_ji)/2, strong threshold 0.25 of
the row maximum, ascending visit, strongest free eligible partner, lowest
index on ties), the absorption of singletons on a stalled level, and the FP32
preconditioner apply (FP64 setup rounded to FP32, FP32 arithmetic in the
V-cycle, the pressure-column residual and the block ILU(0) solve).

Each oracle result is compared bit for bit with something written here from
the rule itself: an optimality certificate that any correct matching must
satisfy, a set-based transcription of the rule, and a step-by-step
numpy.float32 evaluation of the apply.  The inputs force ties (strengths
drawn from a few integers) so that a wrong tie-break shows.  CPU only.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import oracle as O
from paper_2208_08594_amd import synth


# --------------------------------------------------------------------------
# inputs: scalar CSR matrices with many equal strengths
# --------------------------------------------------------------------------
def tie_matrix(n, density, seed, symmetric_pattern, symmetric_values):
    """Random scalar matrix whose off-diagonal values come from
    {-4,-2,-1,-1/2,0,+1}: many strengths tie, some rows have only zero stored
    off-diagonals (ineligible, like Dirichlet well rows), some couple only
    positively (no positive strength)."""
    rng = np.random.default_rng(seed)
    P = rng.random((n, n)) < density
    if symmetric_pattern:
        P = P | P.T
    np.fill_diagonal(P, False)
    V = rng.choice([-4.0, -2.0, -1.0, -1.0, -0.5, -0.5, 0.0, 1.0], size=(n, n))
    if symmetric_values:
        V = np.triu(V) + np.triu(V, 1).T
    V = np.where(P, V, 0.0)
    zero_rows = rng.choice(n, size=max(1, n // 12), replace=False)
    for i in zero_rows:  # stored zeros only
        V[i, P[i]] = 0.0
    pos_rows = rng.choice(n, size=max(1, n // 15), replace=False)
    for i in pos_rows:
        V[i, P[i]] = 1.0
    np.fill_diagonal(P, True)
    np.fill_diagonal(V, 10.0)
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum(P.sum(1))
    ci = np.nonzero(P)[1].astype(np.int32)
    val = V[P]
    return rp, ci, val


def neighbours(rp, ci):
    n = len(rp) - 1
    S = [set() for _ in range(n)]
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            j = int(ci[k])
            if j != i:
                S[i].add(j)
                S[j].add(i)
    return [sorted(s) for s in S]


def entry(rp, ci, val, i, j):
    for k in range(rp[i], rp[i + 1]):
        if ci[k] == j:
            return float(val[k])
    return 0.0


def strengths(rp, ci, val):
    """s[i][j] for j in S_i, the row maxima and eligibility of the pairwise
    rule: a row is eligible when it stores a nonzero off-diagonal value and
    its largest strength is positive."""
    n = len(rp) - 1
    S = neighbours(rp, ci)
    s = [{j: -(entry(rp, ci, val, i, j) + entry(rp, ci, val, j, i)) / 2.0 for j in S[i]}
         for i in range(n)]
    smax = [max(s[i].values()) if s[i] else 0.0 for i in range(n)]
    offnz = [any(ci[k] != i and val[k] != 0.0 for k in range(rp[i], rp[i + 1]))
             for i in range(n)]
    elig = [offnz[i] and bool(s[i]) and smax[i] > 0.0 for i in range(n)]
    return S, s, smax, elig


# --------------------------------------------------------------------------
# pairwise pass
# --------------------------------------------------------------------------
def check_matching_certificate(rp, ci, val, agg, nc):
    """What every result of the rule satisfies, stated without running it:
    aggregates of one or two rows numbered by their lowest row; a pair is a
    strong coupling between eligible rows; its lower row i preferred its
    partner j over every other eligible strong neighbour k that was still free
    when i was visited (k's aggregate starts at a row >= i): s_ik < s_ij, or
    s_ik == s_ij and k > j; an eligible row left alone had no such free
    neighbour at all."""
    n = len(rp) - 1
    S, s, smax, elig = strengths(rp, ci, val)
    members = [[] for _ in range(nc)]
    for i in range(n):
        members[int(agg[i])].append(i)
    assert all(1 <= len(m) <= 2 for m in members)
    leaders = [m[0] for m in members]
    assert leaders == sorted(leaders), "aggregates are numbered in order of creation"
    lead = [leaders[int(agg[i])] for i in range(n)]
    for a, m in enumerate(members):
        i = m[0]
        free = [k for k in S[i] if elig[k] and lead[k] >= i and k != i
                and s[i][k] >= 0.25 * smax[i]]
        if len(m) == 2:
            j = m[1]
            assert elig[i] and elig[j], "only eligible rows pair"
            assert j in s[i] and s[i][j] >= 0.25 * smax[i] and s[i][j] > 0
            for k in free:
                if k != j:
                    assert s[i][k] < s[i][j] or (s[i][k] == s[i][j] and k > j), \
                        f"row {i} took {j} (s={s[i][j]}) over {k} (s={s[i][k]})"
        else:
            assert not (elig[i] and free), f"row {i} stayed alone with free partners {free}"


def literal_pairwise(rp, ci, val):
    """The rule with Python sets: visit rows in ascending order; an unplaced
    row takes, among its unplaced eligible neighbours with strength at least a
    quarter of its largest, the strongest (lowest index among equals)."""
    n = len(rp) - 1
    S, s, smax, elig = strengths(rp, ci, val)
    unplaced = set(range(n))
    agg = [-1] * n
    nc = 0
    for i in range(n):
        if i not in unplaced:
            continue
        unplaced.discard(i)
        cand = {j for j in S[i] if j in unplaced and elig[j] and s[i][j] >= 0.25 * smax[i]} \
            if elig[i] else set()
        agg[i] = nc
        if cand:
            j = min(cand, key=lambda j: (-s[i][j], j))
            agg[j] = nc
            unplaced.discard(j)
        nc += 1
    return np.array(agg, dtype=np.int32), nc


CASES = [(n, d, seed, sp, sv) for seed in range(4) for (n, d) in [(40, 0.12), (90, 0.05)]
         for (sp, sv) in [(True, True), (True, False), (False, False)]]


@pytest.mark.parametrize("n,density,seed,sym_pattern,sym_values", CASES)
def test_npair_pass_is_the_rule(n, density, seed, sym_pattern, sym_values):
    rp, ci, val = tie_matrix(n, density, seed, sym_pattern, sym_values)
    agg, nc = O.npair_pass(rp, ci, val)
    check_matching_certificate(rp, ci, val, agg, nc)
    lagg, lnc = literal_pairwise(rp, ci, val)
    assert nc == lnc and np.array_equal(agg, lagg)


def test_npair_certificate_catches_the_plausible_mistakes():
    """The certificate rejects matchings made with the first free neighbour
    instead of the strongest, with the highest index on ties, or with a
    partner below the threshold: a pin that accepts these would not fix the
    rule."""
    rp, ci, val = tie_matrix(90, 0.05, 1, True, False)
    S, s, smax, elig = strengths(rp, ci, val)
    n = len(rp) - 1

    def variant(pick, beta=0.25):
        unplaced, agg, nc = set(range(n)), [-1] * n, 0
        for i in range(n):
            if i not in unplaced:
                continue
            unplaced.discard(i)
            cand = [j for j in S[i] if j in unplaced and elig[j] and s[i][j] >= beta * smax[i]] \
                if elig[i] else []
            agg[i] = nc
            if cand:
                j = pick(i, cand)
                agg[j] = nc
                unplaced.discard(j)
            nc += 1
        return np.array(agg), nc

    first = variant(lambda i, c: min(c))
    high_tie = variant(lambda i, c: min(c, key=lambda j: (-s[i][j], -j)))
    beta_half = variant(lambda i, c: min(c, key=lambda j: (-s[i][j], j)), beta=0.5)
    for wrong in (first, high_tie, beta_half):
        with pytest.raises(AssertionError):
            check_matching_certificate(rp, ci, val, *wrong)


# --------------------------------------------------------------------------
# absorption of singletons on a stalled level
# --------------------------------------------------------------------------
def literal_absorb(rp, ci, val, agg, nc):
    """Every eligible row alone in its aggregate moves to the aggregate of its
    strongest neighbour j (lowest j among equals) that lies in an aggregate of
    two or more rows, sizes counted before any move, provided s_ij is at least
    a quarter of the row's largest strength; then empty aggregates are dropped
    and the others keep their order."""
    n = len(rp) - 1
    S, s, smax, elig = strengths(rp, ci, val)
    size = np.bincount(agg, minlength=nc)
    target = [int(a) for a in agg]
    for i in range(n):
        if size[agg[i]] != 1 or not elig[i]:
            continue
        cand = [j for j in S[i] if size[agg[j]] >= 2 and s[i][j] >= 0.25 * smax[i]]
        if cand:
            target[i] = int(agg[min(cand, key=lambda j: (-s[i][j], j))])
    alive = sorted(set(target))
    renum = {a: k for k, a in enumerate(alive)}
    return np.array([renum[t] for t in target], dtype=np.int32), len(alive)


def random_grouping(n, seed):
    """An aggregate map with sizes 1..4 (many singletons), numbered in order
    of first member, as the two pairwise passes produce."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    agg = np.empty(n, dtype=np.int32)
    pos, k = 0, 0
    while pos < n:
        sz = int(rng.choice([1, 1, 1, 2, 3, 4]))
        agg[perm[pos:pos + sz]] = k
        pos += sz
        k += 1
    first = {}
    for i in range(n):
        first.setdefault(int(agg[i]), i)
    order = sorted(first, key=first.get)
    ren = {a: r for r, a in enumerate(order)}
    return np.array([ren[int(a)] for a in agg], dtype=np.int32), k


@pytest.mark.parametrize("n,density,seed,sym_pattern,sym_values", CASES)
def test_absorb_singletons_is_the_rule(n, density, seed, sym_pattern, sym_values):
    rp, ci, val = tie_matrix(n, density, seed, sym_pattern, sym_values)
    agg0, nc0 = random_grouping(n, seed + 100)
    agg, nc = O.absorb_singletons(rp, ci, val, agg0, nc0)
    lagg, lnc = literal_absorb(rp, ci, val, agg0, nc0)
    assert nc == lnc and np.array_equal(agg, lagg)
    # what any correct absorption satisfies: rows in aggregates of two or
    # more, and ineligible rows, keep their aggregate mates; a moved row is
    # coupled strongly to its new aggregate
    S, s, smax, elig = strengths(rp, ci, val)
    size0 = np.bincount(agg0, minlength=nc0)
    for i in range(n):
        same0 = set(np.nonzero(agg0 == agg0[i])[0])
        if size0[agg0[i]] >= 2 or not elig[i]:
            assert same0 <= set(np.nonzero(agg == agg[i])[0])
        mates = set(np.nonzero(agg == agg[i])[0]) - {i}
        if size0[agg0[i]] == 1 and mates:
            assert any(j in s[i] and s[i][j] >= 0.25 * smax[i] and s[i][j] > 0 for j in mates)


def test_absorb_rule_rejects_the_plausible_mistakes():
    """Variants of the rule that the bit-for-bit comparison must tell apart
    from the oracle on these inputs: highest index on ties, sizes counted after
    moves (singletons joining singletons that already moved), and the
    threshold dropped."""
    hits = {"high_tie": 0, "no_threshold": 0}
    for seed in range(4):
        rp, ci, val = tie_matrix(90, 0.05, seed, True, False)
        n = len(rp) - 1
        S, s, smax, elig = strengths(rp, ci, val)
        agg0, nc0 = random_grouping(n, seed + 100)
        ref, _ = O.absorb_singletons(rp, ci, val, agg0, nc0)
        size = np.bincount(agg0, minlength=nc0)
        for name in hits:
            target = [int(a) for a in agg0]
            for i in range(n):
                if size[agg0[i]] != 1 or not elig[i]:
                    continue
                beta = 0.0 if name == "no_threshold" else 0.25
                cand = [j for j in S[i] if size[agg0[j]] >= 2 and s[i][j] >= beta * smax[i]]
                if cand:
                    key = (lambda j: (-s[i][j], -j)) if name == "high_tie" else \
                        (lambda j: (-s[i][j], j))
                    target[i] = int(agg0[min(cand, key=key)])
            alive = sorted(set(target))
            renum = {a: k for k, a in enumerate(alive)}
            wrong = np.array([renum[t] for t in target])
            hits[name] += int(not np.array_equal(wrong, ref))
    assert all(v > 0 for v in hits.values()), hits


# --------------------------------------------------------------------------
# FP32 preconditioner apply, step by step in numpy.float32
# --------------------------------------------------------------------------
f32 = np.float32


def f32_gs_row(rp, ci, val, i, f, x):
    s, d = f32(0), f32(0)
    for k in range(rp[i], rp[i + 1]):
        j = ci[k]
        if j == i:
            d = val[k]
        else:
            s = f32(s + f32(val[k] * x[j]))
    x[i] = f32(f32(f[i] - s) / d)


def f32_vcycle(levels, lu, piv, l, f):
    L = levels[l]
    n = L["n"]
    if l == len(levels) - 1:
        xd = lu_solve_f64(lu, piv, [float(v) for v in f])
        return np.array([f32(v) for v in xd], dtype=np.float32)
    rp, ci, val, col, g = L["row_ptr"], L["col_ind"], L["val32"], L["color"], L["ncolors"]
    x = np.zeros(n, dtype=np.float32)
    for c in range(1, g + 1):
        for i in range(n):
            if col[i] == c:
                f32_gs_row(rp, ci, val, i, f, x)
    r = np.zeros(n, dtype=np.float32)
    for i in range(n):
        s = f32(0)
        for k in range(rp[i], rp[i + 1]):
            s = f32(s + f32(val[k] * x[ci[k]]))
        r[i] = f32(f[i] - s)
    fc = np.zeros(L["nc"], dtype=np.float32)
    for i in range(n):
        fc[L["agg"][i]] = f32(fc[L["agg"][i]] + r[i])
    xc = f32_vcycle(levels, lu, piv, l + 1, fc)
    for i in range(n):
        x[i] = f32(x[i] + xc[L["agg"][i]])
    for c in range(g, 0, -1):
        for i in range(n):
            if col[i] == c:
                f32_gs_row(rp, ci, val, i, f, x)
    return x


def lu_solve_f64(lu, piv, f):
    """Row interchanges of getrf, then unit-lower and upper substitution, each
    sum in ascending column order (FP64)."""
    m = lu.shape[0]
    x = list(f)
    for i in range(m):
        j = int(piv[i])
        if j != i:
            x[i], x[j] = x[j], x[i]
    for i in range(m):
        acc = 0.0
        for j in range(i):
            acc = acc + float(lu[i, j]) * x[j]
        x[i] = x[i] - acc
    for i in range(m - 1, -1, -1):
        acc = 0.0
        for j in range(i + 1, m):
            acc = acc + float(lu[i, j]) * x[j]
        x[i] = (x[i] - acc) / float(lu[i, i])
    return x


def f32_bilu_solve(n, b, rp, ci, F, D, order, r):
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n)
    z = r.astype(np.float32).reshape(n, b).copy()
    for i in order:
        low = sorted((k for k in range(rp[i], rp[i + 1]) if pos[ci[k]] < pos[i]),
                     key=lambda k: pos[ci[k]])
        for kk in low:
            k = ci[kk]
            for a in range(b):
                acc = f32(0)
                for t in range(b):
                    acc = f32(acc + f32(F[kk, a, t] * z[k, t]))
                z[i, a] = f32(z[i, a] - acc)
    for i in order[::-1]:
        t_ = z[i].copy()
        up = sorted((k for k in range(rp[i], rp[i + 1]) if pos[ci[k]] > pos[i]),
                    key=lambda k: pos[ci[k]])
        for jj in up:
            j = ci[jj]
            for a in range(b):
                acc = f32(0)
                for t in range(b):
                    acc = f32(acc + f32(F[jj, a, t] * z[j, t]))
                t_[a] = f32(t_[a] - acc)
        for a in range(b):
            acc = f32(0)
            for t in range(b):
                acc = f32(acc + f32(D[i, a, t] * t_[t]))
            z[i, a] = acc
    return z.reshape(-1)


@pytest.mark.parametrize("bilu_order", [0, 1])
def test_fp32_apply_is_float32_arithmetic(bilu_order):
    """The oracle's FP32 apply equals, bit for bit, the same steps evaluated
    one operation at a time in numpy.float32 on the RNE-rounded FP64 setup:
    g_P in FP64 then rounded; the V-cycle (color sweeps, residual,
    restriction, prolongation) in FP32 with the coarsest solve in FP64; the
    pressure-column residual and the block ILU(0) solve in FP32;
    z = (double) zz + (double) e at the pressure entry.  Accumulating in FP64
    over FP32 storage, or storing truncated values, changes the bits."""
    sys_ = synth.lognormal_grid(6, 5, 4, 3, 7, 1.0, 0.5, "corners2")
    o = O.OracleSolver(max_coarse=12, precond_fp32=True, bilu_order=bilu_order)
    o.setup(sys_)
    assert o.nlevels >= 3
    n, b, p = sys_.n, sys_.b, sys_.p
    levels = []
    for l in range(o.nlevels):
        L = o.level(l)
        L["val32"] = L["val"].astype(np.float32)
        levels.append(L)
    Lc = levels[-1]
    m = Lc["n"]
    dense = np.zeros((m, m))
    for i in range(m):
        dense[i, Lc["col_ind"][Lc["row_ptr"][i]:Lc["row_ptr"][i + 1]]] = \
            Lc["val"][Lc["row_ptr"][i]:Lc["row_ptr"][i + 1]]
    lu, piv = scipy.linalg.lu_factor(dense)
    om = o.omega()
    F64, D64 = o.bilu()
    F, D = F64.astype(np.float32), D64.astype(np.float32)
    rp, ci = sys_.row_ptr, sys_.col_ind
    Apc = sys_.vals.reshape(-1, b, b)[:, :, p].astype(np.float32)  # column p of each block
    order = np.arange(n) if bilu_order == 0 else O.multicolor_order(rp, ci)

    for seed in range(2):
        v = np.random.default_rng(seed).uniform(-1, 1, n * b)
        gP = np.zeros(n, dtype=np.float32)
        for c in range(n):
            acc = 0.0
            for k in range(b):
                acc = acc + float(om[c, k]) * float(v[c * b + k])
            gP[c] = f32(acc)
        e = f32_vcycle(levels, lu, piv, 0, gP)
        r = np.zeros(n * b, dtype=np.float32)
        for c in range(n):
            for k in range(b):
                s = f32(0)
                for q in range(rp[c], rp[c + 1]):
                    s = f32(s + f32(Apc[q, k] * e[ci[q]]))
                r[c * b + k] = f32(f32(v[c * b + k]) - s)
        zz = f32_bilu_solve(n, b, rp, ci, F, D, order, r)
        add = np.zeros((n, b))
        add[:, p] = e.astype(np.float64)
        z = zz.astype(np.float64) + add.reshape(-1)
        zo = o.apply(v)
        assert np.array_equal(zo.view(np.int64), z.view(np.int64)), \
            np.max(np.abs(zo - z) / np.abs(z).max())
