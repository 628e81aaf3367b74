"""CPU checks of libmsp: the C-ABI loads and exports every declared symbol, the
ctypes structs match the C layout, host-only entry points behave, and the
library's host setup code (grouping, matching, Galerkin) agrees bit for bit
with the oracle.  No GPU work is launched here."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import scipy.sparse as sp
import pytest

from oracle import oracle as O
from paper_2208_08594_amd import msp, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INC = os.path.join(ROOT, "include")
CSRC = os.path.join(ROOT, "paper_2208_08594_amd", "csrc")


def header_functions():
    names = set()
    for h in ("msp.h", "msp_stages.h"):
        txt = open(os.path.join(INC, h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?(?:int|char\s*\*|const char \*)\s*\**\s*(msp_\w+)\s*\(",
                             txt, flags=re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    L = msp.lib()
    declared = header_functions()
    assert len(declared) >= 19
    assert declared == set(msp.SIGNATURES), declared ^ set(msp.SIGNATURES)
    for name in declared:
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", msp.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert declared <= exported


def test_struct_layout_matches_c():
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "msp.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(msp_options), offsetof(msp_options, stream),
         offsetof(msp_options, alloc_user), offsetof(msp_options, full_smoother),
         offsetof(msp_options, jacobi_weight), offsetof(msp_options, n_stage),
         offsetof(msp_options, host_chain), sizeof(msp_info),
         offsetof(msp_info, rel_true_residual), offsetof(msp_info, phase_ms));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        cpath = os.path.join(d, "t.c")
        open(cpath, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.check_call(["gcc", "-I", INC, cpath, "-o", exe])
        vals = list(map(int, subprocess.check_output([exe]).split()))
    got = [C.sizeof(msp.MspOptions), msp.MspOptions.stream.offset, msp.MspOptions.alloc_user.offset,
           msp.MspOptions.full_smoother.offset, msp.MspOptions.jacobi_weight.offset,
           msp.MspOptions.n_stage.offset, msp.MspOptions.host_chain.offset,
           C.sizeof(msp.MspInfo), msp.MspInfo.rel_true_residual.offset, msp.MspInfo.phase_ms.offset]
    assert vals == got


def test_status_strings_and_defaults():
    for code in list(msp.STATUS) + [12345]:
        assert isinstance(msp.status_string(code), str) and msp.status_string(code)
    opt = msp.MspOptions()
    assert msp.lib().msp_default_options(C.byref(opt)) == 0
    assert (opt.mu, opt.restart, opt.max_iter, opt.max_coarse, opt.precond_fp32) == (0, 30, 1000, 10000, 0)
    assert msp.lib().msp_default_options(None) == -1


def test_host_argument_errors_need_no_gpu():
    L = msp.lib()
    assert L.msp_create(None, None) == -1
    assert L.msp_destroy(None) == 0
    assert L.msp_setup(None, 1, 1, 0, None, None, None, 1) == -1
    assert L.msp_solve(None, None, None, 1e-6, None) == -1
    out = C.c_size_t()
    assert L.msp_footprint(0, 1, 4, None, C.byref(out)) == -1
    assert L.msp_footprint(10, 5, 4, None, C.byref(out)) == -1
    assert L.msp_footprint(10, 10, 9, None, C.byref(out)) == -1
    bad = msp.MspOptions()
    L.msp_default_options(C.byref(bad))
    bad.restart = 0
    h = C.c_void_p()
    assert L.msp_create(C.byref(h), C.byref(bad)) == -1


def test_footprint_scales_with_size():
    small = msp.footprint(1000, 6400, 4)
    big = msp.footprint(1048576, 7274496, 7)
    big32 = msp.footprint(1048576, 7274496, 7, precond_fp32=True)
    assert 0 < small < big and big32 < big
    # the dominant pieces are at least the matrix and the Krylov basis
    assert big > 7274496 * 49 * 8 + 61 * 7340032 * 8


def test_create_without_gpu_reports_no_device():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert msp.lib().msp_create(C.byref(h), None) == -7


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(msp, "_LIB", None)
    monkeypatch.setattr(msp, "LIB_PATH", "/nonexistent/libmsp.so")
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        msp.lib()


# --------------------------------------------------------------------------
# the library's host setup code against the oracle (bit for bit)
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def shim():
    d = tempfile.mkdtemp()
    so = os.path.join(d, "libshim.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared",
                           f"-I{CSRC}", os.path.join(ROOT, "tests", "native", "host_shim.cpp"),
                           os.path.join(CSRC, "msp_host.cpp"), "-o", so])
    L = C.CDLL(so)
    i32 = np.ctypeslib.ndpointer(np.int32, flags="C")
    f64 = np.ctypeslib.ndpointer(np.float64, flags="C")
    L.shim_color.argtypes = [C.c_int, i32, i32, i32]
    L.shim_color_sym.argtypes = [C.c_int, i32, i32, i32, i32]
    L.shim_hierarchy.argtypes = [C.c_int, i32, i32, f64, C.c_int, i32, i32, i32, i32, f64]
    L.shim_pair.argtypes = [C.c_int, i32, i32, f64, i32]
    L.shim_galerkin.argtypes = [C.c_int, i32, i32, f64, i32, C.c_int, i32, i32, f64]
    L.shim_galerkin.restype = C.c_longlong
    L.shim_pattern.argtypes = [C.c_int, i32, i32, C.c_longlong]
    L.shim_levels.argtypes = [C.c_int, i32, i32, C.c_int, i32]
    L.shim_levels_ord.argtypes = [C.c_int, i32, i32, i32, C.c_int, i32, i32]
    L.shim_levels_groups.argtypes = [C.c_int, i32, i32, i32, C.c_int, i32, C.c_int, i32, i32]
    return L


def _lib_color(shim, rp, ci):
    col = np.zeros(len(rp) - 1, dtype=np.int32)
    g = shim.shim_color(len(rp) - 1, rp, ci, col)
    return col, g


@pytest.mark.parametrize("seed", range(10))
def test_library_grouping_matches_oracle(shim, seed):
    rng = np.random.default_rng(seed)
    n = 50 + 30 * seed
    P = rng.random((n, n)) < 0.05
    np.fill_diagonal(P, True)
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum(P.sum(1))
    ci = np.nonzero(P)[1].astype(np.int32)
    c_lib, g_lib = _lib_color(shim, rp, ci)
    c_or, g_or = O.color(rp, ci)
    assert g_lib == g_or and np.array_equal(c_lib, c_or)


@pytest.mark.parametrize("n", [20000, 40000])
def test_library_grouping_large_symmetric_matches_oracle(shim, n):
    """Structurally symmetric patterns large enough for the row-chunked
    (threaded) adjacency build and symmetry test, with enough groups that
    vertices run out of undetermined neighbours while the groups are built."""
    rng = np.random.default_rng(n)
    rows = rng.integers(0, n, 5 * n)
    cols = (rows + rng.integers(1, 400, 5 * n)) % n
    i = np.concatenate([rows, cols, np.arange(n)])
    j = np.concatenate([cols, rows, np.arange(n)])
    key = np.unique(i.astype(np.int64) * n + j)
    r, c = key // n, key % n
    rp = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rp, r + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    ci = c.astype(np.int32)
    c_lib, g_lib = _lib_color(shim, rp, ci)
    c_or, g_or = O.color(rp, ci)
    assert g_lib > 4
    assert g_lib == g_or and np.array_equal(c_lib, c_or)


@pytest.mark.parametrize("case", ["long_coupling", "hub"])
def test_library_grouping_wide_graphs_match_oracle(shim, case):
    """Graphs the greedy cannot hold in 16-bit neighbour offsets or counts:
    one coupling 40,000 rows away in an otherwise local graph, and a vertex
    with more than 65,535 neighbours (a triangle keeps both off the bipartite
    closed form)."""
    if case == "long_coupling":
        n = 50000
        rng = np.random.default_rng(7)
        i = rng.integers(0, n - 300, 3 * n)
        j = i + rng.integers(1, 300, 3 * n)
        i = np.concatenate([i, [5, 5, 6]])
        j = np.concatenate([j, [40005, 6, 40005]])
    else:
        n = 70000
        i = np.concatenate([np.zeros(n - 1, dtype=np.int64), [1, 2]])
        j = np.concatenate([np.arange(1, n), [2, 3]])
        i = np.concatenate([i, [1]])
        j = np.concatenate([j, [3]])
    rp, ci = _pattern_from_edges(n, i, j)
    c_lib, g_lib = _lib_color(shim, rp, ci)
    c_or, g_or = O.color(rp, ci)
    assert g_lib == g_or and np.array_equal(c_lib, c_or)


def _pattern_from_edges(n, i, j, symmetric=True):
    """CSR pattern with a diagonal from an edge list (both directions if
    symmetric)."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    if symmetric:
        i, j = np.concatenate([i, j]), np.concatenate([j, i])
    key = np.unique(np.concatenate([i * n + j, np.arange(n) * (n + 1)]))
    r, c = key // n, key % n
    rp = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rp, r + 1, 1)
    return np.cumsum(rp).astype(np.int32), c.astype(np.int32)


def _symmetric_cases():
    """Structurally symmetric patterns with their diagonals: grids (bipartite
    7-point, 27-point), random local graphs, and graphs the 16-bit lists
    cannot hold (a long coupling, a row without its diagonal)."""
    cases = []
    rp, ci, _ = synth.poisson_csr((9, 7, 5))
    cases.append(("7-point", rp, ci))
    n3 = (6, 5, 4)
    idx = np.arange(np.prod(n3)).reshape(n3)
    i, j = [], []
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                a = idx[max(0, -dx):n3[0] - max(0, dx), max(0, -dy):n3[1] - max(0, dy),
                        max(0, -dz):n3[2] - max(0, dz)]
                b = idx[max(0, dx):n3[0] + min(0, dx), max(0, dy):n3[1] + min(0, dy),
                        max(0, dz):n3[2] + min(0, dz)]
                i.append(a.ravel())
                j.append(b.ravel())
    rp, ci = _pattern_from_edges(idx.size, np.concatenate(i), np.concatenate(j))
    cases.append(("27-point", rp, ci))
    for seed, n in [(3, 3000), (4, 50000)]:
        rng = np.random.default_rng(seed)
        a = rng.integers(0, n - 40, 4 * n)
        rp, ci = _pattern_from_edges(n, a, a + rng.integers(1, 40, 4 * n))
        cases.append((f"random local {n}", rp, ci))
    n = 50000
    rng = np.random.default_rng(5)
    a = rng.integers(0, n - 300, 3 * n)
    rp, ci = _pattern_from_edges(n, np.concatenate([a, [5, 5, 6]]),
                                 np.concatenate([a + rng.integers(1, 300, 3 * n), [40005, 6, 40005]]))
    cases.append(("long coupling", rp, ci))
    rp, ci = _pattern_from_edges(200, np.arange(199), np.arange(1, 200))
    keep = np.ones(len(ci), bool)
    keep[rp[100]:rp[101]] = ci[rp[100]:rp[101]] != 100  # row 100 without its diagonal
    ci2 = ci[keep]
    rp2 = rp.copy()
    rp2[101:] -= 1
    cases.append(("missing diagonal", rp2, ci2))
    return cases


@pytest.mark.parametrize("case", _symmetric_cases(), ids=lambda c: c[0])
def test_library_grouping_from_symmetric_pattern_matches_oracle(shim, case):
    """Groups read straight from a structurally symmetric pattern (the
    coarse levels of the device chain) equal the oracle's; the report that
    every row holds its diagonal once (which lets the level layout count
    entries from the row lengths) is given exactly when it is true and the
    16-bit lists were used."""
    name, rp, ci = case
    n = len(rp) - 1
    col = np.zeros(n, dtype=np.int32)
    diag_once = np.zeros(1, dtype=np.int32)
    g = shim.shim_color_sym(n, rp, ci, col, diag_once)
    c_or, g_or = O.color(rp, ci)
    assert g == g_or and np.array_equal(col, c_or)
    rows = np.repeat(np.arange(n), np.diff(rp))
    one_diag = bool(np.all(np.bincount(rows[ci == rows], minlength=n) == 1))
    assert one_diag == (name != "missing diagonal")
    assert bool(diag_once[0]) == (one_diag and name != "long coupling")


def _bipartite_cases():
    rng = np.random.default_rng(41)
    cases = []
    for shape in [(7, 5, 3), (16, 9, 1), (1, 1, 30), (12, 12, 12)]:
        s = synth.lognormal_grid(*shape, 1, 0, 1.0, 1.0, "none")
        cases.append((f"grid{shape}", s.row_ptr, s.col_ind))
    # random bipartite graphs with several components and isolated vertices;
    # vertex ids shuffled so that sides, components and degrees interleave
    for n in (60, 500, 3000):
        perm = rng.permutation(n)
        half = n // 2
        m = 3 * n
        a = rng.integers(0, half, m)
        b = half + rng.integers(0, n - half, m)
        # cut the graph into components by residue of the side-A end
        keep = (a % 3) == (b % 3)
        a, b = perm[a[keep]], perm[b[keep]]
        iso = perm[rng.choice(n, n // 20, replace=False)]
        sel = ~np.isin(a, iso) & ~np.isin(b, iso)
        rp, ci = _pattern_from_edges(n, a[sel], b[sel])
        cases.append((f"random-bipartite-{n}", rp, ci))
    # a star, a single edge, and no edges at all
    cases.append(("star", *_pattern_from_edges(9, np.zeros(8, int), np.arange(1, 9))))
    cases.append(("edge", *_pattern_from_edges(2, [0], [1])))
    cases.append(("no-edges", *_pattern_from_edges(5, [], [])))
    # nonsymmetric stored pattern whose symmetrisation is bipartite
    rp, ci = _pattern_from_edges(40, np.arange(0, 38, 2), np.arange(1, 39, 2), symmetric=False)
    cases.append(("nonsymmetric-chain", rp, ci))
    return cases


@pytest.mark.parametrize("case", _bipartite_cases(), ids=lambda c: c[0])
def test_library_grouping_of_bipartite_graphs_matches_oracle(shim, case):
    """Bipartite adjacency graphs take the library's closed form of Alg. 4.2
    (each component's side holding its best vertex first, the other sides
    second); the groups must equal the oracle's greedy bit for bit."""
    name, rp, ci = case
    c_lib, g_lib = _lib_color(shim, rp, ci)
    c_or, g_or = O.color(rp, ci)
    assert g_lib == g_or and np.array_equal(c_lib, c_or), name
    assert g_or <= 2


def test_library_grouping_with_one_odd_cycle_matches_oracle(shim):
    """A grid with one extra edge closing an odd cycle is not bipartite: the
    library falls back to the greedy, which must still equal the oracle."""
    s = synth.lognormal_grid(9, 8, 3, 1, 0, 1.0, 1.0, "none")
    n = s.n
    rows = np.repeat(np.arange(n), np.diff(s.row_ptr))
    rp, ci = _pattern_from_edges(n, np.concatenate([rows, [0]]),
                                 np.concatenate([s.col_ind, [10]]))  # 0 and 10: even distance
    c_lib, g_lib = _lib_color(shim, rp, ci)
    c_or, g_or = O.color(rp, ci)
    assert g_or >= 3
    assert g_lib == g_or and np.array_equal(c_lib, c_or)


def test_library_hierarchy_steps_match_oracle(shim):
    for sys, mc in [(synth.config(0), 64), (synth.lognormal_grid(20, 18, 9, 3, 5, 1.5, 0.1,
                                                                  "lateral4"), 200)]:
        s = O.OracleSolver(max_coarse=mc)
        s.setup(sys)
        assert s.nlevels >= 3
        for l in range(s.nlevels - 1):
            L = s.level(l)
            rp, ci, val = L["row_ptr"], L["col_ind"], L["val"]
            n = L["n"]
            col, g = _lib_color(shim, rp, ci)
            assert g == L["ncolors"] and np.array_equal(col, L["color"])
            a1 = np.zeros(n, dtype=np.int32)
            nc1 = shim.shim_pair(n, rp, ci, val, a1)
            crp = np.zeros(nc1 + 1, dtype=np.int32)
            cci = np.zeros(len(ci), dtype=np.int32)
            cv = np.zeros(len(ci))
            m = shim.shim_galerkin(n, rp, ci, val, a1, nc1, crp, cci, cv)
            a2 = np.zeros(nc1, dtype=np.int32)
            nc2 = shim.shim_pair(nc1, crp, cci[:m].copy(), cv[:m].copy(), a2)
            drp = np.zeros(nc2 + 1, dtype=np.int32)
            dci = np.zeros(m, dtype=np.int32)
            dv = np.zeros(m)
            m2 = shim.shim_galerkin(nc1, crp, cci[:m].copy(), cv[:m].copy(), a2, nc2, drp, dci, dv)
            assert np.array_equal(a2[a1], L["agg"])
            nxt = s.level(l + 1)
            assert np.array_equal(drp, nxt["row_ptr"]) and np.array_equal(dci[:m2], nxt["col_ind"])
            assert np.array_equal(dv[:m2], nxt["val"])  # same summation order: exact


def _sparse_nonsymmetric(n, per_row, seed):
    """Random CSR with a diagonal and `per_row` off-diagonal entries per row
    (pattern not symmetric), negative off-diagonals and a dominant diagonal."""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n):
        c = np.unique(np.concatenate([[i], rng.integers(0, n, per_row)]))
        rows.append(c)
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(c) for c in rows])
    ci = np.concatenate(rows).astype(np.int32)
    val = -rng.uniform(0.0, 1.0, len(ci))
    r = np.repeat(np.arange(n), np.diff(rp))
    val[ci == r] = 2.0 * per_row
    return rp, ci, val


@pytest.mark.parametrize("case", ["grid_32k", "nonsymmetric_20k", "nonsymmetric_small"])
def test_library_pair_and_galerkin_large(shim, case):
    """Sizes that take the library's multi-threaded row-chunk paths (and the
    counting-sort transpose of a nonsymmetric pattern) against the oracle."""
    if case == "grid_32k":
        rp, ci, val = synth.poisson_csr((40, 40, 20))
        val = val * np.random.default_rng(3).uniform(0.5, 1.5, len(val))
    elif case == "nonsymmetric_20k":
        rp, ci, val = _sparse_nonsymmetric(20000, 5, 7)
    else:
        rp, ci, val = _sparse_nonsymmetric(300, 4, 8)
    n = len(rp) - 1
    a1 = np.zeros(n, dtype=np.int32)
    nc1 = shim.shim_pair(n, rp, ci, val, a1)
    o1, onc1 = O.npair_pass(rp, ci, val)
    assert nc1 == onc1 and np.array_equal(a1, o1)
    crp = np.zeros(nc1 + 1, dtype=np.int32)
    cci = np.zeros(len(ci), dtype=np.int32)
    cv = np.zeros(len(ci))
    m = shim.shim_galerkin(n, rp, ci, val, a1, nc1, crp, cci, cv)
    orp, oci, ov = O.galerkin(rp, ci, val, o1, onc1)
    assert np.array_equal(crp, orp) and np.array_equal(cci[:m], oci)
    assert np.array_equal(cv[:m], ov)


@pytest.mark.parametrize("dims,mc", [((24, 60, 25), 100), ((20, 44, 17), 60)])
def test_library_hierarchy_with_stalled_level_matches_oracle(shim, dims, mc):
    """Layered channelised grids whose coarsening stalls (the two pairwise
    passes keep more than 90% of a level's rows), so singletons are absorbed:
    the library's chain against the oracle's, bit for bit."""
    sys = synth.layered_grid(*dims, 4, 0)
    o = O.OracleSolver(max_coarse=mc)
    o.setup(sys)
    L0 = o.level(0)
    rp, ci, val = L0["row_ptr"], L0["col_ind"], L0["val"]
    shim.shim_hierarchy.restype = C.c_int
    sizes = np.zeros(32, dtype=np.int32)
    aggs = np.zeros(4 * len(rp), dtype=np.int32)
    crp = np.zeros(len(rp), dtype=np.int32)
    cci = np.zeros(len(ci), dtype=np.int32)
    cv = np.zeros(len(ci))
    nl = shim.shim_hierarchy(len(rp) - 1, rp, ci, val, mc, sizes, aggs, crp, cci, cv)
    assert nl == o.nlevels
    sizes_o = [o.level(l)["n"] for l in range(nl)]
    assert list(sizes[:nl]) == sizes_o
    # the stall rule fired: some level shrank by more than the pairwise factor
    assert any(sizes_o[l + 1] < sizes_o[l] / 5 for l in range(nl - 1))
    off = 0
    for l in range(nl - 1):
        n_l = sizes_o[l]
        assert np.array_equal(aggs[off:off + n_l], o.level(l)["agg"])
        off += n_l
    Lc = o.level(nl - 1)
    m = Lc["n"]
    assert np.array_equal(crp[:m + 1], Lc["row_ptr"])
    nnz = Lc["row_ptr"][-1]
    assert np.array_equal(cci[:nnz], Lc["col_ind"]) and np.array_equal(cv[:nnz], Lc["val"])


def test_library_pattern_check(shim):
    rp, ci, _ = synth.poisson_csr((4, 3, 2))
    assert shim.shim_pattern(len(rp) - 1, rp, ci, len(ci)) == 0
    bad = ci.copy()
    bad[0], bad[1] = bad[1], bad[0]
    assert shim.shim_pattern(len(rp) - 1, rp, bad, len(ci)) == -2
    for v in (-1, len(rp) - 1):
        bad = ci.copy()
        bad[2] = v
        assert shim.shim_pattern(len(rp) - 1, rp, bad, len(ci)) == -2


@pytest.mark.parametrize("shape", [(6, 5, 4), (64, 64, 32), (60, 220, 85)])
def test_bilu_levels_are_hyperplanes(shim, shape):
    nx, ny, nz = shape
    rp, ci, _ = synth.poisson_csr(shape)
    n = len(rp) - 1
    rows = np.zeros(n, dtype=np.int32)
    nlev = shim.shim_levels(n, rp, ci, 1, rows)
    assert nlev == nx + ny + nz - 2
    nlev_b = shim.shim_levels(n, rp, ci, 0, rows)
    assert nlev_b == nx + ny + nz - 2


@pytest.mark.parametrize("seed", range(6))
def test_group_parallel_levels_equal_the_sequential_pass(shim, seed):
    """Dependency levels of the multi-color elimination order, computed group
    by group in parallel, are those of the sequential pass, entry for entry;
    an order whose groups are not independent sets is declined."""
    rng = np.random.default_rng(100 + seed)
    if seed < 3:
        rp, ci, _ = synth.poisson_csr((8 + 4 * seed, 7 + 3 * seed, 5 + seed))
    else:
        # 27-point pattern, large enough for the threaded chunks, with a few
        # random long-range couplings
        dims = (26 + seed, 24, 20 + seed)
        T = [sp.diags([1.0, 1.0, 1.0], [-1, 0, 1], shape=(d, d)) for d in dims]
        Pm = sp.kron(sp.kron(T[2], T[1]), T[0]).tocsr()
        n = Pm.shape[0]
        i = rng.integers(0, n, 40)
        j = rng.integers(0, n, 40)
        E = sp.coo_matrix((np.ones(40), (i, j)), shape=(n, n))
        Pm = ((Pm + E + E.T) != 0).astype(np.float64).tocsr()
        Pm.sort_indices()
        rp, ci = Pm.indptr.astype(np.int32), Pm.indices.astype(np.int32)
    n = len(rp) - 1
    col, g = _lib_color(shim, rp, ci)
    ord_ = np.argsort(col, kind="stable").astype(np.int32)
    grp = np.concatenate([[0], np.cumsum(np.bincount(col, minlength=col.max() + 1))]).astype(np.int32)
    for lower in (1, 0):
        r1, p1 = np.zeros(n, np.int32), np.zeros(n + 1, np.int32)
        r2, p2 = np.zeros(n, np.int32), np.zeros(n + 1, np.int32)
        nl1 = shim.shim_levels_ord(n, rp, ci, ord_, lower, r1, p1)
        nl2 = shim.shim_levels_groups(n, rp, ci, ord_, len(grp) - 1, grp, lower, r2, p2)
        assert nl2 == nl1
        assert np.array_equal(r1, r2) and np.array_equal(p1[:nl1 + 1], p2[:nl2 + 1])
    # natural order cut in two halves: rows of one half are coupled
    half = np.array([0, n // 2, n], dtype=np.int32)
    nat = np.arange(n, dtype=np.int32)
    r2, p2 = np.zeros(n, np.int32), np.zeros(n + 1, np.int32)
    assert shim.shim_levels_groups(n, rp, ci, nat, 2, half, 1, r2, p2) == -1
