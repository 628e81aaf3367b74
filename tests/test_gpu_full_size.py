"""GPU parity at full size, in the launch configuration the benchmark times.

Workloads: 64x64x32 cells b=4 (both block ILU(0) orders), 128x128x64 cells
b=7 (FP64 and FP32 preconditioners; the benchmark's default), and the
60x220x85 layered grid b=4 whose coarsening stalls.  For each: the hierarchy
bit for bit, then every kernel entry by entry against the oracle on the same
inputs (bars as in test_gpu_parity.py), the FGMRES iteration count within one
of the oracle's, and the solution error against the oracle's FP64 solution.
The coarsest-level solve is also checked on its own, on the coarsest matrix of
the real hierarchy (the block LU's full chain of 128-wide steps).
"""
import numpy as np
import pytest
import torch

import _checks as K
from oracle import oracle as O
from paper_2208_08594_amd import msp, synth

pytestmark = pytest.mark.gpu

WORKLOADS = {
    "64x64x32b4": 1,
    "128x128x64b7": 2,
    "60x220x85b4-layered": 3,
}


def announce(*a):
    print("[case]", *a, flush=True)


def to_np(t):
    return t.detach().cpu().numpy()


_SOLUTIONS = {}


def oracle_solution(full):
    """The oracle's FP64 FGMRES solve of the workload (computed once)."""
    name, sys, g, o = full
    if name not in _SOLUTIONS:
        _SOLUTIONS[name] = o.solve(sys.rhs, 1e-6)
    return _SOLUTIONS[name]


@pytest.fixture(scope="module", params=list(WORKLOADS), ids=list(WORKLOADS))
def full(request):
    sys = synth.config(WORKLOADS[request.param])
    announce(request.param, f"n={sys.n} b={sys.b} N={sys.N}")
    g = msp.Solver(max_coarse=10000, bilu_order=1)
    g.setup(sys)
    o = O.OracleSolver(max_coarse=10000, bilu_order=1)
    o.setup(sys)
    yield request.param, sys, g, o
    _SOLUTIONS.pop(request.param, None)
    g.close()
    o.close()
    torch.cuda.empty_cache()


def test_hierarchy_and_weights_bit_exact(full):
    name, sys, g, o = full
    assert g.nlevels == o.nlevels >= 2
    for l in range(o.nlevels):
        a, b = g.level(l), o.level(l)
        assert a["n"] == b["n"], (name, l)
        assert np.array_equal(a["row_ptr"], b["row_ptr"]), (name, l)
        assert np.array_equal(a["col_ind"], b["col_ind"]), (name, l)
        assert np.array_equal(a["val"], b["val"]), (name, l)
        if l < o.nlevels - 1:
            assert a["ncolors"] == b["ncolors"]
            assert np.array_equal(a["color"], b["color"]) and np.array_equal(a["agg"], b["agg"])
    assert o.level(0)["ncolors"] == 2
    assert np.array_equal(g.omega(), o.omega())
    announce(name, "levels", [o.level(l)["n"] for l in range(o.nlevels)],
             "colors", [o.level(l)["ncolors"] for l in range(o.nlevels - 1)])


def test_spmv_entrywise(full):
    name, sys, g, o = full
    x = np.random.default_rng(11).uniform(-1, 1, sys.N)
    r = K.assert_entrywise(to_np(g.spmv(x)), o.spmv(x), 1e-13, K.spmv_scale(K.bsr(sys), x),
                           name + " SpMV")
    announce(name, f"SpMV worst err/scale {r:.2e}")


def test_gs_sweeps_every_level(full):
    name, sys, g, o = full
    rng = np.random.default_rng(12)
    for l in range(o.nlevels - 1):
        L = o.level(l)
        f = rng.uniform(-1, 1, L["n"])
        x0 = rng.uniform(-1, 1, L["n"])
        for fwd in (True, False):
            xg = to_np(g.smooth(l, f, x0, fwd))
            K.gs_local_residual(L, f, x0, xg, fwd, 1e-14, f"{name} GS level {l} fwd={fwd}")
            xo = O.gs_sweep(L["row_ptr"], L["col_ind"], L["val"], L["color"], L["ncolors"],
                            f, x0, fwd)
            K.close(xg, xo, 1e-12, f"{name} GS level {l} fwd={fwd} vs oracle")


def check_bilu(name, sys, g, o):
    Fg, Dg = g.bilu()
    Fo, Do = o.bilu()
    K.blocks_close(Fg, Fo, 1e-12, name + " BILU factors")
    K.blocks_close(Dg, Do, 1e-12, name + " inverted pivot blocks")
    del Fg, Dg
    order = (O.multicolor_order(sys.row_ptr, sys.col_ind) if g.bilu_order == 1
             else np.arange(sys.n))
    L, U = K.bilu_factors(sys, Fo, Do, order)
    r = np.random.default_rng(13).uniform(-1, 1, sys.N)
    zg = to_np(g.bilu_apply(r))
    K.bilu_backward_error(L, U, r, zg, 1e-13, name + " BILU solve backward error")
    K.close(zg, o.bilu_apply(r), 1e-12, name + " BILU solve vs oracle")


def test_bilu_factors_and_solve(full):
    check_bilu(*full)


def test_natural_order_bilu_at_full_size():
    """Block ILU(0) in natural block order (158 hyperplane levels each way on
    64x64x32): factors, solve and the FGMRES iteration count."""
    sys = synth.config(1)
    announce("64x64x32b4 natural-order BILU")
    g = msp.Solver(max_coarse=10000, bilu_order=0)
    g.setup(sys)
    o = O.OracleSolver(max_coarse=10000, bilu_order=0)
    o.setup(sys)
    assert g.info()["bilu_levels_fwd"] == sys.nx + sys.ny + sys.nz - 2
    check_bilu("64x64x32b4 natural order", sys, g, o)
    xg, ig = g.solve(sys.rhs, rtol=1e-6)
    xo, it, rr, st = o.solve(sys.rhs, 1e-6)
    assert abs(ig["iterations"] - it) <= 1 and ig["rel_true_residual"] <= 1e-6
    g.close()
    o.close()


def test_vcycle_and_apply(full):
    name, sys, g, o = full
    t = K.coarse_tol_of(o.level(o.nlevels - 1))
    rng = np.random.default_rng(14)
    f = rng.uniform(-1, 1, sys.n)
    rv = K.close(to_np(g.vcycle(f)), o.vcycle(f), t, name + " V-cycle")
    v = rng.uniform(-1, 1, sys.N)
    ra = K.close(to_np(g.apply(v)), o.apply(v), t, name + " preconditioner apply")
    announce(name, f"coarse tol {t:.1e}; V-cycle worst {rv:.2e}; apply worst {ra:.2e}")


def test_coarsest_solve_on_the_real_coarsest_matrix(full):
    """The coarsest matrix of this hierarchy set up as a whole (scalar)
    system, so the V-cycle is the direct solve of its decoupled form (rows
    scaled by the inverse diagonal) alone: every 128-wide step of the block
    LU and both triangular-inverse sweeps at their real size.  Row by row
    A x = f, and x against the oracle's LAPACK LU solve."""
    name, sys, g, o = full
    Lc = o.level(o.nlevels - 1)
    m = Lc["n"]
    announce(name, f"coarsest matrix alone, n={m}")
    args = dict(n=m, b=1, p=0, row_ptr=Lc["row_ptr"], col_ind=Lc["col_ind"],
                vals=Lc["val"].reshape(-1, 1, 1))
    gc = msp.Solver(max_coarse=10000)
    gc.setup(**args)
    oc = O.OracleSolver(max_coarse=10000)
    oc.setup(**args)
    assert gc.nlevels == 1 and oc.nlevels == 1
    A0 = oc.level(0)
    assert np.array_equal(gc.level(0)["val"], A0["val"])
    t = K.coarse_tol_of(A0)
    f = np.random.default_rng(15).uniform(-1, 1, m)
    xg = to_np(gc.vcycle(f))
    K.dense_backward_error(K.csr(A0), xg, f, t, name + " coarsest solve backward error")
    r = K.close(xg, oc.vcycle(f), t, name + " coarsest solve vs oracle LU")
    announce(name, f"coarsest solve alone: tol {t:.1e}, worst {r:.2e}")
    gc.close()
    oc.close()


def test_fgmres_and_solution_error(full):
    name, sys, g, o = full
    xg, ig = g.solve(sys.rhs, rtol=1e-6)
    xo, it, rr, st = oracle_solution(full)
    xg = to_np(xg)
    err = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    announce(name, f"FP64 iterations gpu {ig['iterations']} oracle {it}; relres "
                   f"{ig['rel_true_residual']:.2e} / {rr:.2e}; |x-xo|/|xo| {err:.2e}")
    assert ig["status"] == 0 and st == 0
    assert abs(ig["iterations"] - it) <= 1
    assert ig["rel_true_residual"] <= 1e-6 and rr <= 1e-6
    # true residual of the GPU solution, recomputed here in FP64
    A = K.bsr(sys)
    assert np.linalg.norm(sys.rhs - A @ xg) <= 1e-6 * np.linalg.norm(sys.rhs)
    assert err <= 1e-4


def test_fp32_preconditioner_against_fp64_oracle(full):
    """The FP32 preconditioner of the benchmark: stored values RNE of the
    FP64 setup, apply against the oracle's FP32 apply, and the solve's
    iterations and solution error against the FP64 oracle."""
    name, sys, g, o = full
    g32 = msp.Solver(max_coarse=10000, precond_fp32=True, bilu_order=g.bilu_order)
    g32.setup(sys)
    for l in range(o.nlevels - 1):
        assert np.array_equal(g32.level_f32(l), o.level(l)["val"].astype(np.float32)), l
    o32 = O.OracleSolver(max_coarse=10000, precond_fp32=True, bilu_order=g.bilu_order)
    o32.setup(sys)
    v = np.random.default_rng(16).uniform(-1, 1, sys.N)
    ra = K.close(to_np(g32.apply(v)), o32.apply(v), 1e-5, name + " FP32 apply")
    o32.close()
    x32, i32 = g32.solve(sys.rhs, rtol=1e-6)
    g32.close()
    xo, it, rr, st = oracle_solution(full)
    x32 = to_np(x32)
    err = np.linalg.norm(x32 - xo) / np.linalg.norm(xo)
    announce(name, f"FP32 apply worst {ra:.2e}; FP32-preconditioned iterations "
                   f"{i32['iterations']} (FP64 oracle {it}); relres {i32['rel_true_residual']:.2e}; "
                   f"|x32-xo|/|xo| {err:.2e}")
    assert abs(i32["iterations"] - it) <= 1
    assert i32["rel_true_residual"] <= 1e-6
    assert err <= 1e-4
