"""ctypes wrapper of the plain sequential FP64 oracle (msp_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the package smoke
check and the CPU-baseline leg of the benchmark.  The product path never
imports it, and it imports nothing from the product package.

The coarsest AMG level is factorised here with LAPACK getrf
(``scipy.linalg.lu_factor``: partial pivoting, first largest pivot), a library
primitive; the C code applies the factors inside the V-cycle.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np
import scipy.linalg

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "msp_oracle.c")
LIB_PATH = os.path.join(HERE, "libmsp_oracle.so")
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11"]

STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_PATTERN", -3: "ERR_SINGULAR", -4: "ERR_NONFINITE",
          -5: "ERR_NOMEM", -8: "ERR_STATE", -9: "ERR_COARSE", 1: "NOT_CONVERGED"}


class OracleError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        super().__init__(f"oracle {where}: {STATUS.get(code, code)}")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no contraction)."""
    deps = [SRC, os.path.join(HERE, "oracle_apply.inc"), os.path.join(HERE, "oracle_cycle.inc")]
    if not force and os.path.exists(LIB_PATH) and all(
            os.path.getmtime(LIB_PATH) >= os.path.getmtime(d) for d in deps):
        return LIB_PATH
    tmp = LIB_PATH + f".tmp{os.getpid()}"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"], cwd=HERE)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_LIB = None

i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    build(force=False)
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.or_validate.argtypes = [C.c_int, C.c_int, C.c_int, i32p, i32p, f64p, C.c_long]
    L.or_decouple.argtypes = [C.c_int, C.c_int, C.c_int, i32p, i32p, f64p, f64p, f64p]
    L.or_color.argtypes = [C.c_int, i32p, i32p, i32p]
    L.or_npair_pass.argtypes = [C.c_int, i32p, i32p, f64p, i32p]
    L.or_absorb_singletons.argtypes = [C.c_int, i32p, i32p, f64p, i32p, C.c_int]
    L.or_galerkin.argtypes = [C.c_int, i32p, i32p, f64p, i32p, C.c_int, i32p, i32p, f64p]
    L.or_galerkin.restype = C.c_long
    L.or_bilu0_factor.argtypes = [C.c_int, C.c_int, i32p, i32p, f64p, f64p, f64p]
    L.or_bilu0_solve.argtypes = [C.c_int, C.c_int, i32p, i32p, f64p, f64p, f64p, f64p]
    L.or_bilu0_solve.restype = None
    L.or_bilu0_factor_ordered.argtypes = [C.c_int, C.c_int, i32p, i32p, f64p, i32p, f64p, f64p]
    L.or_bilu0_solve_ordered.argtypes = [C.c_int, C.c_int, i32p, i32p, f64p, f64p, i32p, f64p,
                                         f64p]
    L.or_bilu0_solve_ordered.restype = None
    L.or_multicolor_order.argtypes = [C.c_int, i32p, i32p, i32p]
    L.or_gs_sweep.argtypes = [C.c_int, i32p, i32p, f64p, i32p, C.c_int, f64p, f64p, C.c_int]
    L.or_jacobi_sweep.argtypes = [C.c_int, i32p, i32p, f64p, C.c_double, f64p, f64p, f64p]
    L.or_gs_sweep.restype = None
    L.or_lu_solve.argtypes = [C.c_int, f64p, i32p, f64p, f64p]
    L.or_lu_solve.restype = None
    L.or_create.argtypes = [C.c_int] * 7 + [C.c_double, C.c_int, C.c_int, C.c_int, C.c_int]
    L.or_create.restype = vp
    L.or_destroy.argtypes = [vp]
    L.or_destroy.restype = None
    L.or_setup.argtypes = [vp, C.c_int, C.c_int, C.c_int, i32p, i32p, f64p, C.c_long,
                           C.POINTER(C.c_int)]
    L.or_coarse_n.argtypes = [vp]
    L.or_get_coarse_dense.argtypes = [vp, f64p]
    L.or_get_coarse_dense.restype = None
    L.or_set_coarse_lu.argtypes = [vp, f64p, i32p]
    L.or_apply.argtypes = [vp, f64p, f64p]
    L.or_vcycle.argtypes = [vp, f64p, f64p]
    L.or_bilu_apply.argtypes = [vp, f64p, f64p]
    L.or_spmv.argtypes = [vp, f64p, f64p]
    L.or_spmv.restype = None
    L.or_solve.argtypes = [vp, f64p, f64p, C.c_double, C.POINTER(C.c_int), C.POINTER(C.c_double)]
    for name in ["or_nlevels", "or_setup_calls"]:
        getattr(L, name).argtypes = [vp]
    for name in ["or_level_n", "or_level_ncolors", "or_level_nc"]:
        getattr(L, name).argtypes = [vp, C.c_int]
    L.or_level_nnz.argtypes = [vp, C.c_int]
    L.or_level_nnz.restype = C.c_long
    L.or_get_level.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp]
    L.or_get_level.restype = None
    L.or_get_omega.argtypes = [vp, f64p]
    L.or_get_omega.restype = None
    L.or_get_nstage.argtypes = [vp, vp, vp]
    L.or_get_bilu.argtypes = [vp, vp, vp]
    L.or_get_bilu.restype = None
    _LIB = L
    return L


def _check(code, where):
    if code < 0:
        raise OracleError(code, where)
    return code


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# Stand-alone steps (pins and per-step parity)
# --------------------------------------------------------------------------
def validate(n, b, p, rp, ci, vals):
    return lib().or_validate(n, b, p, _i32(rp), _i32(ci), _f64(vals).reshape(-1), len(ci))


def decouple(n, b, p, rp, ci, vals):
    """ABF decoupling weights omega [n, b] and pressure matrix values [nnzb]."""
    om = np.zeros(n * b)
    ap = np.zeros(len(ci))
    _check(lib().or_decouple(n, b, p, _i32(rp), _i32(ci), _f64(vals).reshape(-1), om, ap),
           "decouple")
    return om.reshape(n, b), ap


def color(rp, ci):
    """VerticesGrouping colors (1..g) of the symmetrised adjacency graph."""
    n = len(rp) - 1
    col = np.zeros(n, dtype=np.int32)
    g = _check(lib().or_color(n, _i32(rp), _i32(ci), col), "color")
    return col, g


def npair_pass(rp, ci, val):
    n = len(rp) - 1
    agg = np.zeros(n, dtype=np.int32)
    nc = _check(lib().or_npair_pass(n, _i32(rp), _i32(ci), _f64(val), agg), "npair")
    return agg, nc


def absorb_singletons(rp, ci, val, agg, nc):
    """Stalled-coarsening step: eligible rows alone in their aggregate join the
    aggregate of their strongest neighbour in an aggregate of two or more rows;
    returns the new aggregate map and count."""
    n = len(rp) - 1
    out = _i32(agg).copy()
    k = _check(lib().or_absorb_singletons(n, _i32(rp), _i32(ci), _f64(val), out, int(nc)),
               "absorb")
    return out, k


def galerkin(rp, ci, val, agg, nc):
    n = len(rp) - 1
    cap = max(len(ci), 1)
    crp = np.zeros(nc + 1, dtype=np.int32)
    cci = np.zeros(cap, dtype=np.int32)
    cval = np.zeros(cap)
    nnz = _check(lib().or_galerkin(n, _i32(rp), _i32(ci), _f64(val), _i32(agg), nc, crp, cci,
                                   cval), "galerkin")
    return crp, cci[:nnz].copy(), cval[:nnz].copy()


def multicolor_order(rp, ci):
    """Elimination order: the groups of Alg. 4.2 one after another."""
    n = len(rp) - 1
    ord_ = np.zeros(n, dtype=np.int32)
    _check(lib().or_multicolor_order(n, _i32(rp), _i32(ci), ord_), "multicolor_order")
    return ord_


def bilu0_factor(n, b, rp, ci, vals, order=None):
    """Block ILU(0) in natural order, or in the elimination order `order`."""
    F = np.zeros(len(ci) * b * b)
    D = np.zeros(n * b * b)
    if order is None:
        st = lib().or_bilu0_factor(n, b, _i32(rp), _i32(ci), _f64(vals).reshape(-1), F, D)
    else:
        st = lib().or_bilu0_factor_ordered(n, b, _i32(rp), _i32(ci), _f64(vals).reshape(-1),
                                           _i32(order), F, D)
    _check(st, "bilu0_factor")
    return F.reshape(-1, b, b), D.reshape(n, b, b)


def bilu0_solve(n, b, rp, ci, F, D, r, order=None):
    z = np.zeros(n * b)
    if order is None:
        lib().or_bilu0_solve(n, b, _i32(rp), _i32(ci), _f64(F).reshape(-1), _f64(D).reshape(-1),
                             _f64(r), z)
    else:
        lib().or_bilu0_solve_ordered(n, b, _i32(rp), _i32(ci), _f64(F).reshape(-1),
                                     _f64(D).reshape(-1), _i32(order), _f64(r), z)
    return z


def gs_sweep(rp, ci, val, color_, g, f, x, forward=True):
    x = _f64(x).copy()
    lib().or_gs_sweep(len(rp) - 1, _i32(rp), _i32(ci), _f64(val), _i32(color_), g, _f64(f), x,
                      1 if forward else 0)
    return x


def jacobi_sweep(rp, ci, val, w, f, x):
    """One weighted point-Jacobi sweep: x + w D^-1 (f - A x)."""
    out = np.zeros(len(rp) - 1)
    _check(lib().or_jacobi_sweep(len(rp) - 1, _i32(rp), _i32(ci), _f64(val), float(w), _f64(f),
                                 _f64(x), out), "jacobi")
    return out


def lu_factor(A):
    lu, piv = scipy.linalg.lu_factor(np.asarray(A, dtype=np.float64), check_finite=True)
    return np.ascontiguousarray(lu), np.ascontiguousarray(piv, dtype=np.int32)


def lu_solve(lu, piv, f):
    m = lu.shape[0]
    x = np.zeros(m)
    lib().or_lu_solve(m, _f64(lu), _i32(piv), _f64(f), x)
    return x


# --------------------------------------------------------------------------
# Solver context: adaptive setup + FGMRES (a Newton sequence of systems)
# --------------------------------------------------------------------------
class OracleSolver:
    """smoother: 0 = PGS-MC, 1 = weighted point Jacobi (jacobi_weight), 2 =
    sequential Gauss-Seidel in natural order (a comparison reference; the
    library has no such smoother);
    nu_pre/nu_post: sweeps around the coarse correction; full_smoother:
    0 = block ILU(0), 1 = block Jacobi; n_stage: 1 runs the concentration
    stage B_N (one block Gauss-Seidel sweep) before the pressure stage."""

    def __init__(self, mu=0, restart=30, max_iter=1000, max_coarse=10000, precond_fp32=False,
                 bilu_order=1, smoother=0, jacobi_weight=1.0, nu_pre=1, nu_post=1,
                 full_smoother=0, n_stage=0):
        self._lib = lib()
        self.h = self._lib.or_create(int(mu), int(restart), int(max_iter), int(max_coarse),
                                     1 if precond_fp32 else 0, int(bilu_order), int(smoother),
                                     float(jacobi_weight), int(nu_pre), int(nu_post),
                                     int(full_smoother), int(n_stage))
        if not self.h:
            raise MemoryError("or_create")
        self.n = self.b = self.p = None

    def close(self):
        if self.h:
            self._lib.or_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def setup(self, sys=None, *, n=None, b=None, p=0, row_ptr=None, col_ind=None, vals=None):
        """Ingest one Jacobian; rebuild or reuse the preconditioner.  Returns rebuilt."""
        if sys is not None:
            n, b, p, row_ptr, col_ind, vals = sys.n, sys.b, sys.p, sys.row_ptr, sys.col_ind, sys.vals
        reb = C.c_int(0)
        _check(self._lib.or_setup(self.h, n, b, p, _i32(row_ptr), _i32(col_ind),
                                  _f64(vals).reshape(-1), len(col_ind), C.byref(reb)), "setup")
        self.n, self.b, self.p = n, b, p
        if reb.value:
            m = self._lib.or_coarse_n(self.h)
            dense = np.zeros(m * m)
            self._lib.or_get_coarse_dense(self.h, dense)
            lu, piv = lu_factor(dense.reshape(m, m))
            _check(self._lib.or_set_coarse_lu(self.h, lu, piv), "coarse lu")
        return bool(reb.value)

    def solve(self, rhs, rtol=1e-6, x0=None):
        x = np.zeros(self.n * self.b) if x0 is None else _f64(x0).copy()
        it = C.c_int(0)
        rr = C.c_double(0.0)
        st = self._lib.or_solve(self.h, _f64(rhs), x, rtol, C.byref(it), C.byref(rr))
        _check(st, "solve")
        return x, it.value, rr.value, st

    def apply(self, v):
        z = np.zeros(self.n * self.b)
        _check(self._lib.or_apply(self.h, _f64(v), z), "apply")
        return z

    def vcycle(self, f):
        x = np.zeros(self.n)
        _check(self._lib.or_vcycle(self.h, _f64(f), x), "vcycle")
        return x

    def bilu_apply(self, r):
        z = np.zeros(self.n * self.b)
        _check(self._lib.or_bilu_apply(self.h, _f64(r), z), "bilu")
        return z

    def spmv(self, x):
        y = np.zeros(self.n * self.b)
        self._lib.or_spmv(self.h, _f64(x), y)
        return y

    @property
    def setup_calls(self):
        return self._lib.or_setup_calls(self.h)

    @property
    def nlevels(self):
        return self._lib.or_nlevels(self.h)

    def level(self, l):
        L = self._lib
        n = L.or_level_n(self.h, l)
        nnz = L.or_level_nnz(self.h, l)
        rp = np.zeros(n + 1, dtype=np.int32)
        ci = np.zeros(nnz, dtype=np.int32)
        val = np.zeros(nnz)
        last = l == self.nlevels - 1
        color_ = None if last else np.zeros(n, dtype=np.int32)
        agg = None if last else np.zeros(n, dtype=np.int32)
        ptr = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
        L.or_get_level(self.h, l, ptr(rp), ptr(ci), ptr(val), ptr(color_), ptr(agg))
        return dict(n=n, row_ptr=rp, col_ind=ci, val=val, color=color_, agg=agg,
                    ncolors=L.or_level_ncolors(self.h, l), nc=L.or_level_nc(self.h, l))

    def omega(self):
        om = np.zeros(self.n * self.b)
        self._lib.or_get_omega(self.h, om)
        return om.reshape(self.n, self.b)

    def bilu(self):
        nnzb = self.level(0)["row_ptr"][-1]
        F = np.zeros(nnzb * self.b * self.b)
        D = np.zeros(self.n * self.b * self.b)
        self._lib.or_get_bilu(self.h, F.ctypes.data_as(C.c_void_p), D.ctypes.data_as(C.c_void_p))
        return F.reshape(-1, self.b, self.b), D.reshape(self.n, self.b, self.b)

    def nstage(self):
        m = self.b - 1
        nnzb = int(self.level(0)["row_ptr"][-1])
        Dn = np.zeros(self.n * m * self.b)
        Ann = np.zeros(nnzb * m * m)
        _check(self._lib.or_get_nstage(self.h, Dn.ctypes.data_as(C.c_void_p),
                                       Ann.ctypes.data_as(C.c_void_p)), "nstage")
        return Dn.reshape(self.n, m, self.b), Ann.reshape(nnzb, m, m)
