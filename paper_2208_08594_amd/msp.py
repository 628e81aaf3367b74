"""ctypes binding of libmsp (include/msp.h, include/msp_stages.h).

Argument marshalling only: every step of the solve runs in the HIP kernels of
libmsp.so.  Device memory comes from PyTorch's caching allocator (through the
library's allocator callbacks) and work is ordered on a torch stream.  The
binding raises if libmsp.so is missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsp.so")

MSP_OK = 0
MSP_NOT_CONVERGED = 1
STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_PATTERN", -3: "ERR_SINGULAR", -4: "ERR_NONFINITE",
          -5: "ERR_NOMEM", -6: "ERR_HIP", -7: "ERR_NO_DEVICE", -8: "ERR_STATE",
          -9: "ERR_COARSE", -10: "ERR_SCRATCH", 1: "NOT_CONVERGED"}
NOALLOC_SCRATCH_BYTES = 128 << 20
MAX_LEVELS = 25

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class MspOptions(C.Structure):
    _fields_ = [("mu", C.c_int), ("restart", C.c_int), ("max_iter", C.c_int),
                ("max_coarse", C.c_int), ("precond_fp32", C.c_int), ("bilu_order", C.c_int),
                ("use_graphs", C.c_int), ("stream", C.c_void_p), ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN),
                ("alloc_user", C.c_void_p), ("smoother", C.c_int), ("nu_pre", C.c_int),
                ("nu_post", C.c_int), ("full_smoother", C.c_int), ("jacobi_weight", C.c_double),
                ("n_stage", C.c_int), ("host_chain", C.c_int)]


class MspInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", C.c_int), ("restarts", C.c_int),
                ("rebuilt", C.c_int), ("setup_calls", C.c_int), ("solves", C.c_int),
                ("n_levels", C.c_int), ("level_rows", C.c_int * MAX_LEVELS),
                ("n_colors", C.c_int * MAX_LEVELS), ("bilu_levels_fwd", C.c_int),
                ("bilu_levels_bwd", C.c_int), ("rel_true_residual", C.c_double),
                ("setup_ms", C.c_double), ("rebuild_ms", C.c_double), ("solve_ms", C.c_double),
                ("phase_ms", C.c_double * 8)]

    def as_dict(self):
        nl = self.n_levels
        return dict(status=self.status, iterations=self.iterations, restarts=self.restarts,
                    rebuilt=bool(self.rebuilt), setup_calls=self.setup_calls, solves=self.solves,
                    n_levels=nl, level_rows=list(self.level_rows[:nl]),
                    n_colors=list(self.n_colors[:nl]), bilu_levels_fwd=self.bilu_levels_fwd,
                    bilu_levels_bwd=self.bilu_levels_bwd,
                    rel_true_residual=self.rel_true_residual, setup_ms=self.setup_ms,
                    rebuild_ms=self.rebuild_ms, solve_ms=self.solve_ms,
                    phase_ms=list(self.phase_ms))


# every exported symbol and its signature (checked by the CPU tests against the headers)
_vp, _i, _ll, _d = C.c_void_p, C.c_int, C.c_longlong, C.c_double
SIGNATURES = {
    "msp_default_options": ([C.POINTER(MspOptions)], _i),
    "msp_create": ([C.POINTER(_vp), C.POINTER(MspOptions)], _i),
    "msp_setup": ([_vp, _i, _i, _i, _vp, _vp, _vp, _ll], _i),
    "msp_solve": ([_vp, _vp, _vp, _d, C.POINTER(MspInfo)], _i),
    "msp_solve_noalloc": ([_vp, _vp, _vp, _d, C.POINTER(MspInfo)], _i),
    "msp_solve_batch": ([_vp, _i, _vp, _vp, _d, _vp], _i),
    "msp_get_info": ([_vp, C.POINTER(MspInfo)], _i),
    "msp_footprint": ([_i, _ll, _i, C.POINTER(MspOptions), C.POINTER(C.c_size_t)], _i),
    "msp_destroy": ([_vp], _i),
    "msp_status_string": ([_i], C.c_char_p),
    "msp_stage_spmv": ([_vp, _vp, _vp], _i),
    "msp_stage_precond": ([_vp, _vp, _vp], _i),
    "msp_stage_vcycle": ([_vp, _vp, _vp], _i),
    "msp_stage_smooth": ([_vp, _i, _vp, _vp, _i], _i),
    "msp_stage_bilu": ([_vp, _vp, _vp], _i),
    "msp_stage_level_info": ([_vp, _i, C.POINTER(_i), C.POINTER(_ll), C.POINTER(_i),
                              C.POINTER(_i)], _i),
    "msp_stage_get_level": ([_vp, _i, _vp, _vp, _vp, _vp, _vp], _i),
    "msp_stage_get_level_f32": ([_vp, _i, _vp], _i),
    "msp_stage_get_omega": ([_vp, _vp], _i),
    "msp_stage_get_bilu": ([_vp, _vp, _vp], _i),
    "msp_stage_get_bilu_f32": ([_vp, _vp, _vp], _i),
    "msp_stage_repeat": ([_vp, _i, _i, _vp, _vp], _i),
    "msp_stage_get_nstage": ([_vp, _vp, _vp], _i),
    "msp_stage_set_timing": ([_vp, _i], _i),
    "msp_stage_get_timing": ([_vp, C.POINTER(_d), C.POINTER(_i)], _i),
}
STAGE_SPMV, STAGE_GS0, STAGE_PRECOND, STAGE_BILU, STAGE_VCYCLE, STAGE_COARSE, STAGE_TRI_SWEEP = \
    range(7)

_LIB = None
_LOCK = threading.Lock()


class MspError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        super().__init__(f"libmsp {where}: {STATUS.get(code, code)}")


def lib():
    """Load libmsp.so (raises if it has not been built)."""
    global _LIB
    with _LOCK:
        if _LIB is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                                   "paper_2208_08594_amd/build.py (no CPU fallback exists)")
            L = C.CDLL(LIB_PATH)
            for name, (args, res) in SIGNATURES.items():
                fn = getattr(L, name)
                fn.argtypes = args
                fn.restype = res
            _LIB = L
    return _LIB


def status_string(code: int) -> str:
    return lib().msp_status_string(code).decode()


def _check(code, where):
    if code < 0:
        raise MspError(code, where)
    return code


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class _TorchAllocator:
    """Device memory for the library from torch's caching allocator."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device
        self.live = {}
        self.lock = threading.Lock()
        self.alloc_fn = ALLOC_FN(self._alloc)
        self.free_fn = FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=self.device)
        except Exception:
            return None
        ptr = t.data_ptr()
        with self.lock:
            self.live[ptr] = t
        return ptr

    def _free(self, ptr, user):
        with self.lock:
            self.live.pop(ptr, None)

    @property
    def bytes_live(self):
        with self.lock:
            return sum(t.numel() for t in self.live.values())


class Solver:
    """One libmsp context: setup(A^(i)) then solve(rhs, x) per Newton step.

    Tensors are torch CUDA tensors on the context's device (int32 pattern,
    float64 values); host numpy arrays are uploaded for convenience.
    """

    def __init__(self, mu=0, restart=30, max_iter=1000, max_coarse=10000, precond_fp32=False,
                 bilu_order=1, stream=None, device=None, torch_allocator=True, use_graphs=True,
                 smoother=0, jacobi_weight=1.0, nu_pre=1, nu_post=1, full_smoother=0,
                 n_stage=0, host_chain=False):
        import torch
        self.torch = torch
        dev = torch.device("cuda") if device is None else torch.device(device)
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._lib = lib()
        opt = MspOptions()
        _check(self._lib.msp_default_options(C.byref(opt)), "default_options")
        opt.mu, opt.restart, opt.max_iter, opt.max_coarse = mu, restart, max_iter, max_coarse
        opt.precond_fp32 = 1 if precond_fp32 else 0
        opt.bilu_order = int(bilu_order)
        opt.use_graphs = 1 if use_graphs else 0
        opt.smoother, opt.jacobi_weight = int(smoother), float(jacobi_weight)
        opt.nu_pre, opt.nu_post, opt.full_smoother = int(nu_pre), int(nu_post), int(full_smoother)
        opt.n_stage = int(n_stage)
        opt.host_chain = 1 if host_chain else 0
        opt.stream = C.c_void_p(self.stream.cuda_stream)
        self._alloc = None
        if torch_allocator:
            self._alloc = _TorchAllocator(self.device)
            opt.dev_alloc = self._alloc.alloc_fn
            opt.dev_free = self._alloc.free_fn
        self._opt = opt
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(self._lib.msp_create(C.byref(h), C.byref(opt)), "create")
        self.h = h
        self.n = self.b = self.p = None
        self.precond_fp32 = bool(precond_fp32)
        self.bilu_order = int(bilu_order)

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self._lib.msp_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- helpers ----------------------------------------------------------
    def _dev(self, a, dtype):
        t = self.torch
        if isinstance(a, t.Tensor):
            if a.device != self.device or a.dtype != dtype or not a.is_contiguous():
                a = a.to(device=self.device, dtype=dtype).contiguous()
            return a
        return t.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=self.device)

    # -- path -----------------------------------------------------------
    def setup(self, sys=None, *, n=None, b=None, p=0, row_ptr=None, col_ind=None, vals=None):
        """msp_setup on one Jacobian; returns True if the preconditioner was rebuilt."""
        t = self.torch
        if sys is not None:
            n, b, p, row_ptr, col_ind, vals = sys.n, sys.b, sys.p, sys.row_ptr, sys.col_ind, sys.vals
        rp = self._dev(row_ptr, t.int32)
        ci = self._dev(col_ind, t.int32)
        va = self._dev(vals, t.float64).reshape(-1)
        with t.cuda.device(self.device):
            _check(self._lib.msp_setup(self.h, int(n), int(b), int(p), _ptr(rp), _ptr(ci),
                                       _ptr(va), int(ci.numel())), "setup")
        self.n, self.b, self.p = int(n), int(b), int(p)
        return self.info()["rebuilt"]

    def solve(self, rhs, x=None, rtol=1e-6, noalloc=False):
        """msp_solve (msp_solve_noalloc if noalloc); returns (x, info dict).
        x is updated in place if given."""
        t = self.torch
        rhs = self._dev(rhs, t.float64)
        if x is None:
            x = t.zeros_like(rhs)
        info = MspInfo()
        fn = self._lib.msp_solve_noalloc if noalloc else self._lib.msp_solve
        with t.cuda.device(self.device):
            code = fn(self.h, _ptr(rhs), _ptr(x), float(rtol), C.byref(info))
        _check(code, "solve_noalloc" if noalloc else "solve")
        d = info.as_dict()
        d["status"] = code
        return x, d

    def info(self):
        info = MspInfo()
        _check(self._lib.msp_get_info(self.h, C.byref(info)), "info")
        return info.as_dict()

    # -- stage entry points -----------------------------------------------
    def _stage2(self, name, a, out_len):
        t = self.torch
        a = self._dev(a, t.float64)
        out = t.empty(out_len, dtype=t.float64, device=self.device)
        with t.cuda.device(self.device):
            _check(getattr(self._lib, name)(self.h, _ptr(a), _ptr(out)), name)
        return out

    def spmv(self, x):
        return self._stage2("msp_stage_spmv", x, self.n * self.b)

    def apply(self, v):
        return self._stage2("msp_stage_precond", v, self.n * self.b)

    def vcycle(self, f):
        return self._stage2("msp_stage_vcycle", f, self.n)

    def bilu_apply(self, r):
        return self._stage2("msp_stage_bilu", r, self.n * self.b)

    def smooth(self, level, f, x, forward=True):
        t = self.torch
        f = self._dev(f, t.float64)
        x = self._dev(x, t.float64).clone()
        with t.cuda.device(self.device):
            _check(self._lib.msp_stage_smooth(self.h, int(level), _ptr(f), _ptr(x),
                                              1 if forward else 0), "smooth")
        return x

    def repeat(self, stage, reps, inp=None, out=None):
        """msp_stage_repeat: reps back-to-back launches of one stage (for timing)."""
        p = lambda t: None if t is None else _ptr(t)
        with self.torch.cuda.device(self.device):
            _check(self._lib.msp_stage_repeat(self.h, int(stage), int(reps), p(inp), p(out)),
                   "repeat")

    def set_timing(self, on=True):
        """msp_stage_set_timing: HIP events around the parts of every Arnoldi step."""
        _check(self._lib.msp_stage_set_timing(self.h, 1 if on else 0), "set_timing")

    def timing(self):
        """msp_stage_get_timing of the last solve: {part: (summed ms, steps)}."""
        ms = (C.c_double * 3)()
        calls = (C.c_int * 3)()
        _check(self._lib.msp_stage_get_timing(self.h, ms, calls), "get_timing")
        return {k: (ms[i], calls[i]) for i, k in enumerate(("spmv", "apply", "gram_schmidt"))}

    @property
    def nlevels(self):
        return self.info()["n_levels"]

    def level(self, l):
        n = C.c_int()
        nnz = C.c_longlong()
        g = C.c_int()
        nn = C.c_int()
        _check(self._lib.msp_stage_level_info(self.h, l, C.byref(n), C.byref(nnz), C.byref(g),
                                              C.byref(nn)), "level_info")
        n, nnz = n.value, nnz.value
        last = nn.value == 0
        rp = np.zeros(n + 1, dtype=np.int32)
        ci = np.zeros(nnz, dtype=np.int32)
        val = np.zeros(nnz)
        color = None if last else np.zeros(n, dtype=np.int32)
        agg = None if last else np.zeros(n, dtype=np.int32)
        p = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
        _check(self._lib.msp_stage_get_level(self.h, l, p(rp), p(ci), p(val), p(color), p(agg)),
               "get_level")
        return dict(n=n, row_ptr=rp, col_ind=ci, val=val, color=color, agg=agg,
                    ncolors=g.value, nc=nn.value)

    def level_f32(self, l):
        nnz = C.c_longlong()
        _check(self._lib.msp_stage_level_info(self.h, l, None, C.byref(nnz), None, None),
               "level_info")
        out = np.zeros(nnz.value, dtype=np.float32)
        _check(self._lib.msp_stage_get_level_f32(self.h, l, out.ctypes.data_as(C.c_void_p)),
               "get_level_f32")
        return out

    def omega(self):
        out = np.zeros(self.n * self.b)
        _check(self._lib.msp_stage_get_omega(self.h, out.ctypes.data_as(C.c_void_p)), "omega")
        return out.reshape(self.n, self.b)

    def nstage(self):
        """(Dn, Ann) of the concentration stage (FP64, host)."""
        m = self.b - 1
        nnzb = int(self.level(0)["row_ptr"][-1])
        Dn = np.zeros(self.n * m * self.b)
        Ann = np.zeros(nnzb * m * m)
        _check(self._lib.msp_stage_get_nstage(self.h, Dn.ctypes.data_as(C.c_void_p),
                                              Ann.ctypes.data_as(C.c_void_p)), "nstage")
        return Dn.reshape(self.n, m, self.b), Ann.reshape(nnzb, m, m)

    def bilu(self, f32=False):
        nnzb = int(self.level(0)["row_ptr"][-1])
        dt = np.float32 if f32 else np.float64
        F = np.zeros(nnzb * self.b * self.b, dtype=dt)
        D = np.zeros(self.n * self.b * self.b, dtype=dt)
        fn = self._lib.msp_stage_get_bilu_f32 if f32 else self._lib.msp_stage_get_bilu
        _check(fn(self.h, F.ctypes.data_as(C.c_void_p), D.ctypes.data_as(C.c_void_p)), "bilu")
        return F.reshape(-1, self.b, self.b), D.reshape(self.n, self.b, self.b)


def solve_batch(solvers, rhs, xs, rtol=1e-6):
    """msp_solve_batch over several Solver contexts (same device): rhs and xs
    are lists of device float64 tensors (xs updated in place); returns the
    list of info dicts."""
    import torch
    k = len(solvers)
    if not (k == len(rhs) == len(xs)) or k == 0:
        raise ValueError("solve_batch needs equally many solvers, rhs and x")
    ctx = (C.c_void_p * k)(*[s.h.value for s in solvers])
    rp = (C.c_void_p * k)(*[t.data_ptr() for t in rhs])
    xp = (C.c_void_p * k)(*[t.data_ptr() for t in xs])
    infos = (MspInfo * k)()
    with torch.cuda.device(solvers[0].device):
        code = lib().msp_solve_batch(C.cast(ctx, C.c_void_p), k, C.cast(rp, C.c_void_p),
                                     C.cast(xp, C.c_void_p), float(rtol),
                                     C.cast(infos, C.c_void_p))
    _check(code, "solve_batch")
    out = []
    for i in range(k):
        d = infos[i].as_dict()
        out.append(d)
    return out


def footprint(n, nnzb, b, mu=0, restart=30, max_coarse=10000, precond_fp32=False):
    opt = MspOptions()
    lib().msp_default_options(C.byref(opt))
    opt.restart, opt.max_coarse, opt.precond_fp32, opt.mu = restart, max_coarse, int(precond_fp32), mu
    out = C.c_size_t()
    _check(lib().msp_footprint(int(n), int(nnzb), int(b), C.byref(opt), C.byref(out)), "footprint")
    return int(out.value)
