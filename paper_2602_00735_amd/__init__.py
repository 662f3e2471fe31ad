"""RAS-PML GMRES hot path for MI355X: Python binding of libras_pml.so.

Thin ctypes marshalling over the C ABI in include/ras_pml.h: the functions
here have the ABI's names and pass device pointers of torch tensors
(complex128 on the GPU) and the current HIP stream.  Every step of the
method runs in the HIP library; there is no Python or CPU fallback, and
importing a function that needs the library raises if it is not built.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libras_pml.so")

RAS_OK, RAS_EINVAL, RAS_ENOMEM, RAS_EHIP, RAS_EZEROPIVOT = 0, 1, 2, 3, 4
RAS_ENONFINITE, RAS_ENOTCONV, RAS_EBREAKDOWN, RAS_ENOTSUP = 5, 6, 7, 8
RAS_BC_IMP, RAS_BC_DRCH = 0, 1
RAS_POU_LINEAR, RAS_POU_BOOLEAN = 0, 1
RAS_MIXED, RAS_FP64 = 0, 1
RAS_FLAG_TIMING = 1
RAS_FLAG_UNFUSED_ARNOLDI = 2
RAS_FLAG_GRAPH_STEPS = 4
RAS_KNOB_SOLVE_DEEP = 0
RAS_KNOB_SOLVE_QUEUE = 1
RAS_KNOB_ARNOLDI = 2
RAS_DESC_INTS = 24
RAS_WIDTH_RULE = -1


class RasPmlError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (status %d): %s" % (_STATUS.get(status, "?"), status, msg))
        self.status = status


_STATUS = {0: "RAS_OK", 1: "RAS_EINVAL", 2: "RAS_ENOMEM", 3: "RAS_EHIP", 4: "RAS_EZEROPIVOT",
           5: "RAS_ENONFINITE", 6: "RAS_ENOTCONV", 7: "RAS_EBREAKDOWN", 8: "RAS_ENOTSUP"}


class Opts(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("global_pml", ctypes.c_int), ("bc", ctypes.c_int),
                ("pou", ctypes.c_int), ("precision", ctypes.c_int), ("flags", ctypes.c_int),
                ("tune_cache", ctypes.c_char_p), ("width_c_delta", ctypes.c_double),
                ("width_c_kappa", ctypes.c_double), ("width_k0", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("n_solve", ctypes.c_longlong), ("solve_ms", ctypes.c_double),
                ("n_sum", ctypes.c_longlong), ("sum_ms", ctypes.c_double),
                ("n_spmv", ctypes.c_longlong), ("spmv_ms", ctypes.c_double),
                ("n_mgs", ctypes.c_longlong), ("mgs_ms", ctypes.c_double),
                ("n_givens", ctypes.c_longlong), ("givens_ms", ctypes.c_double),
                ("setup_assemble_ms", ctypes.c_double), ("setup_factor_ms", ctypes.c_double),
                ("solve_bytes", ctypes.c_double), ("factor_bytes", ctypes.c_double),
                ("alloc_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# (name, restype, argtypes) of every exported symbol
_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_LL = ctypes.c_longlong
_IP = ctypes.POINTER(ctypes.c_int)
_DP = ctypes.POINTER(ctypes.c_double)
_LLP = ctypes.POINTER(ctypes.c_longlong)
SYMBOLS = [
    ("ras_pml_default_opts", None, [ctypes.POINTER(Opts)]),
    ("ras_pml_plan", _I, [_D, _D, _IP, _IP, _I, _I, ctypes.POINTER(Opts), _IP, _IP, _I]),
    ("ras_pml_plan_error", ctypes.c_char_p, []),
    ("ras_pml_setup", _I, [_D, _D, _IP, _IP, _I, _I, ctypes.POINTER(Opts), _P,
                           ctypes.POINTER(_P)]),
    ("ras_pml_setup_batch", _I, [_I, _DP, _DP, _IP, _IP, _IP, _IP, ctypes.POINTER(Opts), _P,
                                 ctypes.POINTER(_P)]),
    ("ras_pml_destroy", None, [_P]),
    ("ras_pml_num_dofs", _I, [_P, _LLP]),
    ("ras_pml_num_problems", _I, [_P, _IP]),
    ("ras_pml_problem_offset", _I, [_P, _I, _LLP, _LLP]),
    ("ras_pml_num_subdomains", _I, [_P, _IP]),
    ("ras_pml_num_local", _I, [_P, _LLP]),
    ("ras_pml_subdomain_desc", _I, [_P, _IP, _I]),
    ("ras_pml_rhs", _I, [_P, _P, _P, _P]),
    ("ras_pml_spmv", _I, [_P, _P, _P, _P]),
    ("ras_pml_apply", _I, [_P, _P, _P, _P]),
    ("ras_pml_local_solve", _I, [_P, _P, _P, _P]),
    ("gmres_solve", _I, [_P, _P, _P, _D, _I, _I, _IP, _DP, _DP, _P]),
    ("gmres_solve_batch", _I, [_P, _P, _P, _DP, _I, _I, _IP, _DP, _DP, _P]),
    ("ras_pml_richardson", _I, [_P, _P, _P, _D, _I, _IP, _DP, _DP, _P]),
    ("ras_pml_richardson_noalloc", _I, [_P, _P, _P, _D, _I, _IP, _DP, _DP, _P]),
    ("ras_pml_set_knob", _I, [_P, _I, _I]),
    ("ras_pml_tune_report", _I, [_P, _DP, _I, _IP]),
    ("ras_pml_get_knob", _I, [_P, _I, _IP]),
    ("ras_pml_width_rule", _I, [_D, _D, _D, _D, _IP]),
    ("ras_pml_batch_result", _I, [_P, _I, _IP, _DP, _IP]),
    ("ras_pml_wsnet_create", _I, [_I, _IP, _I, ctypes.POINTER(_P)]),
    ("ras_pml_wsnet_destroy", None, [_P]),
    ("ras_pml_wsnet_num_weights", _I, [_P, _LLP]),
    ("ras_pml_wsnet_set_weights", _I, [_P, _P, _LL]),
    ("ras_pml_wsnet_get_weights", _I, [_P, _P, _LL]),
    ("ras_pml_wsnet_forward", _I, [_P, _P, _I, _P, _P]),
    ("ras_pml_wsnet_gradient", _I, [_P, _P, _P, _I, _DP, _P, _P]),
    ("ras_pml_wsnet_adam", _I, [_P, ctypes.c_float, _P]),
    ("ras_pml_wsnet_train_step", _I, [_P, _P, _P, _I, ctypes.c_float, _DP, _P]),
    ("ras_pml_wsnet_last_error", ctypes.c_char_p, [_P]),
    ("ras_pml_grid_sample", _I, [_P, _P, _D, _P, _P]),
    ("ras_pml_warm_start", _I, [_P, _P, _P, _P, _P, _D, _IP, _P]),
    ("ras_pml_export_stencil", _I, [_P, _P]),
    ("ras_pml_export_local", _I, [_P, _I, _P]),
    ("ras_pml_export_factor", _I, [_P, _I, _P, _LL]),
    ("ras_pml_get_stats", _I, [_P, ctypes.POINTER(Stats)]),
    ("ras_pml_reset_stats", _I, [_P]),
    ("ras_pml_empty_cache", _I, [ctypes.POINTER(ctypes.c_longlong)]),
    ("ras_pml_set_cache_limit", _I, [ctypes.c_longlong]),
    ("ras_pml_fill_idle_cache", _I, [_I]),
    ("ras_pml_cache_info", _I, [ctypes.POINTER(ctypes.c_longlong),
                                ctypes.POINTER(ctypes.c_longlong)]),
    ("ras_pml_autotune", _I, [_P, ctypes.c_char_p, _P]),
    ("ras_pml_tuning", _I, [_P, _IP, _IP, _I, _IP]),
    ("ras_pml_strerror", ctypes.c_char_p, [_I]),
    ("ras_pml_last_error", ctypes.c_char_p, [_P]),
    ("ras_pml_shutdown", _I, []),
]

_lib = None


def lib():
    """Load libras_pml.so; raise (never fall back) if it is not built.

    torch is imported first when it is installed: it carries its own HIP
    runtime, and the library must bind to that same runtime (a second HIP
    runtime in the process would not see the GPU that torch holds)."""
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError("libras_pml.so is not built; run "
                              "`python -m paper_2602_00735_amd.build` (HIP for gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SYMBOLS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        import atexit
        atexit.register(_shutdown)
    return _lib


def _shutdown():
    """Exit hook: the library's streams and idle device blocks go before
    the HIP runtime (and any profiler's tool library) is torn down."""
    if _lib is not None:
        _lib.ras_pml_shutdown()


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().ras_pml_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "tune_cache" and isinstance(v, (str, os.PathLike)):
            v = os.fsencode(v)
        setattr(o, k, v)
    return o


def _i2(a):
    return (ctypes.c_int * 2)(int(a[0]), int(a[1]))


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _check_vec(t, n, name):
    import torch
    if t.dtype != torch.complex128 or not t.is_cuda or not t.is_contiguous() or t.numel() != n:
        raise ValueError("%s must be a contiguous complex128 CUDA tensor of %d values" % (name, n))


def ras_pml_plan(k, h, grid, subdomains, overlap, pml_width, opts=None):
    """Host-only planning; returns the descriptor table as a list of lists."""
    L = lib()
    o = opts if opts is not None else default_opts()
    ns = ctypes.c_int(0)
    rc = L.ras_pml_plan(k, h, _i2(grid), _i2(subdomains), overlap, pml_width, ctypes.byref(o),
                        ctypes.byref(ns), None, 0)
    if rc != RAS_OK:
        raise RasPmlError(rc, L.ras_pml_plan_error().decode())
    buf = (ctypes.c_int * (ns.value * RAS_DESC_INTS))()
    rc = L.ras_pml_plan(k, h, _i2(grid), _i2(subdomains), overlap, pml_width, ctypes.byref(o),
                        ctypes.byref(ns), buf, ns.value)
    if rc != RAS_OK:
        raise RasPmlError(rc, L.ras_pml_plan_error().decode())
    return [list(buf[i * RAS_DESC_INTS:(i + 1) * RAS_DESC_INTS]) for i in range(ns.value)]


class Handle:
    """Owns a ras_pml_t; destroyed with the object or by ras_pml_destroy."""

    def __init__(self, ptr):
        self.ptr = ptr
        L = lib()
        n = ctypes.c_longlong(0)
        L.ras_pml_num_dofs(self.ptr, ctypes.byref(n))
        self.ndof = n.value
        ns = ctypes.c_int(0)
        L.ras_pml_num_subdomains(self.ptr, ctypes.byref(ns))
        self.nsub = ns.value
        nl = ctypes.c_longlong(0)
        L.ras_pml_num_local(self.ptr, ctypes.byref(nl))
        self.nloc = nl.value
        npb = ctypes.c_int(0)
        L.ras_pml_num_problems(self.ptr, ctypes.byref(npb))
        self.nprob = npb.value

    def _raise(self, rc):
        raise RasPmlError(rc, lib().ras_pml_last_error(self.ptr).decode())

    def close(self):
        if self.ptr:
            lib().ras_pml_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def grid_side(self):
        """Interior grid nodes per side (single-problem handles): N_c - 2G."""
        import math
        n1 = math.isqrt(self.ndof)
        return n1 + 1 - 2 * self.desc()[0][22]

    def problem_offset(self, p):
        off, n = ctypes.c_longlong(0), ctypes.c_longlong(0)
        rc = lib().ras_pml_problem_offset(self.ptr, p, ctypes.byref(off), ctypes.byref(n))
        if rc:
            self._raise(rc)
        return off.value, n.value

    def desc(self):
        buf = (ctypes.c_int * (self.nsub * RAS_DESC_INTS))()
        rc = lib().ras_pml_subdomain_desc(self.ptr, buf, self.nsub)
        if rc:
            self._raise(rc)
        return [list(buf[i * RAS_DESC_INTS:(i + 1) * RAS_DESC_INTS]) for i in range(self.nsub)]


def ras_pml_setup(k, h, grid, subdomains, overlap, pml_width, opts=None, stream=None) -> Handle:
    L = lib()
    o = opts if opts is not None else default_opts()
    out = ctypes.c_void_p()
    rc = L.ras_pml_setup(k, h, _i2(grid), _i2(subdomains), overlap, pml_width, ctypes.byref(o),
                         _stream(stream), ctypes.byref(out))
    if rc != RAS_OK:
        raise RasPmlError(rc, L.ras_pml_plan_error().decode())
    return Handle(out)


def ras_pml_setup_batch(ks, hs, grids, subdomains, overlaps, pml_widths, opts=None,
                        stream=None) -> Handle:
    L = lib()
    n = len(ks)
    o = opts if opts is not None else default_opts()
    D = ctypes.c_double * n
    I = ctypes.c_int * n
    I2 = ctypes.c_int * (2 * n)
    g = [int(x) for gg in grids for x in gg]
    s = [int(x) for ss in subdomains for x in ss]
    out = ctypes.c_void_p()
    rc = L.ras_pml_setup_batch(n, D(*ks), D(*hs), I2(*g), I2(*s), I(*overlaps), I(*pml_widths),
                               ctypes.byref(o), _stream(stream), ctypes.byref(out))
    if rc != RAS_OK:
        raise RasPmlError(rc, L.ras_pml_plan_error().decode())
    return Handle(out)


def ras_pml_destroy(H: Handle):
    H.close()


def ras_pml_rhs(H: Handle, f, b, stream=None):
    _check_vec(f, H.ndof, "f")
    _check_vec(b, H.ndof, "b")
    rc = lib().ras_pml_rhs(H.ptr, _ptr(f), _ptr(b), _stream(stream))
    if rc:
        H._raise(rc)


def ras_pml_spmv(H: Handle, x, y, stream=None):
    _check_vec(x, H.ndof, "x")
    _check_vec(y, H.ndof, "y")
    rc = lib().ras_pml_spmv(H.ptr, _ptr(x), _ptr(y), _stream(stream))
    if rc:
        H._raise(rc)


def ras_pml_apply(H: Handle, v, z, stream=None):
    _check_vec(v, H.ndof, "v")
    _check_vec(z, H.ndof, "z")
    rc = lib().ras_pml_apply(H.ptr, _ptr(v), _ptr(z), _stream(stream))
    if rc:
        H._raise(rc)


def ras_pml_local_solve(H: Handle, v, xloc, stream=None):
    """xloc=None: the batched band solve alone (result kept in the handle)."""
    _check_vec(v, H.ndof, "v")
    if xloc is not None:
        _check_vec(xloc, H.nloc, "xloc")
    rc = lib().ras_pml_local_solve(H.ptr, _ptr(v), None if xloc is None else _ptr(xloc),
                                   _stream(stream))
    if rc:
        H._raise(rc)


def gmres_solve(H: Handle, b, x, rtol=1e-6, restart=100, maxit=500, stream=None, check=True):
    """Returns (status, iters, relres, hist).  Raises on errors other than
    RAS_ENOTCONV / RAS_EBREAKDOWN unless check=False."""
    import numpy as np
    _check_vec(b, H.ndof, "b")
    _check_vec(x, H.ndof, "x")
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    hist = np.zeros(maxit + 1)
    rc = lib().gmres_solve(H.ptr, _ptr(b), _ptr(x), rtol, restart, maxit, ctypes.byref(it),
                           ctypes.byref(rr), hist.ctypes.data_as(_DP), _stream(stream))
    if check and rc not in (RAS_OK, RAS_ENOTCONV, RAS_EBREAKDOWN):
        H._raise(rc)
    return rc, it.value, rr.value, hist[:it.value + 1]


def ras_pml_richardson(H: Handle, b, x, rtol=1e-6, maxit=500, stream=None, check=True):
    """Algorithm 1 iteration.  Returns (status, iters, relres, hist).  Raises
    on errors other than RAS_ENOTCONV unless check=False."""
    import numpy as np
    _check_vec(b, H.ndof, "b")
    _check_vec(x, H.ndof, "x")
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    hist = np.zeros(maxit + 1)
    rc = lib().ras_pml_richardson(H.ptr, _ptr(b), _ptr(x), rtol, maxit, ctypes.byref(it),
                                  ctypes.byref(rr), hist.ctypes.data_as(_DP), _stream(stream))
    if check and rc not in (RAS_OK, RAS_ENOTCONV):
        H._raise(rc)
    return rc, it.value, rr.value, hist[:it.value + 1]


def ras_pml_richardson_noalloc(H: Handle, b, x, rtol=1e-6, maxit=500, stream=None, check=True):
    """ras_pml_richardson with every buffer in the library's static scratch
    (no device allocation).  Returns (status, iters, relres, hist)."""
    import numpy as np
    _check_vec(b, H.ndof, "b")
    _check_vec(x, H.ndof, "x")
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    hist = np.zeros(maxit + 1)
    rc = lib().ras_pml_richardson_noalloc(H.ptr, _ptr(b), _ptr(x), rtol, maxit, ctypes.byref(it),
                                          ctypes.byref(rr), hist.ctypes.data_as(_DP),
                                          _stream(stream))
    if check and rc not in (RAS_OK, RAS_ENOTCONV):
        H._raise(rc)
    return rc, it.value, rr.value, hist[:it.value + 1]


def ras_pml_set_knob(H: Handle, knob, value):
    """Kernel variant choice of a handle (RAS_KNOB_*)."""
    rc = lib().ras_pml_set_knob(H.ptr, int(knob), int(value))
    if rc:
        H._raise(rc)


def ras_pml_get_knob(H: Handle, knob):
    v = ctypes.c_int(0)
    rc = lib().ras_pml_get_knob(H.ptr, int(knob), ctypes.byref(v))
    if rc:
        H._raise(rc)
    return v.value


def ras_pml_width_rule(k, h, C, k0=150.0):
    """Section 3 (iii) width in mesh cells (host only)."""
    cells = ctypes.c_int(0)
    rc = lib().ras_pml_width_rule(float(k), float(h), float(C), float(k0), ctypes.byref(cells))
    if rc:
        raise ValueError(lib().ras_pml_plan_error().decode())
    return cells.value


def gmres_solve_batch(H: Handle, b, x, rtols, restart=100, maxit=500, stream=None, check=True):
    """One tolerance per problem.  Returns (status, iters per problem, relres
    per problem, hist of the worst problem)."""
    import numpy as np
    _check_vec(b, H.ndof, "b")
    _check_vec(x, H.ndof, "x")
    r = np.ascontiguousarray(rtols, dtype=np.float64)
    if r.size != H.nprob:
        raise ValueError("one tolerance per problem (%d)" % H.nprob)
    it = np.zeros(H.nprob, dtype=np.int32)
    rr = np.zeros(H.nprob)
    hist = np.full(maxit + 1, np.nan)
    rc = lib().gmres_solve_batch(H.ptr, _ptr(b), _ptr(x), r.ctypes.data_as(_DP), restart, maxit,
                                 it.ctypes.data_as(_IP), rr.ctypes.data_as(_DP),
                                 hist.ctypes.data_as(_DP), _stream(stream))
    if check and rc not in (RAS_OK, RAS_ENOTCONV, RAS_EBREAKDOWN):
        H._raise(rc)
    return rc, it.tolist(), rr.tolist(), hist[~np.isnan(hist)]


def ras_pml_batch_result(H: Handle, p):
    it, rr, cv = ctypes.c_int(0), ctypes.c_double(0.0), ctypes.c_int(0)
    rc = lib().ras_pml_batch_result(H.ptr, p, ctypes.byref(it), ctypes.byref(rr), ctypes.byref(cv))
    if rc:
        H._raise(rc)
    return it.value, rr.value, bool(cv.value)


def ras_pml_export_stencil(H: Handle):
    import numpy as np
    out = np.zeros(4 * H.ndof, dtype=np.complex128)
    rc = lib().ras_pml_export_stencil(H.ptr, out.ctypes.data_as(_P))
    if rc:
        H._raise(rc)
    return out.reshape(4, H.ndof)


def ras_pml_export_local(H: Handle, j, n_local):
    import numpy as np
    out = np.zeros(4 * n_local, dtype=np.complex128)
    rc = lib().ras_pml_export_local(H.ptr, j, out.ctypes.data_as(_P))
    if rc:
        H._raise(rc)
    return out.reshape(n_local, 4)


def ras_pml_export_factor(H: Handle, j, npad, W):
    """Returns (L by columns (npad, W), L by rows (npad, W), D^{-1} (npad,)),
    both copies in slot order."""
    import numpy as np
    cnt = npad * (2 * W + 1)
    out = np.zeros(cnt, dtype=np.complex128)
    rc = lib().ras_pml_export_factor(H.ptr, j, out.ctypes.data_as(_P), cnt)
    if rc:
        H._raise(rc)
    return (out[:npad * W].reshape(npad, W), out[npad * W:2 * npad * W].reshape(npad, W),
            out[2 * npad * W:])


def ras_pml_get_stats(H: Handle) -> dict:
    s = Stats()
    rc = lib().ras_pml_get_stats(H.ptr, ctypes.byref(s))
    if rc:
        H._raise(rc)
    return s.as_dict()


def ras_pml_empty_cache() -> int:
    """Hand the idle cached device blocks back to the driver; returns their bytes."""
    n = ctypes.c_longlong(0)
    lib().ras_pml_empty_cache(ctypes.byref(n))
    return n.value


def ras_pml_set_cache_limit(nbytes: int):
    lib().ras_pml_set_cache_limit(int(nbytes))


def ras_pml_fill_idle_cache(byte: int):
    rc = lib().ras_pml_fill_idle_cache(int(byte))
    if rc != RAS_OK:
        raise RasPmlError(rc, "filling the idle device blocks failed")


def ras_pml_cache_info():
    """(idle cached bytes, handed-out bytes)."""
    a, b = ctypes.c_longlong(0), ctypes.c_longlong(0)
    lib().ras_pml_cache_info(ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def ras_pml_reset_stats(H: Handle):
    rc = lib().ras_pml_reset_stats(H.ptr)
    if rc:
        H._raise(rc)


def ras_pml_autotune(H: Handle, cache_path=None, stream=None):
    path = None if cache_path is None else os.fsencode(cache_path)
    rc = lib().ras_pml_autotune(H.ptr, path, _stream(stream))
    if rc:
        H._raise(rc)


def ras_pml_tuning(H: Handle) -> dict:
    """{"solve_deep": bool, "solve_queue": bool, "ldlt": [(tiles, subdomains, variant), ...]}
    (variant 0: matrix-core kernel, 1: the same held to the occupancy register
    budget, 2: one-column vector-ALU kernel)"""
    deep, ng = ctypes.c_int(0), ctypes.c_int(0)
    cap = 16
    buf = (ctypes.c_int * (3 * cap))()
    rc = lib().ras_pml_tuning(H.ptr, ctypes.byref(deep), buf, cap, ctypes.byref(ng))
    if rc:
        H._raise(rc)
    groups = [(buf[3 * i], buf[3 * i + 1], int(buf[3 * i + 2])) for i in range(min(cap, ng.value))]
    return {"solve_deep": bool(deep.value),
            "solve_queue": bool(ras_pml_get_knob(H, RAS_KNOB_SOLVE_QUEUE)),
            "arnoldi": ras_pml_get_knob(H, RAS_KNOB_ARNOLDI), "ldlt": groups}


def ras_pml_tune_report(H: Handle) -> dict:
    """Timings (ms) of the last autotune: {"ldlt": [(tiles, [t0, t1, t2]), ...],
    "solve": {"hardware_half": t, "hardware_deep": t, "queue_half": t, "queue_deep": t}}
    (None where not measured)."""
    n = ctypes.c_int(0)
    buf = (ctypes.c_double * 64)()
    rc = lib().ras_pml_tune_report(H.ptr, buf, 64, ctypes.byref(n))
    if rc:
        H._raise(rc)
    vals = [None if v >= 1e29 else round(v, 4) for v in buf[:min(64, n.value)]]
    if not vals:
        return {}
    groups = ras_pml_tuning(H)["ldlt"]
    ldlt = [(g[0], vals[3 * i:3 * i + 3]) for i, g in enumerate(groups)]
    sv = vals[3 * len(groups):3 * len(groups) + 4]
    av = vals[3 * len(groups) + 4:3 * len(groups) + 7]
    return {"ldlt": ldlt, "solve": dict(zip(("hardware_half", "hardware_deep", "queue_half",
                                             "queue_deep"), sv)),
            "arnoldi": dict(zip(("e8", "e16", "lean_e12"), av))}


def ras_pml_strerror(status: int) -> str:
    return lib().ras_pml_strerror(status).decode()


# ---------------------------------------------------------------- learned warm start
WS_LAYERS = ("e0", "e1", "e2", "e3", "e4", "d3", "d2", "d1", "d0", "head")


def ws_shapes(channels):
    """(cin, cout) of every convolution, in the order of the weights."""
    c0, c1, c2, c3, c4 = channels
    return [(2, c0), (c0, c1), (c1, c2), (c2, c3), (c3, c4), (c4, c2), (c2, c1), (c1, c0),
            (c0, c0), (c0, 2)]


class WSNet:
    """The warm-start encoder-decoder (all compute in the library's kernels)."""

    def __init__(self, grid, channels, batch_max):
        self.grid, self.channels, self.batch_max = int(grid), tuple(channels), int(batch_max)
        ptr = _P()
        rc = lib().ras_pml_wsnet_create(self.grid, (ctypes.c_int * 5)(*self.channels),
                                        self.batch_max, ctypes.byref(ptr))
        if rc:
            raise RasPmlError(rc, "ras_pml_wsnet_create: %s" % _STATUS.get(rc, rc))
        self.ptr = ptr
        n = _LL(0)
        lib().ras_pml_wsnet_num_weights(self.ptr, ctypes.byref(n))
        self.nweights = n.value

    def _check(self, rc):
        if rc:
            msg = lib().ras_pml_wsnet_last_error(self.ptr).decode()
            raise RasPmlError(rc, "%s: %s" % (_STATUS.get(rc, rc), msg))

    def set_weights(self, flat):
        import numpy as np
        w = np.ascontiguousarray(flat, dtype=np.float32)
        assert w.size == self.nweights
        self._check(lib().ras_pml_wsnet_set_weights(self.ptr, w.ctypes.data_as(_P), w.size))

    def get_weights(self):
        import numpy as np
        w = np.zeros(self.nweights, dtype=np.float32)
        self._check(lib().ras_pml_wsnet_get_weights(self.ptr, w.ctypes.data_as(_P), w.size))
        return w

    def _grid(self, t, name):
        import torch
        if (t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.dim() != 4
                or tuple(t.shape[1:]) != (self.grid, self.grid, 2) or t.shape[0] > self.batch_max):
            raise ValueError("%s must be a contiguous float32 CUDA tensor (B, %d, %d, 2), B <= %d"
                             % (name, self.grid, self.grid, self.batch_max))

    def forward(self, x, y=None, stream=None):
        import torch
        self._grid(x, "x")
        if y is None:
            y = torch.empty_like(x)
        self._grid(y, "y")
        self._check(lib().ras_pml_wsnet_forward(self.ptr, _ptr(x), x.shape[0], _ptr(y),
                                                _stream(stream)))
        return y

    def gradient(self, x, target, want_grad=True, stream=None):
        """Returns (loss, flat gradient or None)."""
        import numpy as np
        self._grid(x, "x")
        self._grid(target, "target")
        loss = ctypes.c_double(0.0)
        g = np.zeros(self.nweights, dtype=np.float32) if want_grad else None
        self._check(lib().ras_pml_wsnet_gradient(self.ptr, _ptr(x), _ptr(target), x.shape[0],
                                                 ctypes.byref(loss),
                                                 g.ctypes.data_as(_P) if want_grad else None,
                                                 _stream(stream)))
        return loss.value, g

    def adam(self, lr, stream=None):
        self._check(lib().ras_pml_wsnet_adam(self.ptr, float(lr), _stream(stream)))

    def train_step(self, x, target, lr, want_loss=False, stream=None):
        loss = ctypes.c_double(0.0)
        self._check(lib().ras_pml_wsnet_train_step(self.ptr, _ptr(x), _ptr(target), x.shape[0],
                                                   float(lr),
                                                   ctypes.byref(loss) if want_loss else None,
                                                   _stream(stream)))
        return loss.value if want_loss else None

    def close(self):
        if getattr(self, "ptr", None):
            lib().ras_pml_wsnet_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ras_pml_grid_sample(H: Handle, vec, scale=1.0, out=None, stream=None):
    """vec (complex128 over the unknowns) on the interior grid, times scale:
    float32 (grid, grid, 2)."""
    import torch
    _check_vec(vec, H.ndof, "vec")
    n = H.grid_side()
    if out is None:
        out = torch.empty((n, n, 2), dtype=torch.float32, device=vec.device)
    rc = lib().ras_pml_grid_sample(H.ptr, _ptr(vec), float(scale), _ptr(out), _stream(stream))
    if rc:
        H._raise(rc)
    return out


def ras_pml_warm_start(H: Handle, net: WSNet, f, b, x0, fscale=1.0, stream=None):
    """Fills x0 with the network's guess (or zeros); returns whether it was kept."""
    for t, nm in ((f, "f"), (b, "b"), (x0, "x0")):
        _check_vec(t, H.ndof, nm)
    used = ctypes.c_int(0)
    rc = lib().ras_pml_warm_start(H.ptr, net.ptr, _ptr(f), _ptr(b), _ptr(x0), float(fscale),
                                  ctypes.byref(used), _stream(stream))
    if rc:
        H._raise(rc)
    return bool(used.value)
