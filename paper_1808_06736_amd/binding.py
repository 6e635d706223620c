"""ctypes binding of libesnufft.so (the C ABI in include/esnufft.h).

Argument marshalling only: every step of the transforms runs in the HIP
library.  The ``esn_*`` functions mirror the C entry points one to one (device
pointers are plain integers); ``Plan`` is a thin convenience wrapper that takes
torch CUDA tensors, passes their ``data_ptr()`` and torch's current stream, and
raises on error statuses.  There is no CPU fallback: without the built library
every call raises.
"""
from __future__ import annotations

import ctypes
import math
import os
import warnings

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libesnufft.so")

ESN_SINGLE = 1
ESN_DOUBLE = 2

STATUS = {
    0: "ESN_OK", 1: "ESN_WARN_EPS_TOO_SMALL", 2: "ESN_ERR_BAD_ARG",
    3: "ESN_ERR_PTS_OUT_OF_RANGE", 4: "ESN_ERR_NAN_PTS", 5: "ESN_ERR_BUDGET",
    6: "ESN_ERR_ALLOC", 7: "ESN_ERR_FFT_PLAN", 8: "ESN_ERR_HIP",
    9: "ESN_ERR_UNSUPPORTED", 10: "ESN_ERR_NO_POINTS", 11: "ESN_ERR_QUEUE",
}
for _k, _v in STATUS.items():
    globals()[_v] = _k

i64 = ctypes.c_int64
vp = ctypes.c_void_p
ci = ctypes.c_int
cd = ctypes.c_double


class EsnOpts(ctypes.Structure):
    _fields_ = [("debug", ci), ("chkbnds", ci), ("modeord", ci), ("upsampfac", cd),
                ("sort", ci), ("spread_method", ci), ("interp_method", ci),
                ("bin", ci * 3), ("maxsubprob", ci), ("ntransf_chunk", ci), ("block", ci),
                ("kerevalmeth", ci)]


class EsnParams(ctypes.Structure):
    _fields_ = [("w", ci), ("beta", cd), ("nquad", ci), ("nf", i64 * 3)]


class EsnInfo(ctypes.Structure):
    _fields_ = [("type", ci), ("dim", ci), ("isign", ci), ("ntransf", ci), ("prec", ci),
                ("w", ci), ("nquad", ci), ("modeord", ci), ("beta", cd), ("eps", cd),
                ("nmodes", i64 * 3), ("nf", i64 * 3), ("M", i64), ("bin", ci * 3),
                ("maxsubprob", ci), ("nsubprob", ci), ("nbins_nonempty", ci),
                ("ntransf_chunk", ci), ("spread_method", ci), ("interp_method", ci),
                ("point_code", ci), ("device_bytes", i64), ("ndense_units", ci),
                ("kerevalmeth", ci)]


class EsnStats(ctypes.Structure):
    _fields_ = [("t_setpts", cd), ("t_spread_or_interp", cd), ("t_fft", cd),
                ("t_deconv_or_amplify", cd), ("t_execute", cd)]


class EsnRequest(ctypes.Structure):
    _fields_ = [("type", ci), ("dim", ci), ("nmodes", i64 * 3), ("isign", ci), ("eps", cd),
                ("prec", ci), ("M", i64), ("coord_prec", ci), ("x", vp), ("y", vp), ("z", vp),
                ("c", vp), ("f", vp), ("points_id", ctypes.c_longlong), ("stream", vp)]


class EsnServeStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_longlong) for n in
                ("submitted", "completed", "failed", "rejected", "queued", "running",
                 "plan_cache_hits", "plan_cache_misses", "point_cache_hits", "cached_plans",
                 "hbm_in_use", "hbm_peak")] + \
               [(n, cd) for n in ("p50_ms", "p99_ms", "mean_ms", "max_ms", "pts_per_s")]


class EsnError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} ({strerror(status)})")


_lib = None

# (name, argtypes) of every C entry point; restype int unless noted
_SIGS = {
    "esn_default_opts": ([ctypes.POINTER(EsnOpts)], None),
    "esn_choose_params": ([cd, ci, ci, ctypes.POINTER(i64), cd, ctypes.POINTER(EsnParams)], ci),
    "esn_makeplan": ([ci, ci, ctypes.POINTER(i64), ci, ci, cd, ci, ctypes.POINTER(vp),
                      ctypes.POINTER(EsnOpts), vp], ci),
    "esn_setpts": ([vp, i64, ci, vp, vp, vp], ci),
    "esn_setpts3": ([vp, i64, ci, vp, vp, vp, i64, vp, vp, vp], ci),
    "esn_execute": ([vp, vp, vp], ci),
    "esn_execute_adjoint": ([vp, vp, vp], ci),
    "esn_spread": ([vp, vp, vp], ci),
    "esn_interp": ([vp, vp, vp], ci),
    "esn_get_info": ([vp, ctypes.POINTER(EsnInfo)], ci),
    "esn_get_stats": ([vp, ctypes.POINTER(EsnStats)], ci),
    "esn_destroy": ([vp], ci),
    "esn_1d1": ([i64, vp, vp, ci, cd, i64, vp, ci, ctypes.POINTER(EsnOpts), vp], ci),
    "esn_1d2": ([i64, vp, vp, ci, cd, i64, vp, ci, ctypes.POINTER(EsnOpts), vp], ci),
    "esn_2d1": ([i64, vp, vp, vp, ci, cd, i64, i64, vp, ci, ctypes.POINTER(EsnOpts), vp], ci),
    "esn_2d2": ([i64, vp, vp, vp, ci, cd, i64, i64, vp, ci, ctypes.POINTER(EsnOpts), vp], ci),
    "esn_3d1": ([i64, vp, vp, vp, vp, ci, cd, i64, i64, i64, vp, ci, ctypes.POINTER(EsnOpts),
                 vp], ci),
    "esn_3d2": ([i64, vp, vp, vp, vp, ci, cd, i64, i64, i64, vp, ci, ctypes.POINTER(EsnOpts),
                 vp], ci),
    "esn_strerror": ([ci], ctypes.c_char_p),
    "esn_gauss_legendre": ([ci, vp, vp], ci),
    "esn_correction_factors": ([ci, cd, ci, i64, i64, vp], ci),
    "esn_kernel_poly": ([ci, cd, vp], ci),
    "esn_toeplitz_makeplan": ([ci, ctypes.POINTER(i64), ci, cd, ci, i64, ci, vp, vp, vp, vp,
                               ctypes.POINTER(vp), ctypes.POINTER(EsnOpts), vp], ci),
    "esn_toeplitz_apply": ([vp, vp, vp], ci),
    "esn_get_stats_history": ([vp, ctypes.POINTER(EsnStats), ci, ctypes.POINTER(ci)], ci),
    "esn_toeplitz_destroy": ([vp], ci),
    "esn_plan_correction": ([vp, ci, vp, i64], ci),
    "esn_debug_sort": ([vp, vp, vp, vp, vp, vp], ci),
    "esn_setpts_noalloc": ([vp, i64, ci, vp, vp, vp], ci),
    "esn_server_create": ([ctypes.POINTER(EsnOpts), ci, ctypes.c_longlong, ctypes.POINTER(vp)], ci),
    "esn_server_submit": ([vp, ctypes.POINTER(EsnRequest), ctypes.POINTER(ctypes.c_longlong)], ci),
    "esn_server_wait": ([vp, ctypes.c_longlong, ctypes.POINTER(ci), ctypes.POINTER(cd)], ci),
    "esn_server_stats": ([vp, ctypes.POINTER(EsnServeStats)], ci),
    "esn_server_reset_stats": ([vp], ci),
    "esn_server_destroy": ([vp], ci),
}


def lib():
    """Load libesnufft.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1808_06736_amd.build`")
        try:
            # torch ships its own HIP runtime under the same soname; loading torch
            # first makes this library bind to that one runtime, so torch's
            # streams and device pointers are valid here.
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def strerror(status: int) -> str:
    try:
        return lib().esn_strerror(int(status)).decode()
    except Exception:          # the library itself failed to load
        return STATUS.get(status, "unknown")


def _i64x3(vals):
    v = list(vals or ()) + [1] * (3 - len(vals or ()))
    return (i64 * 3)(*[int(a) for a in v[:3]])


# ---- C entry points, same names ------------------------------------------------
def esn_default_opts() -> EsnOpts:
    o = EsnOpts()
    lib().esn_default_opts(ctypes.byref(o))
    return o


def esn_choose_params(eps, prec, dim, nmodes, upsampfac=2.0):
    out = EsnParams()
    st = lib().esn_choose_params(float(eps), int(prec), int(dim), _i64x3(nmodes),
                                 float(upsampfac), ctypes.byref(out))
    return st, out


def esn_makeplan(type_, dim, nmodes, isign, ntransf, eps, prec, opts=None, stream=None):
    h = vp()
    st = lib().esn_makeplan(int(type_), int(dim), _i64x3(nmodes), int(isign), int(ntransf),
                            float(eps), int(prec), ctypes.byref(h),
                            ctypes.byref(opts) if opts is not None else None, stream)
    return st, h


def esn_setpts(plan, M, coord_prec, x, y=None, z=None):
    return lib().esn_setpts(plan, int(M), int(coord_prec), x, y, z)


def esn_setpts3(plan, M, coord_prec, xs, N, ss):
    xs = list(xs) + [None] * (3 - len(xs))
    ss = list(ss) + [None] * (3 - len(ss))
    return lib().esn_setpts3(plan, int(M), int(coord_prec), xs[0], xs[1], xs[2], int(N),
                             ss[0], ss[1], ss[2])


def esn_execute(plan, c, f):
    return lib().esn_execute(plan, c, f)


def esn_execute_adjoint(plan, c, f):
    return lib().esn_execute_adjoint(plan, c, f)


def esn_spread(plan, c, grid):
    return lib().esn_spread(plan, c, grid)


def esn_interp(plan, grid, c):
    return lib().esn_interp(plan, grid, c)


def esn_get_info(plan) -> EsnInfo:
    info = EsnInfo()
    st = lib().esn_get_info(plan, ctypes.byref(info))
    if st:
        raise EsnError(st, "esn_get_info")
    return info


def esn_get_stats(plan) -> EsnStats:
    s = EsnStats()
    st = lib().esn_get_stats(plan, ctypes.byref(s))
    if st:
        raise EsnError(st, "esn_get_stats")
    return s


def esn_gauss_legendre(p):
    """Host arrays (nodes, weights) of the p positive nodes of the 2p-node rule."""
    import numpy as np
    q = np.zeros(p)
    w = np.zeros(p)
    check(lib().esn_gauss_legendre(int(p), q.ctypes.data, w.ctypes.data), "esn_gauss_legendre")
    return q, w


def esn_correction_factors(w, beta, nquad, nf, N):
    import numpy as np
    out = np.zeros(int(N) // 2 + 1)
    check(lib().esn_correction_factors(int(w), float(beta), int(nquad), int(nf), int(N),
                                       out.ctypes.data), "esn_correction_factors")
    return out


def esn_kernel_poly(w, beta):
    """Piecewise polynomial kernel table (Sec. 5.3): array [w, w + 4], row k the
    monomial coefficients (t^0 first) of interval k's polynomial in t in [-1, 1]."""
    import numpy as np
    out = np.zeros((int(w), int(w) + 4))
    check(lib().esn_kernel_poly(int(w), float(beta), out.ctypes.data), "esn_kernel_poly")
    return out


def esn_plan_correction(plan, m, N_m):
    import numpy as np
    out = np.zeros(int(N_m) // 2 + 1)
    check(lib().esn_plan_correction(plan, int(m), out.ctypes.data, out.shape[0]),
          "esn_plan_correction")
    return out


def esn_debug_sort(plan):
    """The plan's bin sort as host numpy arrays: dict with M, nbins,
    cells_per_bin, nsub, method, perm[M], key[M], bin_start[nbins + 1] and
    sub[nsub, 3] ({bin, first position, length}); bin_start and sub only for
    sorted plans."""
    import numpy as np
    geom = np.zeros(5, dtype=np.int64)
    check(lib().esn_debug_sort(plan, vp(geom.ctypes.data), None, None, None, None),
          "esn_debug_sort")
    M, nbins, cpb, nsub, method = (int(v) for v in geom)
    out = dict(M=M, nbins=nbins, cells_per_bin=cpb, nsub=nsub, method=method)
    perm = np.zeros(max(M, 0), dtype=np.int32)
    key = np.zeros(max(M, 0), dtype=np.uint32)
    ptr = lambda a: vp(a.ctypes.data) if a.size else None
    bstart = sub = None
    if method:
        bstart = np.zeros(nbins + 1, dtype=np.int32)
        sub = np.zeros((nsub, 3), dtype=np.int32)
    check(lib().esn_debug_sort(plan, vp(geom.ctypes.data), ptr(perm), ptr(key),
                               ptr(bstart) if bstart is not None else None,
                               ptr(sub) if sub is not None else None), "esn_debug_sort")
    out.update(perm=perm, key=key, bin_start=bstart, sub=sub)
    return out


def esn_destroy(plan):
    return lib().esn_destroy(plan)


def _oneshot(name, *args):
    return getattr(lib(), name)(*args)


def esn_1d1(M, x, c, isign, eps, N1, f, prec, opts=None, stream=None):
    return _oneshot("esn_1d1", M, x, c, isign, eps, N1, f, prec, opts, stream)


def esn_1d2(M, x, c, isign, eps, N1, f, prec, opts=None, stream=None):
    return _oneshot("esn_1d2", M, x, c, isign, eps, N1, f, prec, opts, stream)


def esn_2d1(M, x, y, c, isign, eps, N1, N2, f, prec, opts=None, stream=None):
    return _oneshot("esn_2d1", M, x, y, c, isign, eps, N1, N2, f, prec, opts, stream)


def esn_2d2(M, x, y, c, isign, eps, N1, N2, f, prec, opts=None, stream=None):
    return _oneshot("esn_2d2", M, x, y, c, isign, eps, N1, N2, f, prec, opts, stream)


def esn_3d1(M, x, y, z, c, isign, eps, N1, N2, N3, f, prec, opts=None, stream=None):
    return _oneshot("esn_3d1", M, x, y, z, c, isign, eps, N1, N2, N3, f, prec, opts, stream)


def esn_3d2(M, x, y, z, c, isign, eps, N1, N2, N3, f, prec, opts=None, stream=None):
    return _oneshot("esn_3d2", M, x, y, z, c, isign, eps, N1, N2, N3, f, prec, opts, stream)


def check(status, where=""):
    """Raise EsnError for error statuses; warn for status 1."""
    if status >= 2:
        raise EsnError(status, where)
    if status == 1:
        warnings.warn(f"{where}: {strerror(1)}", RuntimeWarning, stacklevel=3)
    return status


# ---- torch convenience wrapper --------------------------------------------------
def _stream_handle(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def make_opts(**kw) -> EsnOpts:
    o = esn_default_opts()
    for k, v in kw.items():
        if k == "bin":
            for m, b in enumerate(list(v) + [0] * (3 - len(v))):
                o.bin[m] = int(b)
        else:
            setattr(o, k, v)
    return o


class Plan:
    """A type 1 or type 2 plan over torch CUDA tensors.

    ``Plan(type_, N, eps, dtype=torch.complex64, isign=None, ntransf=1, **opts)``
    with N a tuple of 1..3 mode counts (N1 first).  isign defaults to +1 for
    type 1 and -1 for type 2.  Work is enqueued on torch's current stream.
    """

    def __init__(self, type_, N, eps, dtype=None, isign=None, ntransf=1, **opts):
        import torch
        self.torch = torch
        self.type = int(type_)
        self.N = tuple(int(n) for n in N)
        self.dim = len(self.N)
        self.dtype = dtype or torch.complex64
        if self.dtype not in (torch.complex64, torch.complex128):
            raise ValueError("dtype must be torch.complex64 or torch.complex128")
        self.prec = ESN_SINGLE if self.dtype == torch.complex64 else ESN_DOUBLE
        self.isign = isign if isign is not None else (1 if self.type == 1 else -1)
        self.ntransf = int(ntransf)
        self.eps = float(eps)
        self.opts = make_opts(**opts)
        self.device = torch.device("cuda", torch.cuda.current_device())
        st, h = esn_makeplan(self.type, self.dim, self.N, self.isign, self.ntransf, self.eps,
                             self.prec, self.opts, _stream_handle(torch))
        check(st, "esn_makeplan")
        self.handle = h
        self.M = None

    def info(self) -> EsnInfo:
        return esn_get_info(self.handle)

    def stats(self) -> EsnStats:
        return esn_get_stats(self.handle)

    def stats_history(self, max_entries=256):
        """Stage times of the latest setpts / execute calls, oldest first (debug plans)."""
        return esn_get_stats_history(self.handle, max_entries)

    def debug_sort(self):
        """The bin sort of the current points (see esn_debug_sort)."""
        return esn_debug_sort(self.handle)

    def setpts_noalloc(self, *coords):
        """setpts without device allocation (esn_setpts_noalloc): the plan
        must already hold room for these points (an earlier setpts of at
        least as many)."""
        torch = self.torch
        if len(coords) != self.dim:
            raise ValueError(f"need {self.dim} coordinate arrays")
        M = coords[0].numel()
        cdt = coords[0].dtype
        if cdt not in (torch.float32, torch.float64):
            raise ValueError("coordinates must be float32 or float64")
        ptrs = []
        for a in coords:
            if a.dtype != cdt or a.numel() != M or not a.is_cuda or not a.is_contiguous():
                raise ValueError("coordinates: same dtype, same length, contiguous, on the GPU")
            ptrs.append(vp(a.data_ptr()) if M > 0 else None)
        ptrs += [None] * (3 - len(ptrs))
        st = lib().esn_setpts_noalloc(self.handle, M,
                                      ESN_SINGLE if cdt == torch.float32 else ESN_DOUBLE, *ptrs)
        check(st, "esn_setpts_noalloc")
        self.M = M
        return self

    def setpts(self, *coords):
        torch = self.torch
        if len(coords) != self.dim:
            raise ValueError(f"need {self.dim} coordinate arrays")
        M = coords[0].numel()
        cdt = coords[0].dtype
        if cdt not in (torch.float32, torch.float64):
            raise ValueError("coordinates must be float32 or float64")
        ptrs = []
        for a in coords:
            if a.dtype != cdt or a.numel() != M or not a.is_cuda or not a.is_contiguous():
                raise ValueError("coordinates: same dtype, same length, contiguous, on the GPU")
            ptrs.append(vp(a.data_ptr()) if M > 0 else None)
        ptrs += [None] * (3 - len(ptrs))
        st = esn_setpts(self.handle, M, ESN_SINGLE if cdt == torch.float32 else ESN_DOUBLE,
                        *ptrs)
        check(st, "esn_setpts")
        self.M = M
        return self

    def _shape_c(self):
        return (self.ntransf, self.M) if self.ntransf > 1 else (self.M,)

    def _shape_f(self):
        Nrev = tuple(reversed(self.N))
        return ((self.ntransf,) + Nrev) if self.ntransf > 1 else Nrev

    def _check(self, t, shape, name):
        if t.dtype != self.dtype or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name}: must be a contiguous {self.dtype} CUDA tensor")
        if t.numel() != int(__import__("math").prod(shape)):
            raise ValueError(f"{name}: expected {shape} elements, got {tuple(t.shape)}")

    def execute(self, c, f):
        if self.M is None:
            raise EsnError(ESN_ERR_NO_POINTS, "execute")
        self._check(c, self._shape_c(), "c")
        self._check(f, self._shape_f(), "f")
        st = esn_execute(self.handle, vp(c.data_ptr()) if c.numel() else None,
                         vp(f.data_ptr()))
        check(st, "esn_execute")
        return c, f

    def execute_adjoint(self, c, f):
        """The adjoint transform on the same sorted points (type 1 plan: reads f,
        writes c; type 2 plan: reads c, writes f; exponent sign -isign)."""
        if self.M is None:
            raise EsnError(ESN_ERR_NO_POINTS, "execute_adjoint")
        self._check(c, self._shape_c(), "c")
        self._check(f, self._shape_f(), "f")
        st = esn_execute_adjoint(self.handle, vp(c.data_ptr()) if c.numel() else None,
                                 vp(f.data_ptr()))
        check(st, "esn_execute_adjoint")
        return c, f

    def adjoint(self, x, out=None):
        """Adjoint of this plan's transform applied to x: for a type 1 plan x
        holds modes f and the result is c at the points; for a type 2 plan x
        holds strengths c and the result is modes f."""
        if self.type == 1:
            c = out if out is not None else self.torch.empty(self._shape_c(), dtype=self.dtype,
                                                             device=self.device)
            self.execute_adjoint(c, x)
            return c
        f = out if out is not None else self.torch.empty(self._shape_f(), dtype=self.dtype,
                                                         device=self.device)
        self.execute_adjoint(x, f)
        return f

    def type1(self, c, out=None):
        f = out if out is not None else self.torch.empty(self._shape_f(), dtype=self.dtype,
                                                         device=self.device)
        self.execute(c, f)
        return f

    def type2(self, f, out=None):
        c = out if out is not None else self.torch.empty(self._shape_c(), dtype=self.dtype,
                                                         device=self.device)
        self.execute(c, f)
        return c

    def fine_grid_shape(self):
        info = self.info()
        nf = [int(info.nf[m]) for m in range(self.dim)]
        return ((self.ntransf,) if self.ntransf > 1 else ()) + tuple(reversed(nf))

    def spread(self, c, grid=None):
        grid = grid if grid is not None else self.torch.empty(self.fine_grid_shape(),
                                                              dtype=self.dtype,
                                                              device=self.device)
        self._check(c, self._shape_c(), "c")
        check(esn_spread(self.handle, vp(c.data_ptr()) if c.numel() else None,
                         vp(grid.data_ptr())), "esn_spread")
        return grid

    def interp(self, grid, c=None):
        c = c if c is not None else self.torch.empty(self._shape_c(), dtype=self.dtype,
                                                      device=self.device)
        check(esn_interp(self.handle, vp(grid.data_ptr()), vp(c.data_ptr()) if c.numel() else None),
              "esn_interp")
        return c

    def close(self):
        if getattr(self, "handle", None):
            esn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan3:
    """A type 3 plan (eq. (3), Sec. 3.3) over torch CUDA tensors:
    ``Plan3(dim, eps, dtype=torch.complex64, isign=+1, ntransf=1, **opts)``,
    then ``setpts(sources, targets)`` (lists of dim coordinate tensors) and
    ``execute(c)`` -> f at the N targets, f_k = sum_j c_j exp(isign i s_k.x_j).
    Work is enqueued on torch's current stream."""

    def __init__(self, dim, eps, dtype=None, isign=1, ntransf=1, **opts):
        import torch
        self.torch = torch
        self.dim = int(dim)
        self.dtype = dtype or torch.complex64
        if self.dtype not in (torch.complex64, torch.complex128):
            raise ValueError("dtype must be torch.complex64 or torch.complex128")
        self.prec = ESN_SINGLE if self.dtype == torch.complex64 else ESN_DOUBLE
        self.isign = int(isign)
        self.ntransf = int(ntransf)
        self.opts = make_opts(**opts)
        self.device = torch.device("cuda", torch.cuda.current_device())
        st, h = esn_makeplan(3, self.dim, (1,) * self.dim, self.isign, self.ntransf, eps,
                             self.prec, self.opts, _stream_handle(torch))
        check(st, "esn_makeplan")
        self.handle = h
        self.M = self.N = None

    def info(self) -> EsnInfo:
        return esn_get_info(self.handle)

    def stats(self) -> EsnStats:
        return esn_get_stats(self.handle)

    def setpts(self, sources, targets):
        torch = self.torch
        if len(sources) != self.dim or len(targets) != self.dim:
            raise ValueError(f"need {self.dim} source and {self.dim} target coordinate arrays")
        arrs = list(sources) + list(targets)
        cdt = arrs[0].dtype
        if cdt not in (torch.float32, torch.float64):
            raise ValueError("coordinates must be float32 or float64")
        M, N = sources[0].numel(), targets[0].numel()
        for k, a in enumerate(arrs):
            n = M if k < self.dim else N
            if a.dtype != cdt or a.numel() != n or not a.is_cuda or not a.is_contiguous():
                raise ValueError("coordinates: same dtype, same length per set, contiguous, "
                                 "on the GPU")
        ptr = lambda a: vp(a.data_ptr()) if a.numel() else None
        self.M = self.N = None   # a failed call leaves the plan without points
        st = esn_setpts3(self.handle, M, ESN_SINGLE if cdt == torch.float32 else ESN_DOUBLE,
                         [ptr(a) for a in sources], N, [ptr(a) for a in targets])
        check(st, "esn_setpts3")
        self.M, self.N = M, N
        return self

    def execute(self, c, out=None):
        if self.M is None:
            raise EsnError(ESN_ERR_NO_POINTS, "execute")
        shp_c = (self.ntransf, self.M) if self.ntransf > 1 else (self.M,)
        shp_f = (self.ntransf, self.N) if self.ntransf > 1 else (self.N,)
        if c.dtype != self.dtype or not c.is_cuda or not c.is_contiguous() or \
                c.numel() != self.ntransf * self.M:
            raise ValueError(f"c: must be a contiguous {self.dtype} CUDA tensor of {shp_c}")
        f = out if out is not None else self.torch.empty(shp_f, dtype=self.dtype,
                                                         device=self.device)
        st = esn_execute(self.handle, vp(c.data_ptr()) if c.numel() else None,
                         vp(f.data_ptr()) if f.numel() else None)
        check(st, "esn_execute")
        return f

    def close(self):
        if getattr(self, "handle", None):
            esn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- normal operator in Toeplitz form --------------------------------------------
def esn_get_stats_history(plan, max_entries=256):
    """Stage times of the plan's latest setpts / execute calls, oldest first."""
    buf = (EsnStats * int(max_entries))()
    n = ci()
    check(lib().esn_get_stats_history(plan, buf, int(max_entries), ctypes.byref(n)),
          "esn_get_stats_history")
    return [buf[k] for k in range(n.value)]


def esn_toeplitz_makeplan(dim, nmodes, isign, eps, prec, M, coord_prec, xs, weights=None,
                          opts=None, stream=None):
    h = vp()
    xs = list(xs) + [None] * (3 - len(xs))
    st = lib().esn_toeplitz_makeplan(int(dim), _i64x3(nmodes), int(isign), float(eps), int(prec),
                                     int(M), int(coord_prec), xs[0], xs[1], xs[2], weights,
                                     ctypes.byref(h),
                                     ctypes.byref(opts) if opts is not None else None, stream)
    return st, h


def esn_toeplitz_apply(t, f, g):
    return lib().esn_toeplitz_apply(t, f, g)


def esn_toeplitz_destroy(t):
    return lib().esn_toeplitz_destroy(t)


class Toeplitz:
    """The normal operator T = A^H W A of a type 2 transform A (sign isign, modes
    N) on given points, W = diag(weights), over torch CUDA tensors:
    ``Toeplitz(coords, N, eps, dtype=torch.complex64, isign=-1, weights=None,
    **opts)``; ``apply(f)`` -> T f (modes in the order of opts modeord).  Work is
    enqueued on torch's current stream."""

    def __init__(self, coords, N, eps, dtype=None, isign=-1, weights=None, **opts):
        import torch
        self.torch = torch
        self.N = tuple(int(n) for n in N)
        self.dim = len(self.N)
        self.dtype = dtype or torch.complex64
        if self.dtype not in (torch.complex64, torch.complex128):
            raise ValueError("dtype must be torch.complex64 or torch.complex128")
        prec = ESN_SINGLE if self.dtype == torch.complex64 else ESN_DOUBLE
        if len(coords) != self.dim:
            raise ValueError(f"need {self.dim} coordinate arrays")
        cdt = coords[0].dtype
        M = coords[0].numel()
        for a in coords:
            if a.dtype != cdt or a.numel() != M or not a.is_cuda or not a.is_contiguous():
                raise ValueError("coordinates: same dtype and length, contiguous, on the GPU")
        if weights is not None and (weights.dtype != self.dtype or weights.numel() != M or
                                    not weights.is_cuda or not weights.is_contiguous()):
            raise ValueError(f"weights: a contiguous {self.dtype} CUDA tensor of {M} values")
        ptr = lambda a: vp(a.data_ptr()) if a is not None and a.numel() else None
        self.opts = make_opts(**opts)
        self.device = torch.device("cuda", torch.cuda.current_device())
        st, h = esn_toeplitz_makeplan(self.dim, self.N, int(isign), eps, prec, M,
                                      ESN_SINGLE if cdt == torch.float32 else ESN_DOUBLE,
                                      [ptr(a) for a in coords], ptr(weights), self.opts,
                                      _stream_handle(torch))
        check(st, "esn_toeplitz_makeplan")
        self.handle = h

    def apply(self, f, out=None):
        shape = tuple(reversed(self.N))
        if f.dtype != self.dtype or not f.is_cuda or not f.is_contiguous() or \
                f.numel() != math.prod(self.N):
            raise ValueError(f"f: must be a contiguous {self.dtype} CUDA tensor of {shape}")
        g = out if out is not None else self.torch.empty(shape, dtype=self.dtype,
                                                         device=self.device)
        check(esn_toeplitz_apply(self.handle, vp(f.data_ptr()), vp(g.data_ptr())),
              "esn_toeplitz_apply")
        return g

    def close(self):
        if getattr(self, "handle", None):
            esn_toeplitz_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- serving -------------------------------------------------------------------
def esn_server_create(opts, nslots, hbm_budget_bytes):
    h = vp()
    st = lib().esn_server_create(ctypes.byref(opts) if opts is not None else None, int(nslots),
                                 int(hbm_budget_bytes), ctypes.byref(h))
    return st, h


def esn_server_submit(server, req):
    t = ctypes.c_longlong()
    st = lib().esn_server_submit(server, ctypes.byref(req), ctypes.byref(t))
    return st, t.value


def esn_server_wait(server, ticket):
    st = ci()
    lat = cd()
    rc = lib().esn_server_wait(server, int(ticket), ctypes.byref(st), ctypes.byref(lat))
    return rc, st.value, lat.value


def esn_server_stats(server):
    o = EsnServeStats()
    check(lib().esn_server_stats(server, ctypes.byref(o)), "esn_server_stats")
    return o


def esn_server_reset_stats(server):
    return lib().esn_server_reset_stats(server)


def esn_server_destroy(server):
    return lib().esn_server_destroy(server)


class Server:
    """Continuous-batching request loop over torch CUDA tensors.

    ``submit`` takes the request's tensors (kept referenced until ``wait``) and
    returns a ticket; ``wait`` blocks until that request is done and returns
    (status, latency in ms).
    """

    def __init__(self, nslots=4, hbm_budget_bytes=64 << 30, **opts):
        import torch
        self.torch = torch
        self.opts = make_opts(**opts)
        st, self.handle = esn_server_create(self.opts, nslots, hbm_budget_bytes)
        check(st, "esn_server_create")
        self._keep = {}

    def submit(self, type_, coords, c, f, eps, isign=None, points_id=0):
        torch = self.torch
        dim = len(coords)
        N = tuple(reversed(f.shape[-dim:]))
        r = EsnRequest()
        r.type = int(type_)
        r.dim = dim
        for m in range(3):
            r.nmodes[m] = int(N[m]) if m < dim else 1
        r.isign = isign if isign is not None else (1 if type_ == 1 else -1)
        r.eps = float(eps)
        r.prec = ESN_SINGLE if f.dtype == torch.complex64 else ESN_DOUBLE
        r.M = coords[0].numel()
        r.coord_prec = ESN_SINGLE if coords[0].dtype == torch.float32 else ESN_DOUBLE
        ptrs = [a.data_ptr() if r.M else None for a in coords] + [None] * (3 - dim)
        r.x, r.y, r.z = ptrs[0], ptrs[1], ptrs[2]
        r.c = c.data_ptr() if r.M else None
        r.f = f.data_ptr()
        r.points_id = int(points_id)
        # the request waits for the work queued so far on torch's current stream
        r.stream = _stream_handle(torch)
        st, t = esn_server_submit(self.handle, r)
        check(st, "esn_server_submit")
        self._keep[t] = (coords, c, f)
        return t

    def wait(self, ticket):
        rc, st, lat = esn_server_wait(self.handle, ticket)
        check(rc, "esn_server_wait")
        self._keep.pop(ticket, None)
        return st, lat

    def stats(self):
        return esn_server_stats(self.handle)

    def reset_stats(self):
        esn_server_reset_stats(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            esn_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
