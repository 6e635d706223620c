"""Python front end of the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the GPU library or its binding.

It evaluates the type 1 / type 2 / type 3 exponential sums of Sec. 1, eqs.
(1)-(3), by their definitions in double precision (see ``oracle.c``), plus the
relative l2 error metric of Sec. 4.2 used to compare any approximation against
them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i64, dp, ip = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
        lib.oracle_type1.argtypes = [ip, i64, dp, dp, dp, dp, ip, i64, dp, i64, dp,
                                     i64, dp, dp, ip]
        lib.oracle_type1.restype = ip
        lib.oracle_type2.argtypes = [ip, i64, dp, dp, dp, dp, i64, i64, i64, ip, dp,
                                     ip]
        lib.oracle_type2.restype = ip
        lib.oracle_type3.argtypes = [ip, i64, dp, dp, dp, dp, i64, dp, dp, dp, ip, dp, ip]
        lib.oracle_type3.restype = ip
        _lib = lib
    return _lib


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _coords64(coords, d):
    out = [np.ascontiguousarray(np.asarray(coords[m], dtype=np.float64)) for m in range(d)]
    while len(out) < 3:
        out.append(None)
    return out


def mode_indices(N: int) -> np.ndarray:
    """I_N in increasing order: -floor(N/2) .. -floor(N/2)+N-1 (Sec. 1)."""
    return np.arange(N, dtype=np.int64) - (N // 2)


def type1(coords, c, isign: int, N=None, modes=None, nthreads=None) -> np.ndarray:
    """f_k = sum_j c_j exp(isign i k.x_j)  (eq. (1)), in complex128.

    ``coords``: list of d coordinate arrays (any float dtype; upcast exactly).
    ``c``: M complex strengths.  Either ``N`` (modes per dim; full mode set) or
    ``modes`` (list of d integer index arrays; their product set) selects the
    outputs.  Returns an array of shape (n_d, ..., n_1) (first dim fastest).
    """
    d = len(coords)
    if modes is None:
        modes = [mode_indices(int(N[m])) for m in range(d)]
    ks = [np.ascontiguousarray(np.asarray(modes[m], dtype=np.int64)) for m in range(d)]
    while len(ks) < 3:
        ks.append(np.zeros(1, dtype=np.int64))
    xs = _coords64(coords, d)
    cc = np.ascontiguousarray(np.asarray(c, dtype=np.complex128)).reshape(-1)
    M = cc.shape[0]
    for m in range(d):
        assert xs[m].shape[0] == M
    out = np.zeros(len(ks[0]) * len(ks[1]) * len(ks[2]), dtype=np.complex128)
    rc = _load().oracle_type1(d, M, _ptr(xs[0]), _ptr(xs[1]), _ptr(xs[2]), _ptr(cc),
                              int(isign), len(ks[0]), _ptr(ks[0]), len(ks[1]),
                              _ptr(ks[1]), len(ks[2]), _ptr(ks[2]), _ptr(out),
                              nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_type1: bad arguments")
    shape = tuple(len(ks[m]) for m in reversed(range(d)))
    return out.reshape(shape)


def type2(coords, f, isign: int, nthreads=None) -> np.ndarray:
    """c_j = sum_k f_k exp(isign i k.x_j)  (eq. (2)), in complex128.

    ``f`` has shape (N_d, ..., N_1) (first dim fastest), each dimension in
    increasing mode order from -floor(N_m/2).  Returns M values.
    """
    d = len(coords)
    ff = np.ascontiguousarray(np.asarray(f, dtype=np.complex128))
    assert ff.ndim == d
    Ns = list(reversed(ff.shape)) + [1] * (3 - d)
    xs = _coords64(coords, d)
    M = xs[0].shape[0]
    out = np.zeros(M, dtype=np.complex128)
    rc = _load().oracle_type2(d, M, _ptr(xs[0]), _ptr(xs[1]), _ptr(xs[2]),
                              _ptr(ff), Ns[0], Ns[1], Ns[2], int(isign), _ptr(out),
                              nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_type2: bad arguments")
    return out


def type3(coords, c, targets, isign: int, nthreads=None) -> np.ndarray:
    """f_k = sum_j c_j exp(isign i s_k.x_j)  (eq. (3)), in complex128.

    ``coords``: d source coordinate arrays (M values each); ``targets``: d
    target frequency arrays (N values each); ``c``: M strengths.  Returns N
    values.
    """
    d = len(coords)
    assert len(targets) == d
    xs = _coords64(coords, d)
    ss = _coords64(targets, d)
    cc = np.ascontiguousarray(np.asarray(c, dtype=np.complex128)).reshape(-1)
    M, N = cc.shape[0], ss[0].shape[0]
    for m in range(d):
        assert xs[m].shape[0] == M and ss[m].shape[0] == N
    out = np.zeros(N, dtype=np.complex128)
    rc = _load().oracle_type3(d, M, _ptr(xs[0]), _ptr(xs[1]), _ptr(xs[2]), _ptr(cc), N,
                              _ptr(ss[0]), _ptr(ss[1]), _ptr(ss[2]), int(isign), _ptr(out),
                              nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_type3: bad arguments")
    return out


def rel_l2(approx, exact) -> float:
    """Relative l2 error ||approx - exact|| / ||exact|| (Sec. 4.2)."""
    a = np.asarray(approx, dtype=np.complex128).reshape(-1)
    e = np.asarray(exact, dtype=np.complex128).reshape(-1)
    return float(np.linalg.norm(a - e) / np.linalg.norm(e))


def rel_l2_interval(approx, exact, nboot: int = 1000, seed: int = 0, level: float = 0.95):
    """Relative l2 error on a sample of outputs with a bootstrap interval: the
    sampled outputs are resampled with replacement nboot times and the error
    recomputed; returns (error, low, high) with [low, high] the central
    `level` range of the resampled errors."""
    a = np.asarray(approx, dtype=np.complex128).reshape(-1)
    e = np.asarray(exact, dtype=np.complex128).reshape(-1)
    d2 = np.abs(a - e) ** 2
    e2 = np.abs(e) ** 2
    g = np.random.default_rng(seed)
    idx = g.integers(0, a.size, size=(nboot, a.size))
    errs = np.sqrt(d2[idx].sum(axis=1) / e2[idx].sum(axis=1))
    lo, hi = np.quantile(errs, [(1 - level) / 2, (1 + level) / 2])
    return float(np.sqrt(d2.sum() / e2.sum())), float(lo), float(hi)
