"""Autotuner for the plan options that only change speed.

Bin size, subproblem size (Sec. 5.1, 5.2), the spreading / interpolation method
and the number of vectors fused per launch do not change the result beyond
rounding, only the time.  ``tune`` times a small candidate set on the caller's
actual points (execute only, best of a few runs, after a warm-up) and returns
the fastest options; results are cached in a JSON file keyed by the problem
class (type, dim, precision, kernel width, fine-grid size and point-density
buckets, ntransf), so a later plan of the same class skips the search.

Everything runs through the C ABI (binding.Plan); nothing here computes a
transform.
"""
from __future__ import annotations

import json
import math
import os
import time

from . import binding as B

CACHE_ENV = "ESN_TUNE_CACHE"


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(
        os.path.expanduser("~"), ".cache", "esnufft", "tune.json")


def _bucket(v: float) -> int:
    """Power-of-two bucket of a positive number."""
    return int(round(math.log2(max(v, 1e-9))))


def problem_key(type_, N, eps, prec, ntransf, M) -> str:
    dim = len(N)
    st, par = B.esn_choose_params(eps, prec, dim, N)
    nf = [int(par.nf[m]) for m in range(dim)]
    density = M / math.prod(nf)
    return (f"t{type_}-d{dim}-p{prec}-w{par.w}-n{'x'.join(str(_bucket(n)) for n in nf)}"
            f"-rho{_bucket(density)}-nt{ntransf}")


def candidates(type_, dim, prec, w, ntransf):
    """Candidate option dicts (bin, maxsubprob, method, ntransf_chunk)."""
    out = []
    chunks = [0] if ntransf == 1 else sorted({0, 1, 4, 8, 16, 32, ntransf} & set(range(ntransf + 1)))
    mkey = "spread_method" if type_ == 1 else "interp_method"
    if dim == 1:
        bins = [(256,), (1024,), (4096,)]
    elif dim == 2:
        bins = [(8, 8), (16, 8), (16, 16), (32, 32)]
    else:
        bins = [(4, 4, 4), (8, 8, 8)]
    for b in bins:
        for ms in (1024, 4096):
            for ch in chunks:
                out.append({"bin": b, "maxsubprob": ms, "ntransf_chunk": ch, mkey: 1})
    if dim == 3 and prec == B.ESN_SINGLE and w <= 7:
        # matrix-core kernels: bins of even sizes (2 x 2 column blocks)
        for b in ((4, 4, 4), (8, 4, 4), (8, 8, 4), (16, 8, 8)):
            for ms in (512, 1024, 2048):
                out.append({"bin": b, "maxsubprob": ms, mkey: 3})
    return out


def _time_plan(type_, N, eps, dtype, ntransf, coords, data, opts, reps):
    import torch
    p = B.Plan(type_, N, eps, dtype=dtype, ntransf=ntransf, **opts)
    try:
        p.setpts(*coords)
        if type_ == 1:
            out = torch.empty(p._shape_f(), dtype=dtype, device=p.device)
            run = lambda: p.execute(data, out)
        else:
            out = torch.empty(p._shape_c(), dtype=dtype, device=p.device)
            run = lambda: p.execute(out, data)
        run()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return best
    finally:
        p.close()


def tune(type_, N, eps, coords, data, dtype=None, ntransf=1, reps=3, use_cache=True,
         verbose=False):
    """Fastest option set for this problem, from the cache or by timing.

    ``coords``: the device coordinate tensors; ``data``: the input of execute
    (strengths c for type 1, coefficients f for type 2).  Returns (opts dict,
    seconds per execute or None when taken from the cache).
    """
    import torch
    dtype = dtype or torch.complex64
    prec = B.ESN_SINGLE if dtype == torch.complex64 else B.ESN_DOUBLE
    M = coords[0].numel()
    key = problem_key(type_, tuple(N), eps, prec, ntransf, M)
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        opts = dict(cache[key]["opts"])
        if "bin" in opts:
            opts["bin"] = tuple(opts["bin"])
        return opts, None
    st, par = B.esn_choose_params(eps, prec, len(N), N)
    best, best_t = None, float("inf")
    for opts in candidates(type_, len(N), prec, par.w, ntransf):
        try:
            t = _time_plan(type_, tuple(N), eps, dtype, ntransf, coords, data, opts, reps)
        except B.EsnError:
            continue          # e.g. a fused chunk that does not fit in LDS
        if verbose:
            print(f"autotune {key}: {opts} -> {1e3 * t:.3f} ms")
        if t < best_t:
            best, best_t = opts, t
    if best is None:
        return {}, None
    if use_cache:
        cache[key] = {"opts": best, "ms": 1e3 * best_t}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".tmp{os.getpid()}"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, path)
    return best, best_t
