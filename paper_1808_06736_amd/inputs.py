"""Seeded synthetic inputs for the NUFFT workloads.

This module only draws random numbers and lays out index samples.  It holds
none of the transform's arithmetic, so both the GPU path's tests/benchmarks and
the CPU oracle's tests can use it without sharing any of the method.

Workloads (point distributions follow the paper's performance tests, Sec. 6
"Tasks": iid uniform points in 1D/2D/3D, radial "disc quad"-like sets whose
density diverges at the origin, and complex Gaussian strengths):

* ``uniform_points``          iid U[-pi, pi)^d
* ``wrapped_gaussian_points`` each coordinate iid N(0, s^2), wrapped into [-pi, pi)
* ``radial_spokes``           spokes at uniform angles x uniformly spaced radii
* ``complex_normal``          re, im iid N(0, 1)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * math.pi


def rng(seed: int) -> np.random.Generator:
    """numpy PCG64 generator for a seed (the recipe every workload uses)."""
    return np.random.Generator(np.random.PCG64(seed))


def uniform_points(M: int, d: int, seed: int, dtype=np.float64):
    """d arrays of M coordinates iid uniform in [-pi, pi)."""
    g = rng(seed)
    return [g.uniform(-math.pi, math.pi, size=M).astype(dtype) for _ in range(d)]


def _wrap(a: np.ndarray) -> np.ndarray:
    """Wrap real numbers into [-pi, pi)."""
    return a - TWO_PI * np.floor((a + math.pi) / TWO_PI)


def wrapped_gaussian_points(M: int, d: int, seed: int, sigma: float = 0.3,
                            dtype=np.float64):
    """d arrays of M coordinates iid N(0, sigma^2) wrapped into [-pi, pi)."""
    g = rng(seed)
    out = []
    for _ in range(d):
        a = _wrap(g.normal(0.0, sigma, size=M))
        a = a.astype(dtype)
        # rounding to float32 can land exactly on +pi; keep the half-open range
        a[a >= math.pi] = -math.pi
        out.append(a)
    return out


def radial_spokes(nspokes: int = 400, nrad: int = 512, dtype=np.float64):
    """Polar sample set: angles pi*s/nspokes, radii -pi + 2*pi*m/nrad.

    Points are ordered spoke-major (all radii of spoke 0 first).  M =
    nspokes*nrad; every spoke passes through the origin once (m = nrad/2).
    """
    s = np.arange(nspokes, dtype=np.float64)
    m = np.arange(nrad, dtype=np.float64)
    th = math.pi * s / nspokes
    r = -math.pi + TWO_PI * m / nrad
    x = (r[None, :] * np.cos(th)[:, None]).reshape(-1)
    y = (r[None, :] * np.sin(th)[:, None]).reshape(-1)
    return [x.astype(dtype), y.astype(dtype)]


def complex_normal(shape, seed: int, dtype=np.complex128) -> np.ndarray:
    """Complex array with re, im iid N(0, 1)."""
    g = rng(seed)
    re = g.standard_normal(size=shape)
    im = g.standard_normal(size=shape)
    return (re + 1j * im).astype(dtype)


def device_points(M: int, d: int, seed: int, kind: str = "uniform", sigma: float = 0.3,
                  dtype=None):
    """d coordinate tensors on the GPU from torch's seeded CUDA generator (for
    large benchmark inputs that no oracle reads): iid U[-pi, pi), or iid
    N(0, sigma^2) wrapped into [-pi, pi)."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    dtype = dtype or torch.float32
    out = []
    for _ in range(d):
        if kind == "uniform":
            a = (torch.rand(M, generator=g, device="cuda", dtype=torch.float64) * 2 - 1) * math.pi
        else:
            a = torch.randn(M, generator=g, device="cuda", dtype=torch.float64) * sigma
            a = a - TWO_PI * torch.floor((a + math.pi) / TWO_PI)
        a = a.to(dtype)
        a[a >= math.pi] = -math.pi
        out.append(a.contiguous())
    return out


def device_complex(shape, seed: int, dtype=None):
    """Complex tensor on the GPU with re, im iid N(0, 1) (torch seeded generator)."""
    import torch
    dtype = dtype or torch.complex64
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    real = torch.float32 if dtype == torch.complex64 else torch.float64
    re = torch.randn(shape, generator=g, device="cuda", dtype=real)
    im = torch.randn(shape, generator=g, device="cuda", dtype=real)
    return torch.complex(re, im).contiguous()


def mode_range(N: int) -> np.ndarray:
    """Integer mode indices of one dimension, in increasing order."""
    return np.arange(N, dtype=np.int64) - (N // 2)


def sample_modes(N: int, count: int, seed: int) -> np.ndarray:
    """Sorted seeded subset of one dimension's mode indices.

    Always contains the smallest, zero and the largest index; ``count`` is
    clipped to N (then every index is returned).
    """
    k = mode_range(N)
    if count >= N:
        return k
    g = rng(seed)
    must = {int(k[0]), 0, int(k[-1])}
    rest = np.array([v for v in k if int(v) not in must], dtype=np.int64)
    pick = g.choice(rest, size=max(0, count - len(must)), replace=False)
    return np.sort(np.concatenate([np.array(sorted(must), dtype=np.int64), pick]))


def sample_points(coords, count: int, seed: int) -> np.ndarray:
    """Sorted seeded subset of point indices, including each coordinate's
    smallest and largest point."""
    M = len(coords[0])
    if count >= M:
        return np.arange(M, dtype=np.int64)
    must = set()
    for a in coords:
        must.add(int(np.argmin(a)))
        must.add(int(np.argmax(a)))
    g = rng(seed)
    pick = g.choice(M, size=count, replace=False)
    idx = np.unique(np.concatenate([pick, np.array(sorted(must), dtype=np.int64)]))
    return idx.astype(np.int64)


@dataclass
class Workload:
    """One named transform configuration with its input recipe."""
    name: str
    dim: int
    types: tuple
    N: tuple
    M: int
    eps: float
    prec: str                 # "f32" or "f64": dtype of strengths / coefficients
    points: str               # "uniform", "wrapped_gaussian", "radial"
    ntransf: int = 1
    seed: int = 0
    extra: dict = field(default_factory=dict)

    def coords(self, dtype=None):
        dt = dtype or (np.float32 if self.prec == "f32" else np.float64)
        if self.points == "uniform":
            return uniform_points(self.M, self.dim, self.seed, dt)
        if self.points == "wrapped_gaussian":
            return wrapped_gaussian_points(self.M, self.dim, self.seed,
                                           self.extra.get("sigma", 0.3), dt)
        if self.points == "radial":
            return radial_spokes(self.extra.get("nspokes", 400),
                                 self.extra.get("nrad", 512), dt)
        raise ValueError(self.points)

    def strengths(self):
        dt = np.complex64 if self.prec == "f32" else np.complex128
        shape = (self.ntransf, self.M) if self.ntransf > 1 else (self.M,)
        return complex_normal(shape, self.seed + 1000, dt)

    def targets(self, dtype=None):
        """Type 3 target frequencies: iid uniform in [-S, S)^d (extra['S'],
        extra['targets'] of them)."""
        dt = dtype or (np.float32 if self.prec == "f32" else np.float64)
        g = rng(self.seed + 3000)
        S = float(self.extra["S"])
        return [g.uniform(-S, S, int(self.extra["targets"])).astype(dt) for _ in range(self.dim)]

    def coefficients(self):
        dt = np.complex64 if self.prec == "f32" else np.complex128
        Nrev = tuple(reversed(self.N[: self.dim]))        # slowest first
        shape = ((self.ntransf,) + Nrev) if self.ntransf > 1 else Nrev
        return complex_normal(shape, self.seed + 2000, dt)


# The named workloads: a small 1D case, the large 2D and 3D cases, a 3D type 3
# case, the batched radial 2D case.  (The serving mix draws its requests in serve_mix below.)
WORKLOADS = {
    "1d_t1_small": Workload("1d_t1_small", 1, (1,), (1000, 1, 1), 10_000, 1e-6,
                            "f64", "uniform", seed=1),
    "2d_f32": Workload("2d_f32", 2, (1, 2), (1000, 1000, 1), 10_000_000, 1e-5,
                       "f32", "uniform", seed=2),
    "2d_f64": Workload("2d_f64", 2, (1, 2), (1000, 1000, 1), 10_000_000, 1e-9,
                       "f64", "uniform", seed=2),
    "3d_clustered": Workload("3d_clustered", 3, (1, 2), (128, 128, 128),
                             10_000_000, 1e-6, "f32", "wrapped_gaussian", seed=3,
                             extra={"sigma": 0.3}),
    # type 3: sources iid uniform in [-pi, pi)^3, target frequencies iid uniform
    # in [-32, 32)^3 (space-frequency product X S = 32 pi per dimension)
    "3d_type3": Workload("3d_type3", 3, (3,), (1, 1, 1), 10_000_000, 1e-6, "f32",
                         "uniform", seed=6, extra={"targets": 10_000_000, "S": 32.0}),
    "2d_t2_batched_radial": Workload("2d_t2_batched_radial", 2, (2,),
                                     (256, 256, 1), 400 * 512, 1e-4, "f32",
                                     "radial", ntransf=32, seed=4,
                                     extra={"nspokes": 400, "nrad": 512, "autotune": True}),
}


def serve_mix(nreq: int, seed: int = 5):
    """Request descriptors of the serving mix (no data; data is drawn per request).

    type U{1,2}; d U{2,3}; N_i integer-uniform in [64,512] (2D) or [64,160]
    (3D); M log-uniform in [1e5, 5e6]; points uniform or wrapped Gaussian
    (s=0.3) with equal probability; eps U{1e-3 (f32), 1e-6 (f32), 1e-9 (f64)}.
    """
    g = rng(seed)
    reqs = []
    for r in range(nreq):
        t = int(g.integers(1, 3))
        d = int(g.integers(2, 4))
        hi = 512 if d == 2 else 160
        N = [int(g.integers(64, hi + 1)) for _ in range(d)] + [1] * (3 - d)
        M = int(round(10 ** g.uniform(5.0, math.log10(5e6))))
        pts = "uniform" if g.integers(0, 2) == 0 else "wrapped_gaussian"
        e = int(g.integers(0, 3))
        eps, prec = [(1e-3, "f32"), (1e-6, "f32"), (1e-9, "f64")][e]
        reqs.append(Workload(f"req{r}", d, (t,), tuple(N), M, eps, prec, pts,
                             seed=10_000 + r))
    return reqs
