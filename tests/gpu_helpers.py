"""Helpers for the GPU tests: move seeded numpy inputs to the GPU, run the HIP
library through the binding, and bring results back for the oracle."""
import numpy as np

from paper_1808_06736_amd import binding as B


def torch():
    import torch as t
    return t


def dev(a):
    t = torch()
    return t.from_numpy(np.ascontiguousarray(a)).cuda()


def host(x):
    return x.detach().cpu().numpy()


def cdtype(prec):
    t = torch()
    return t.complex64 if prec == "f32" else t.complex128


def coord_np(coords, prec):
    dt = np.float32 if prec == "f32" else np.float64
    return [np.ascontiguousarray(np.asarray(a, dtype=dt)) for a in coords]


def run_type1(coords, c, N, eps, prec, isign=1, ntransf=1, **opts):
    """GPU type 1; returns (f as numpy with shape (.., N_d, .., N_1), plan info)."""
    t = torch()
    plan = B.Plan(1, N, eps, dtype=cdtype(prec), isign=isign, ntransf=ntransf, **opts)
    plan.setpts(*[dev(a) for a in coords])
    f = plan.type1(dev(c))
    t.cuda.synchronize()
    info = plan.info()
    plan.close()
    return host(f), info


def run_type2(coords, f, N, eps, prec, isign=-1, ntransf=1, **opts):
    t = torch()
    plan = B.Plan(2, N, eps, dtype=cdtype(prec), isign=isign, ntransf=ntransf, **opts)
    plan.setpts(*[dev(a) for a in coords])
    c = plan.type2(dev(f))
    t.cuda.synchronize()
    info = plan.info()
    plan.close()
    return host(c), info
