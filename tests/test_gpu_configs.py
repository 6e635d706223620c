"""GPU parity at the full sizes of the named workloads, on seeded oracle samples.

Bar: relative l2 error <= 10 eps on the sample.  Type 1 samples a product set
of mode indices (always with min, 0 and max per dimension); type 2 samples
points (always with each coordinate's smallest and largest point).  The GPU runs
in exactly the configuration bench.py times (default options, full M).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1808_06736_amd import inputs as I
from tests.gpu_helpers import cdtype, dev, host, torch

pytestmark = pytest.mark.gpu


def _plan(t, wl, **opts):
    from paper_1808_06736_amd import binding as B
    return B.Plan(t, wl.N[:wl.dim], wl.eps, dtype=cdtype(wl.prec), ntransf=wl.ntransf, **opts)


def _check_type1(wl, coords, c, f_gpu, per_dim):
    N = wl.N[:wl.dim]
    modes = [I.sample_modes(n, per_dim, seed=51 + m) for m, n in enumerate(N)]
    ref = O.type1(coords, c, +1, modes=modes)
    idx = np.ix_(*[m + n // 2 for m, n in zip(reversed(modes), reversed(N))])
    return O.rel_l2(f_gpu[idx], ref)


def _check_type2(wl, coords, f, c_gpu, npts):
    sel = I.sample_points(coords, npts, seed=53)
    ref = O.type2([a[sel] for a in coords], f, -1)
    return O.rel_l2(c_gpu[sel], ref)


@pytest.mark.parametrize("name", ["2d_f32", "2d_f64", "3d_clustered"])
def test_full_size_type1(name):
    wl = I.WORKLOADS[name]
    coords = wl.coords()
    c = wl.strengths()
    p = _plan(1, wl)
    p.setpts(*[dev(a) for a in coords])
    f = host(p.type1(dev(c)))
    torch().cuda.synchronize()
    info = p.info()
    p.close()
    err = _check_type1(wl, coords, c, f, 32 if wl.dim == 2 else 12)
    print(f"{name} type 1: rel l2 {err:.3e} (w {info.w}, method {info.spread_method}, "
          f"subproblems {info.nsubprob})")
    assert err <= 10 * wl.eps


@pytest.mark.parametrize("name", ["2d_f32", "2d_f64", "3d_clustered"])
def test_full_size_type2(name):
    wl = I.WORKLOADS[name]
    coords = wl.coords()
    f = wl.coefficients()
    p = _plan(2, wl)
    p.setpts(*[dev(a) for a in coords])
    c = host(p.type2(dev(f)))
    torch().cuda.synchronize()
    info = p.info()
    p.close()
    err = _check_type2(wl, coords, f, c, 1024)
    print(f"{name} type 2: rel l2 {err:.3e} (w {info.w}, method {info.interp_method})")
    assert err <= 10 * wl.eps


def test_batched_radial_type2():
    """32 coefficient vectors on one radial point set (400 spokes x 512 radii),
    eps 1e-4: every vector meets the bar, and the fused batch equals running
    each vector alone."""
    wl = I.WORKLOADS["2d_t2_batched_radial"]
    coords = wl.coords()
    f = wl.coefficients()                       # (32, 256, 256)
    p = _plan(2, wl)
    p.setpts(*[dev(a) for a in coords])
    cb = host(p.type2(dev(f)))                   # (32, M)
    info = p.info()
    print(f"batched: chunk {info.ntransf_chunk}, method {info.interp_method}")
    p.close()
    sel = I.sample_points(coords, 1024, seed=55)
    errs = []
    for t in range(wl.ntransf):
        ref = O.type2([a[sel] for a in coords], f[t], -1)
        errs.append(O.rel_l2(cb[t][sel], ref))
    print(f"batched radial: max rel l2 over 32 vectors {max(errs):.3e}")
    assert max(errs) <= 10 * wl.eps
    from paper_1808_06736_amd import binding as B
    single = B.Plan(2, wl.N[:2], wl.eps, dtype=cdtype(wl.prec))
    single.setpts(*[dev(a) for a in coords])
    for t in (0, 17, 31):
        c1 = host(single.type2(dev(f[t])))
        assert O.rel_l2(cb[t], c1) < 1e-6
    single.close()


def test_headline_step_one_plan_type1_and_adjoint():
    """The timed step of the headline workload exactly as it runs in the
    benchmark: one type 1 plan (default options, debug timing on), one setpts,
    execute (type 1, isign +1) and execute_adjoint (type 2, isign -1) on the
    same sorted points.  Both outputs meet the bar on the oracle samples; the
    sampled errors are printed with bootstrap 95% intervals."""
    wl = I.WORKLOADS["3d_clustered"]
    coords = wl.coords()
    c = wl.strengths()
    f = wl.coefficients()
    p = _plan(1, wl, debug=1)
    p.setpts(*[dev(a) for a in coords])
    f_out = torch().empty(f.shape, dtype=cdtype(wl.prec), device="cuda")
    c_out = torch().empty(c.shape, dtype=cdtype(wl.prec), device="cuda")
    p.execute(dev(c), f_out)
    p.execute_adjoint(c_out, dev(f))
    torch().cuda.synchronize()
    info = p.info()
    f_gpu, c_gpu = host(f_out), host(c_out)
    p.close()
    N = wl.N[:wl.dim]
    modes = [I.sample_modes(n, 12, seed=61 + m) for m, n in enumerate(N)]
    idx = np.ix_(*[m + n // 2 for m, n in zip(reversed(modes), reversed(N))])
    e1 = O.rel_l2_interval(f_gpu[idx], O.type1(coords, c, +1, modes=modes), seed=1)
    sel = I.sample_points(coords, 1024, seed=63)
    e2 = O.rel_l2_interval(c_gpu[sel], O.type2([a[sel] for a in coords], f, -1), seed=2)
    print(f"headline step: type 1 rel l2 {e1[0]:.3e} [{e1[1]:.3e}, {e1[2]:.3e}], adjoint "
          f"(type 2) rel l2 {e2[0]:.3e} [{e2[1]:.3e}, {e2[2]:.3e}] (methods "
          f"{info.spread_method}/{info.interp_method}, subproblems {info.nsubprob})")
    assert e1[0] <= 10 * wl.eps and e2[0] <= 10 * wl.eps


def test_clustered_3d_batch_of_eight_on_matrix_cores():
    """Eight strength vectors on one clustered point set (1e6 points, 64^3
    modes, eps 1e-6; the headline's distribution at a size the oracle samples
    quickly): the batched execute runs on the matrix cores, every vector
    equals the same vector run alone on the same sorted points, and vectors 0
    and 7 meet the oracle bar on sampled modes."""
    N = (64, 64, 64)
    M = 1_000_000
    eps = 1e-6
    coords = I.wrapped_gaussian_points(M, 3, 401, 0.3, np.float32)
    c = I.complex_normal((8, M), 402, np.complex64)
    t = torch()
    from paper_1808_06736_amd import binding as B
    pb = B.Plan(1, N, eps, dtype=t.complex64, ntransf=8)
    pb.setpts(*[dev(a) for a in coords])
    info = pb.info()
    assert info.spread_method == 3
    fb = host(pb.type1(dev(c)))
    pb.close()
    p1 = B.Plan(1, N, eps, dtype=t.complex64)
    p1.setpts(*[dev(a) for a in coords])
    for k in range(8):
        one = host(p1.type1(dev(c[k])))
        assert O.rel_l2(fb[k], one) < 1e-5, k
    p1.close()
    modes = [I.sample_modes(n, 8, seed=405 + m) for m, n in enumerate(N)]
    idx = np.ix_(*[m + n // 2 for m, n in zip(reversed(modes), reversed(N))])
    for k in (0, 7):
        err, lo, hi = O.rel_l2_interval(fb[k][idx], O.type1(coords, c[k], +1, modes=modes), seed=k)
        print(f"batch of 8, vector {k}: rel l2 {err:.3e} [{lo:.3e}, {hi:.3e}]")
        assert err <= 10 * eps
