"""GPU tests of the serving loop (continuous batching over worker streams)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1808_06736_amd import binding as B
from paper_1808_06736_amd import inputs as I
from tests.gpu_helpers import dev, host, torch

pytestmark = pytest.mark.gpu


def _request_data(wl, scale=20, cap=200_000):
    """Seeded data of a serving-mix request, with M scaled down for the test."""
    M = max(1, min(cap, wl.M // scale))
    small = I.Workload(wl.name, wl.dim, wl.types, wl.N, M, wl.eps, wl.prec, wl.points,
                       seed=wl.seed)
    coords = small.coords()
    dt = np.complex64 if wl.prec == "f32" else np.complex128
    c = I.complex_normal(M, wl.seed + 1, dt)
    f = I.complex_normal(tuple(reversed(wl.N[:wl.dim])), wl.seed + 2, dt)
    return small, coords, c, f


def _alone(wl, coords, c, f):
    t = torch()
    p = B.Plan(wl.types[0], wl.N[:wl.dim], wl.eps,
               dtype=t.complex64 if wl.prec == "f32" else t.complex128)
    p.setpts(*[dev(a) for a in coords])
    if wl.types[0] == 1:
        out = host(p.type1(dev(c)))
    else:
        out = host(p.type2(dev(f)))
    p.close()
    return out


def test_mix_results_equal_alone_and_oracle():
    """Requests of mixed type, dimension, size and tolerance, all in flight at
    once on 4 worker streams: each result equals the same request run alone,
    and a sample of them meets the oracle bar."""
    reqs = I.serve_mix(24, seed=7)
    srv = B.Server(nslots=4, hbm_budget_bytes=32 << 30)
    t = torch()
    jobs = []
    for wl in reqs:
        small, coords, c, f = _request_data(wl)
        xs = [dev(a) for a in coords]
        cd = dev(c) if wl.types[0] == 1 else t.empty(small.M, dtype=dev(c).dtype, device="cuda")
        fd = dev(f) if wl.types[0] == 2 else t.empty(f.shape, dtype=dev(f).dtype, device="cuda")
        tk = srv.submit(wl.types[0], xs, cd, fd, wl.eps)
        jobs.append((small, coords, c, f, cd, fd, tk))
    for k, (small, coords, c, f, cd, fd, tk) in enumerate(jobs):
        st, lat = srv.wait(tk)
        assert st in (0, 1), (k, st)
        got = host(fd) if small.types[0] == 1 else host(cd)
        ref = _alone(small, coords, c, f)
        tol = 1e-5 if small.prec == "f32" else 1e-12
        assert O.rel_l2(got, ref) < tol, (k, small)
        if k % 6 == 0:
            if small.types[0] == 1:
                N = small.N[:small.dim]
                modes = [I.sample_modes(n, 6, seed=9 + m) for m, n in enumerate(N)]
                orc = O.type1(coords, c, +1, modes=modes)
                idx = np.ix_(*[m + n // 2 for m, n in zip(reversed(modes), reversed(N))])
                err = O.rel_l2(got[idx], orc)
            else:
                sel = I.sample_points(coords, 256, seed=11)
                err = O.rel_l2(got[sel], O.type2([a[sel] for a in coords], f, -1))
            assert err <= 10 * small.eps, (k, err, small.eps)
    s = srv.stats()
    print(f"served {s.completed}: p50 {s.p50_ms:.2f} ms p99 {s.p99_ms:.2f} ms, "
          f"plan hits {s.plan_cache_hits} misses {s.plan_cache_misses}, peak HBM {s.hbm_peak / 2**20:.0f} MiB")
    assert s.completed == len(reqs) and s.failed == 0
    assert s.p50_ms <= s.p99_ms
    srv.close()


def test_budget_rejects_and_queues():
    t = torch()
    N = (96, 80)
    M = 50000
    coords = I.uniform_points(M, 2, 21, np.float32)
    c = I.complex_normal(M, 22, np.complex64)
    xs = [dev(a) for a in coords]
    # a budget far below one request: rejected, nothing hangs
    srv = B.Server(nslots=2, hbm_budget_bytes=1 << 20)
    f = t.empty((80, 96), dtype=t.complex64, device="cuda")
    tk = srv.submit(1, xs, dev(c), f, 1e-5)
    st, _ = srv.wait(tk)
    assert st == B.ESN_ERR_BUDGET
    srv.close()
    # a budget for about one request at a time: all complete, one after another
    srv = B.Server(nslots=4, hbm_budget_bytes=40 << 20)
    outs, tks = [], []
    for k in range(6):
        f = t.empty((80, 96), dtype=t.complex64, device="cuda")
        tks.append(srv.submit(1, xs, dev(c), f, 1e-5))
        outs.append(f)
    for tk in tks:
        st, _ = srv.wait(tk)
        assert st == 0
    s = srv.stats()
    assert s.completed == 6
    ref = O.type1(coords, c, +1, N=N)
    for f in outs:
        assert O.rel_l2(host(f), ref) <= 1e-4
    srv.close()


def test_point_cache_and_failure_isolation():
    t = torch()
    N = (40, 36, 32)
    M = 30000
    coords = I.wrapped_gaussian_points(M, 3, 31, 0.3, np.float32)
    xs = [dev(a) for a in coords]
    srv = B.Server(nslots=2, hbm_budget_bytes=8 << 30)
    c1 = I.complex_normal(M, 32, np.complex64)
    c2 = I.complex_normal(M, 33, np.complex64)
    f1 = t.empty((32, 36, 40), dtype=t.complex64, device="cuda")
    f2 = t.empty((32, 36, 40), dtype=t.complex64, device="cuda")
    st, _ = srv.wait(srv.submit(1, xs, dev(c1), f1, 1e-6, points_id=77))
    assert st == 0
    st, _ = srv.wait(srv.submit(1, xs, dev(c2), f2, 1e-6, points_id=77))
    assert st == 0
    s = srv.stats()
    assert s.point_cache_hits == 1 and s.plan_cache_hits == 1
    assert O.rel_l2(host(f2), O.type1(coords, c2, +1, N=N)) <= 1e-5
    # a request with a NaN coordinate fails alone
    bad = [a.clone() for a in xs]
    bad[0][5] = float("nan")
    f3 = t.empty((32, 36, 40), dtype=t.complex64, device="cuda")
    f4 = t.empty((32, 36, 40), dtype=t.complex64, device="cuda")
    tb = srv.submit(1, bad, dev(c1), f3, 1e-6)
    tg = srv.submit(1, xs, dev(c1), f4, 1e-6, points_id=77)
    assert srv.wait(tb)[0] == B.ESN_ERR_NAN_PTS
    assert srv.wait(tg)[0] == 0
    assert O.rel_l2(host(f4), O.type1(coords, c1, +1, N=N)) <= 1e-5
    srv.close()


def _oracle_sample(wl, coords, c, f, got, seed):
    """Oracle relative error (with its bootstrap interval) of a request result
    on 256 sampled outputs: a product grid of modes (16 x 16 in 2D, 8 x 8 x 4
    in 3D, always with the lowest, zero and highest mode) for type 1, 256
    points for type 2."""
    N = wl.N[:wl.dim]
    if wl.types[0] == 1:
        per = (16, 16) if wl.dim == 2 else (8, 8, 4)
        modes = [I.sample_modes(n, s, seed=seed + m) for m, (n, s) in enumerate(zip(N, per))]
        orc = O.type1(coords, c, +1, modes=modes)
        idx = np.ix_(*[m + n // 2 for m, n in zip(reversed(modes), reversed(N))])
        return O.rel_l2_interval(got[idx], orc, seed=seed)
    sel = I.sample_points(coords, 256, seed=seed)
    return O.rel_l2_interval(got[sel], O.type2([a[sel] for a in coords], f, -1), seed=seed)


def test_mix_at_full_size_every_request_against_oracle():
    """Sixteen serving-mix requests at their own sizes (M from 1e5 to 5e6, so
    both the counting and the radix sort run, in FP32 and FP64, 2D and 3D,
    both types, all three tolerances), all submitted at once to 4 worker
    streams: every result meets the oracle bar on 256 sampled outputs and
    equals the same request run alone."""
    reqs = I.serve_mix(16, seed=28)
    assert {(r.types[0], r.dim) for r in reqs if r.M >= (1 << 21)} == {(1, 2), (1, 3), (2, 2), (2, 3)}
    assert {r.eps for r in reqs} == {1e-3, 1e-6, 1e-9}
    t = torch()
    srv = B.Server(nslots=4, hbm_budget_bytes=64 << 30)
    jobs = []
    for wl in reqs:
        coords = wl.coords()
        dt = np.complex64 if wl.prec == "f32" else np.complex128
        c = I.complex_normal(wl.M, wl.seed + 1, dt)
        f = I.complex_normal(tuple(reversed(wl.N[:wl.dim])), wl.seed + 2, dt)
        xs = [dev(a) for a in coords]
        cd = dev(c) if wl.types[0] == 1 else t.empty(wl.M, dtype=dev(c[:1]).dtype, device="cuda")
        fd = dev(f) if wl.types[0] == 2 else t.empty(f.shape, dtype=dev(f[:1]).dtype, device="cuda")
        jobs.append((wl, coords, c, f, cd, fd, srv.submit(wl.types[0], xs, cd, fd, wl.eps)))
    for k, (wl, coords, c, f, cd, fd, tk) in enumerate(jobs):
        st, lat = srv.wait(tk)
        assert st in (0, 1), (k, st)
        got = host(fd) if wl.types[0] == 1 else host(cd)
        err, lo, hi = _oracle_sample(wl, coords, c, f, got, seed=100 + k)
        print(f"request {k}: type {wl.types[0]} dim {wl.dim} N {wl.N[:wl.dim]} M {wl.M} "
              f"eps {wl.eps:g} {wl.prec}: oracle rel l2 {err:.2e} [{lo:.2e}, {hi:.2e}] "
              f"latency {lat:.1f} ms", flush=True)
        assert err <= 10 * wl.eps, (k, err, wl.eps)
        ref = _alone(wl, coords, c, f)
        tol = 1e-5 if wl.prec == "f32" else 1e-12
        assert O.rel_l2(got, ref) < tol, (k, wl)
    s = srv.stats()
    assert s.completed == len(reqs) and s.failed == 0
    srv.close()


def test_inputs_written_by_queued_work_are_complete():
    """Inputs written by work still queued on the caller's stream when the
    request is submitted (no synchronisation in between) are read only after
    that work: the served result equals the result computed afterwards from
    the finished inputs."""
    t = torch()
    N = (64, 48, 40)
    M = 300_000
    coords = I.wrapped_gaussian_points(M, 3, 71, 0.3, np.float32)
    c = I.complex_normal(M, 72, np.complex64)
    srv = B.Server(nslots=2, hbm_budget_bytes=8 << 30)
    side = t.cuda.Stream()
    src = [dev(a) for a in coords] + [dev(c)]
    t.cuda.synchronize()
    with t.cuda.stream(side):
        xs = [t.zeros(M, dtype=t.float32, device="cuda") for _ in range(3)]
        cd = t.zeros(M, dtype=t.complex64, device="cuda")
        a = t.rand(2048, 2048, device="cuda")
        for _ in range(40):                 # work queued ahead of the writes below
            a = t.tanh(a @ a)
        for dst, s in zip(xs + [cd], src):
            dst.copy_(s)
        fd = t.empty((40, 48, 64), dtype=t.complex64, device="cuda")
        tk = srv.submit(1, xs, cd, fd, 1e-6)
    st, _ = srv.wait(tk)
    assert st == 0
    t.cuda.synchronize()
    ref = _alone(I.Workload("q", 3, (1,), N, M, 1e-6, "f32", "wrapped_gaussian"),
                 coords, c, None)
    assert O.rel_l2(host(fd), ref) < 1e-5
    srv.close()
