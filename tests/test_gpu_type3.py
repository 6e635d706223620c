"""GPU parity of the type 3 transform (eq. (3), Sec. 3.3) with the FP64 oracle.

Bar: rel. l2 error <= 10 eps (the paper reports errors close to eps with the
same eps in the spreading and type 2 steps; Sec. 3.3 remark on tolerances).
Sources and targets are seeded and synthetic: iid uniform in boxes (centred or
not) and clusters, with space-frequency products X S that give fine grids of
tens to a few hundred points per dimension.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1808_06736_amd import binding as B
from paper_1808_06736_amd import inputs as I
from tests.gpu_helpers import cdtype, dev, host, run_type1, torch

pytestmark = pytest.mark.gpu


def _box(n, d, seed, lo, hi, dt):
    rng = np.random.default_rng(seed)
    return [rng.uniform(lo[m], hi[m], n).astype(dt) for m in range(d)]


def run_type3(xs, c, ss, eps, prec, isign=1, ntransf=1, **opts):
    t = torch()
    p = B.Plan3(len(xs), eps, dtype=cdtype(prec), isign=isign, ntransf=ntransf, **opts)
    p.setpts([dev(a) for a in xs], [dev(a) for a in ss])
    f = p.execute(dev(c))
    t.cuda.synchronize()
    info = p.info()
    p.close()
    return host(f), info


CASES = [
    # dim, M, N, source box, target box, prec, eps
    (1, 3000, 2500, ([-3.0], [3.0]), ([-200.0], [200.0]), "f64", 1e-12),
    (1, 3000, 2500, ([-1.0], [9.0]), ([50.0], [700.0]), "f32", 1e-6),
    (2, 4000, 3000, ([-2.0, -1.0], [2.0, 5.0]), ([-40.0, -60.0], [80.0, 60.0]), "f64", 1e-9),
    (2, 4000, 3000, ([0.0, 0.0], [6.0, 6.0]), ([-30.0, -30.0], [30.0, 30.0]), "f32", 1e-5),
    (3, 5000, 2000, ([-1.0] * 3, [1.0] * 3), ([-30.0, -20.0, -25.0], [30.0, 20.0, 25.0]), "f32", 1e-6),
    (3, 5000, 2000, ([2.0, -3.0, 0.0], [4.0, -1.0, 1.5]), ([-15.0] * 3, [40.0] * 3), "f64", 1e-9),
    (3, 5000, 2000, ([-1.0] * 3, [1.0] * 3), ([-20.0] * 3, [20.0] * 3), "f32", 1e-3),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}d-{c[5]}-{c[6]:g}-{i}" for i, c in enumerate(CASES)])
@pytest.mark.parametrize("isign", [1, -1])
def test_type3_matches_oracle(case, isign):
    dim, M, N, (xlo, xhi), (slo, shi), prec, eps = case
    dt = np.float32 if prec == "f32" else np.float64
    xs = _box(M, dim, 301 + dim, xlo, xhi, dt)
    ss = _box(N, dim, 302 + dim, slo, shi, dt)
    c = I.complex_normal(M, 303, np.complex64 if prec == "f32" else np.complex128)
    f, info = run_type3(xs, c, ss, eps, prec, isign=isign)
    ref = O.type3(xs, c, ss, isign)
    err = O.rel_l2(f, ref)
    print(f"type 3 {dim}d {prec} eps {eps:g} isign {isign}: rel l2 {err:.2e}, grid "
          f"{[int(info.nf[m]) for m in range(dim)]}")
    assert err <= 10 * eps


def test_type3_clustered_sources_and_targets():
    """Wrapped-Gaussian clusters for sources and targets (3D, single)."""
    xs = I.wrapped_gaussian_points(20000, 3, 311, 0.3, np.float32)
    rng = np.random.default_rng(312)
    ss = [np.clip(rng.normal(0, 12, 3000), -48, 48).astype(np.float32) for _ in range(3)]
    c = I.complex_normal(20000, 313, np.complex64)
    f, _ = run_type3(xs, c, ss, 1e-6, "f32")
    assert O.rel_l2(f, O.type3(xs, c, ss, 1)) <= 1e-5


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_type3_integer_targets_match_type1(dim):
    """Targets on the integer mode grid: the type 3 result equals a type 1 plan's
    modes (both within eps of the same sums)."""
    Ns = (24, 18, 12)[:dim]
    xs = I.uniform_points(6000, dim, 321, np.float64)
    c = I.complex_normal(6000, 322, np.complex128)
    modes = [I.mode_range(n) for n in Ns]
    mesh = np.meshgrid(*reversed(modes), indexing="ij")
    ss = [m.reshape(-1).astype(np.float64) for m in reversed(mesh)]
    f3, _ = run_type3(xs, c, ss, 1e-10, "f64")
    f1, _ = run_type1(xs, c, Ns, 1e-10, "f64")
    assert O.rel_l2(f3, f1.reshape(-1)) <= 1e-9


def test_type3_batched_equals_single():
    xs = _box(3000, 2, 331, [-2, -2], [2, 2], np.float32)
    ss = _box(2000, 2, 332, [-50, -50], [50, 50], np.float32)
    c = I.complex_normal((3, 3000), 333, np.complex64)
    fb, _ = run_type3(xs, c, ss, 1e-5, "f32", ntransf=3)
    for t in range(3):
        f1, _ = run_type3(xs, c[t], ss, 1e-5, "f32")
        assert O.rel_l2(fb[t], f1) < 1e-6
    assert O.rel_l2(fb[1], O.type3(xs, c[1], ss, 1)) <= 1e-4


def test_type3_degenerate_sets():
    t = torch()
    rng = np.random.default_rng(341)
    # every target at one frequency (S = 0): f = sum_j c_j exp(i s0 x_j)
    xs = [rng.uniform(-2, 3, 500)]
    ss = [np.full(7, 4.25)]
    c = I.complex_normal(500, 342, np.complex128)
    f, _ = run_type3(xs, c, ss, 1e-9, "f64")
    assert O.rel_l2(f, O.type3(xs, c, ss, 1)) <= 1e-8
    # every source at one point (X = 0)
    xs = [np.full(300, -1.5), np.full(300, 0.75)]
    ss = [rng.uniform(-40, 40, 200), rng.uniform(-10, 70, 200)]
    c = I.complex_normal(300, 343, np.complex128)
    f, _ = run_type3(xs, c, ss, 1e-9, "f64")
    assert O.rel_l2(f, O.type3(xs, c, ss, 1)) <= 1e-8
    # no sources: zeros; no targets: nothing to write
    p = B.Plan3(2, 1e-6, dtype=t.complex128)
    p.setpts([t.zeros(0, dtype=t.float64, device="cuda")] * 2,
             [dev(rng.uniform(-5, 5, 9)) for _ in range(2)])
    f = host(p.execute(t.zeros(0, dtype=t.complex128, device="cuda")))
    assert f.shape == (9,) and np.all(f == 0)
    p.setpts([dev(rng.uniform(-1, 1, 5)) for _ in range(2)],
             [t.zeros(0, dtype=t.float64, device="cuda")] * 2)
    assert p.execute(dev(I.complex_normal(5, 344, np.complex128))).numel() == 0
    p.close()


def test_type3_setpts_again_and_bad_points():
    """A plan takes new point sets of other sizes and extents (its inner plans
    are remade when the fine grid changes); NaN coordinates are errors."""
    t = torch()
    p = B.Plan3(3, 1e-6, dtype=t.complex64)
    for k, (M, N, S) in enumerate([(4000, 1500, 20.0), (9000, 700, 45.0), (2000, 3000, 20.0)]):
        xs = _box(M, 3, 351 + k, [-1] * 3, [1] * 3, np.float32)
        ss = _box(N, 3, 361 + k, [-S] * 3, [S] * 3, np.float32)
        c = I.complex_normal(M, 371 + k, np.complex64)
        p.setpts([dev(a) for a in xs], [dev(a) for a in ss])
        f = host(p.execute(dev(c)))
        assert O.rel_l2(f, O.type3(xs, c, ss, 1)) <= 1e-5
    bad = [dev(np.array([0.1, np.nan, 0.3], dtype=np.float32))] * 3
    good = [dev(np.array([1.0, 2.0], dtype=np.float32))] * 3
    with pytest.raises(B.EsnError) as e:
        p.setpts(bad, good)
    assert e.value.status == B.ESN_ERR_NAN_PTS
    with pytest.raises(B.EsnError):
        p.execute(dev(I.complex_normal(3, 381, np.complex64)))
    p.close()
