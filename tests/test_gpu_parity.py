"""GPU parity of the HIP path with the FP64 oracle (relative l2 error, Sec. 4.2).

Bar: rel. l2 error <= 10 eps on every case (eps = requested tolerance).  Inputs
are seeded (paper_1808_06736_amd.inputs); the oracle gets exactly the values
the GPU gets, upcast to FP64.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1808_06736_amd import binding as B
from paper_1808_06736_amd import inputs as I
from tests.gpu_helpers import coord_np, dev, host, run_type1, run_type2, torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("prec,eps", [("f32", 1e-5), ("f64", 1e-9)])
def test_single_point_at_origin_gives_ones(dim, prec, eps):
    N = (12, 9, 7)[:dim]
    coords = coord_np([np.zeros(1)] * dim, prec)
    c = np.ones(1, dtype=np.complex64 if prec == "f32" else np.complex128)
    f, _ = run_type1(coords, c, N, eps, prec)
    assert f.shape == tuple(reversed(N))
    assert np.max(np.abs(f - 1.0)) < 10 * eps


def test_small_1d_type1_full():
    """1D type 1, M = 10^4 iid uniform points, N = 1000, eps = 1e-6, FP64: full output."""
    w = I.WORKLOADS["1d_t1_small"]
    coords = w.coords()
    c = w.strengths()
    f, info = run_type1(coords, c, (1000,), w.eps, "f64")
    assert info.w == 7
    ref = O.type1(coords, c, +1, N=(1000,))
    err = O.rel_l2(f, ref)
    print(f"1d t1 rel l2 = {err:.3e}")
    assert err <= 10 * w.eps


CASES = [
    # dim, N, M, points, prec, eps
    (1, (257,), 5001, "uniform", "f64", 1e-9),
    (1, (100,), 3000, "wrapped_gaussian", "f32", 1e-4),
    (2, (40, 33), 20011, "uniform", "f32", 1e-5),
    (2, (31, 64), 20011, "wrapped_gaussian", "f64", 1e-10),
    (3, (16, 13, 20), 30007, "uniform", "f32", 1e-6),
    (3, (24, 24, 24), 30007, "wrapped_gaussian", "f32", 1e-4),
    (3, (11, 16, 9), 20011, "wrapped_gaussian", "f64", 1e-9),
]


def _inputs(dim, N, M, points, prec, seed):
    dt = np.float32 if prec == "f32" else np.float64
    if points == "uniform":
        coords = I.uniform_points(M, dim, seed, dt)
    else:
        coords = I.wrapped_gaussian_points(M, dim, seed, 0.3, dt)
    cdt = np.complex64 if prec == "f32" else np.complex128
    c = I.complex_normal(M, seed + 1, cdt)
    f = I.complex_normal(tuple(reversed(N)), seed + 2, cdt)
    return coords, c, f


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}d-{c[4]}-{c[3]}-{c[5]:g}" for c in CASES])
def test_small_type1_full(case):
    dim, N, M, points, prec, eps = case
    coords, c, _ = _inputs(dim, N, M, points, prec, 100 + dim)
    f, _ = run_type1(coords, c, N, eps, prec)
    ref = O.type1(coords, c, +1, N=N)
    err = O.rel_l2(f, ref)
    print(f"type1 {case}: {err:.3e}")
    assert err <= 10 * eps


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}d-{c[4]}-{c[3]}-{c[5]:g}" for c in CASES])
def test_small_type2_full(case):
    dim, N, M, points, prec, eps = case
    coords, _, f = _inputs(dim, N, M, points, prec, 200 + dim)
    c, _ = run_type2(coords, f, N, eps, prec)
    ref = O.type2(coords, f, -1)
    err = O.rel_l2(c, ref)
    print(f"type2 {case}: {err:.3e}")
    assert err <= 10 * eps


METHOD_CASES = [
    # dim, N, M, points, prec, eps
    (3, (16, 13, 20), 30007, "uniform", "f32", 1e-6),
    (3, (24, 20, 28), 300007, "wrapped_gaussian", "f32", 1e-6),
    (3, (12, 12, 12), 200003, "wrapped_gaussian", "f32", 1e-3),
    (2, (40, 33), 50011, "wrapped_gaussian", "f64", 1e-9),
    (2, (64, 50), 80021, "uniform", "f32", 1e-5),
    (2, (37, 48), 60013, "wrapped_gaussian", "f64", 1e-12),
]


def _methods(dim, prec, eps):
    """Methods a case runs: LDS tiles, atomics / gathers, and the matrix cores
    where they apply (3D single precision at w <= 7; 2D at w <= 13)."""
    if dim == 3 and prec == "f32" and eps >= 1e-6:
        return [1, 2, 3]
    if dim == 2 and eps >= 1e-12:
        return [1, 2, 3]
    return [1, 2]


@pytest.mark.parametrize("case", METHOD_CASES,
                         ids=[f"{c[0]}d-{c[4]}-{c[3]}-{c[5]:g}" for c in METHOD_CASES])
def test_spread_methods_agree(case):
    """Every spreading method (LDS tiles, global atomics, dense columns on the
    matrix cores) meets the bar, and they agree with each other to rounding."""
    dim, N, M, points, prec, eps = case
    coords, c, _ = _inputs(dim, N, M, points, prec, 300 + dim)
    ref = O.type1(coords, c, +1, N=N)
    outs = {}
    methods = _methods(dim, prec, eps)
    for m in methods:
        f, info = run_type1(coords, c, N, eps, prec, spread_method=m)
        err = O.rel_l2(f, ref)
        print(f"method {m}: rel l2 {err:.3e}, dense units {info.ndense_units}")
        assert err <= 10 * eps
        if m == 3 and points == "wrapped_gaussian":
            assert info.ndense_units > 0
        outs[m] = f
    for m in methods[1:]:
        assert O.rel_l2(outs[m], outs[methods[0]]) < (1e-5 if prec == "f32" else 1e-12)


@pytest.mark.parametrize("case", METHOD_CASES,
                         ids=[f"{c[0]}d-{c[4]}-{c[3]}-{c[5]:g}" for c in METHOD_CASES])
def test_interp_methods_agree(case):
    """Every interpolation method (LDS tiles, direct gathers, dense columns on
    the matrix cores) meets the bar, and they agree with each other to rounding."""
    dim, N, M, points, prec, eps = case
    coords, _, f = _inputs(dim, N, M, points, prec, 400 + dim)
    ref = O.type2(coords, f, -1)
    outs = {}
    methods = _methods(dim, prec, eps)
    for m in methods:
        cc, info = run_type2(coords, f, N, eps, prec, interp_method=m)
        err = O.rel_l2(cc, ref)
        print(f"interp method {m}: rel l2 {err:.3e}, dense units {info.ndense_units}")
        assert err <= 10 * eps
        if m == 3 and points == "wrapped_gaussian":
            assert info.ndense_units > 0
        outs[m] = cc
    for m in methods[1:]:
        assert O.rel_l2(outs[m], outs[methods[0]]) < (1e-5 if prec == "f32" else 1e-12)


def _many_small_cases(count, seed):
    rng = np.random.default_rng(seed)
    cases = []
    for i in range(count):
        N = tuple(int(x) for x in rng.integers(12, 48, 3))
        M = int(10 ** rng.uniform(3.5, 5.2))
        points = "uniform" if i % 2 == 0 else "wrapped_gaussian"
        eps = [1e-6, 1e-5, 1e-4, 1e-3][i % 4]
        cases.append((N, M, points, eps, 1000 + i))
    return cases


@pytest.mark.parametrize("type_", [1, 2])
def test_matrix_core_matches_lds_tiles_on_many_small_problems(type_):
    """The matrix-core kernels (3D, single precision) agree with the LDS-tile
    kernels to rounding on 60 small problems of random shape, size, point
    distribution and tolerance.  Small problems leave few waves per SIMD, where
    the matrix results' latency is least hidden by other waves' work; a value
    read too early shows up as a few wrong points."""
    for N, M, points, eps, seed in _many_small_cases(60, 17 + type_):
        coords, c, f = _inputs(3, N, M, points, "f32", seed)
        outs = {}
        for m in (1, 3):
            if type_ == 1:
                outs[m], _ = run_type1(coords, c, N, eps, "f32", spread_method=m)
            else:
                outs[m], _ = run_type2(coords, f, N, eps, "f32", interp_method=m)
        err = O.rel_l2(outs[3], outs[1])
        assert err < 1e-5, (N, M, points, eps, err)


def _many_small_cases_2d(count, seed):
    rng = np.random.default_rng(seed)
    cases = []
    for i in range(count):
        N = tuple(int(x) for x in rng.integers(12, 120, 2))
        M = int(10 ** rng.uniform(3.0, 5.0))
        points = "uniform" if i % 2 == 0 else "wrapped_gaussian"
        prec, eps = [("f32", 1e-6), ("f32", 1e-4), ("f64", 1e-9), ("f64", 1e-12)][i % 4]
        cases.append((N, M, points, prec, eps, 2000 + i))
    return cases


@pytest.mark.parametrize("type_", [1, 2])
def test_matrix_core_2d_matches_lds_tiles_on_many_small_problems(type_):
    """The 2D matrix-core kernels (single and double precision, w up to 13)
    agree with the LDS-tile kernels to rounding on 40 small problems of random
    shape, size, point distribution and tolerance."""
    for N, M, points, prec, eps, seed in _many_small_cases_2d(40, 27 + type_):
        coords, c, f = _inputs(2, N, M, points, prec, seed)
        outs = {}
        for m in (1, 3):
            if type_ == 1:
                outs[m], info = run_type1(coords, c, N, eps, prec, spread_method=m)
            else:
                outs[m], info = run_type2(coords, f, N, eps, prec, interp_method=m)
        err = O.rel_l2(outs[3], outs[1])
        assert err < (1e-5 if prec == "f32" else 1e-12), (N, M, points, prec, eps, err)


@pytest.mark.parametrize("prec,eps", [("f32", 1e-5), ("f64", 1e-9)])
@pytest.mark.parametrize("type_", [1, 2])
def test_matrix_core_2d_batched_equals_single(prec, eps, type_):
    """Five vectors on one point set through the 2D matrix-core kernels, fused
    in launches of two (the weights staged once for both) and run one at a
    time: the results agree and meet the oracle bar."""
    N = (56, 44)
    M = 40_000
    coords, _, _ = _inputs(2, N, M, "wrapped_gaussian", prec, 77)
    cdt = np.complex64 if prec == "f32" else np.complex128
    c = I.complex_normal((5, M), 78, cdt)
    f = I.complex_normal((5,) + tuple(reversed(N)), 79, cdt)
    if type_ == 1:
        fused, info = run_type1(coords, c, N, eps, prec, ntransf=5, spread_method=3,
                                ntransf_chunk=2)
    else:
        fused, info = run_type2(coords, f, N, eps, prec, ntransf=5, interp_method=3,
                                ntransf_chunk=2)
    assert info.ntransf_chunk == 2
    for t in range(5):
        if type_ == 1:
            one, _ = run_type1(coords, c[t], N, eps, prec, spread_method=3)
            ref = O.type1(coords, c[t], +1, N=N)
        else:
            one, _ = run_type2(coords, f[t], N, eps, prec, interp_method=3)
            ref = O.type2(coords, f[t], -1)
        assert O.rel_l2(fused[t], one) < (1e-5 if prec == "f32" else 1e-12)
        assert O.rel_l2(fused[t], ref) <= 10 * eps


SEAM_CASES = [
    # dim, N, prec, eps, method (0 = automatic)
    (3, (16, 20, 24), "f32", 1e-6, 3),
    (3, (16, 20, 24), "f32", 1e-6, 1),
    (3, (13, 9, 11), "f64", 1e-9, 0),
    (2, (30, 17), "f32", 1e-5, 0),
    (1, (45,), "f64", 1e-12, 0),
]


@pytest.mark.parametrize("case", SEAM_CASES, ids=[f"{c[0]}d-{c[2]}-m{c[4]}" for c in SEAM_CASES])
@pytest.mark.parametrize("type_", [1, 2])
def test_points_at_the_fine_grid_seam(case, type_):
    """Points in the last and first fine-grid cells of every dimension (x just
    below and just above 0, i.e. t near n and near 0 after the fold): those in
    the upper half of cell n - 1 have their window start wrap past n and are
    binned with the first cells.  Every method meets the bar there."""
    dim, N, prec, eps, method = case
    st, par = B.esn_choose_params(eps, B.ESN_SINGLE if prec == "f32" else B.ESN_DOUBLE, dim,
                                  tuple(N) + (1,) * (3 - dim))
    assert st == 0
    rng = np.random.default_rng(77 + dim)
    M = 6000
    dt = np.float32 if prec == "f32" else np.float64
    coords = []
    for m in range(dim):
        h = 2 * np.pi / par.nf[m]
        x = rng.uniform(-h, h, M)
        x[: M // 4] = rng.uniform(-np.pi, np.pi, M // 4)   # some spread-out points too
        coords.append(x.astype(dt))
    coords = [np.ascontiguousarray(a) for a in coords]
    cdt = np.complex64 if prec == "f32" else np.complex128
    opts = {}
    if type_ == 1:
        if method:
            opts["spread_method"] = method
        c = I.complex_normal(M, 78, cdt)
        f, _ = run_type1(coords, c, N, eps, prec, **opts)
        err = O.rel_l2(f, O.type1(coord_np(coords, prec), c, +1, N=N))
    else:
        if method:
            opts["interp_method"] = method
        f = I.complex_normal(int(np.prod(N)), 79, cdt).reshape(tuple(reversed(N)))
        c, _ = run_type2(coords, f, N, eps, prec, **opts)
        err = O.rel_l2(c, O.type2(coord_np(coords, prec), f, -1))
    print(f"seam {dim}d {prec} method {method} type {type_}: rel l2 {err:.2e}")
    assert err <= 10 * eps


KEREVAL_CASES = [
    # dim, N, M, points, prec, eps
    (1, (500,), 20000, "uniform", "f64", 1e-12),
    (2, (64, 48), 50000, "wrapped_gaussian", "f64", 1e-9),
    (3, (24, 20, 16), 60000, "uniform", "f64", 1e-9),
    (3, (32, 28, 24), 200000, "wrapped_gaussian", "f32", 1e-6),
    (2, (100, 80), 100000, "uniform", "f32", 1e-5),
    (3, (20, 20, 20), 50000, "uniform", "f32", 1e-3),
]


@pytest.mark.parametrize("case", KEREVAL_CASES,
                         ids=[f"{c[0]}d-{c[4]}-{c[3]}-{c[5]:g}" for c in KEREVAL_CASES])
@pytest.mark.parametrize("type_", [1, 2])
def test_kernel_table_and_direct_evaluation(case, type_):
    """Both kernel evaluations (exp and sqrt at every weight, and the piecewise
    polynomial table of Sec. 5.3) meet the bar with every spreading or
    interpolation method, and agree with each other to eps (double precision)
    or to the single precision rounding floor."""
    dim, N, M, points, prec, eps = case
    coords, c, f = _inputs(dim, N, M, points, prec, 600 + dim)
    cn = coord_np(coords, prec)
    ref = O.type1(cn, c, +1, N=N) if type_ == 1 else O.type2(cn, f, -1)
    mkey = "spread_method" if type_ == 1 else "interp_method"
    methods = [0, 1, 2]
    if dim == 3 and prec == "f32" and eps >= 1e-6:
        methods.append(3)
    for m in methods:
        outs = {}
        for kev in (1, 2):
            opts = {"kerevalmeth": kev}
            if m:
                opts[mkey] = m
            if type_ == 1:
                out, info = run_type1(coords, c, N, eps, prec, **opts)
            else:
                out, info = run_type2(coords, f, N, eps, prec, **opts)
            assert info.kerevalmeth == kev
            err = O.rel_l2(out, ref)
            print(f"{dim}d {prec} type {type_} method {m} kerevalmeth {kev}: rel l2 {err:.2e}")
            assert err <= 10 * eps
            outs[kev] = out
        # (single precision: both sit on the FP32 rounding floor, about 1e-6)
        assert O.rel_l2(outs[2], outs[1]) <= (eps if prec == "f64" else max(eps, 1e-5))


LOW_SIGMA_CASES = [
    # dim, N, M, points, prec, eps
    (1, (600,), 20000, "uniform", "f64", 1e-8),
    (2, (80, 64), 60000, "wrapped_gaussian", "f64", 1e-6),
    (2, (100, 90), 80000, "uniform", "f32", 1e-4),
    (3, (24, 20, 28), 100000, "uniform", "f64", 1e-5),
    (3, (32, 28, 24), 200000, "wrapped_gaussian", "f32", 1e-3),
]


@pytest.mark.parametrize("case", LOW_SIGMA_CASES,
                         ids=[f"{c[0]}d-{c[4]}-{c[3]}-{c[5]:g}" for c in LOW_SIGMA_CASES])
@pytest.mark.parametrize("type_", [1, 2])
def test_low_upsampling_meets_bar(case, type_):
    """sigma = 5/4 (fine grid n >= 1.25 N, the wider kernel of the low
    upsampling rule): every method meets the bar against the oracle."""
    dim, N, M, points, prec, eps = case
    coords, c, f = _inputs(dim, N, M, points, prec, 700 + dim)
    cn = coord_np(coords, prec)
    ref = O.type1(cn, c, +1, N=N) if type_ == 1 else O.type2(cn, f, -1)
    mkey = "spread_method" if type_ == 1 else "interp_method"
    methods = [0, 1, 2]
    for m in methods:
        opts = {"upsampfac": 1.25}
        if m:
            opts[mkey] = m
        if type_ == 1:
            out, info = run_type1(coords, c, N, eps, prec, **opts)
        else:
            out, info = run_type2(coords, f, N, eps, prec, **opts)
        err = O.rel_l2(out, ref)
        print(f"sigma 1.25 {dim}d {prec} type {type_} method {m}: w {info.w}, "
              f"nf {list(info.nf)[:dim]}, rel l2 {err:.2e}")
        assert all(info.nf[d] < 2 * N[d] for d in range(dim))
        assert err <= 10 * eps


COLUMN_FFT_CASES = [
    # N, sigma, ntransf, fine grid: y and z lengths 2^a 3^b 5^c (a >= 5) up to
    # 512, x a multiple of 32
    ((31, 127, 16), 2.0, 1, (64, 256, 32)),   # odd N1: kept x runs of 16 and 15 columns
    ((16, 16, 256), 2.0, 1, (32, 32, 512)),   # radix-2 last stage in y (32) and z (512)
    ((101, 25, 25), 1.25, 1, (128, 32, 32)),  # kept runs reach every block of 32 columns
    ((31, 127, 16), 2.0, 3, (64, 256, 32)),   # three transforms per launch
    ((47, 143, 79), 2.0, 1, (96, 288, 160)),  # radix 3 and 5 stages, odd N
    ((192, 240, 48), 2.0, 1, (384, 480, 96)),  # radix 3 then 5 in one transform
]


@pytest.mark.parametrize("case", COLUMN_FFT_CASES,
                         ids=[f"{c[0]}-s{c[1]:g}-t{c[2]}" for c in COLUMN_FFT_CASES])
def test_column_fft_grids(case):
    """3D single-precision plans on power-of-two fine grids run the y and z
    passes of the FFT as column FFTs over the kept x columns: type 1 and type 2
    meet the bar against the oracle, for each transform of a batch."""
    N, sigma, ntr, nf = case
    eps, M = 1e-5, 3000
    coords = coord_np(I.uniform_points(M, 3, 901, np.float32), "f32")
    c = I.complex_normal((ntr, M) if ntr > 1 else M, 902, np.complex64)
    f = I.complex_normal(((ntr,) if ntr > 1 else ()) + tuple(reversed(N)), 903, np.complex64)
    opts = {"upsampfac": sigma} if sigma != 2.0 else {}
    out1, info = run_type1(coords, c, N, eps, "f32", ntransf=ntr, **opts)
    assert tuple(int(info.nf[m]) for m in range(3)) == nf
    out2, _ = run_type2(coords, f, N, eps, "f32", ntransf=ntr, **opts)
    cs = c.reshape(ntr, M)
    fs = f.reshape((ntr,) + tuple(reversed(N)))
    o1 = out1.reshape((ntr,) + tuple(reversed(N)))
    o2 = out2.reshape(ntr, M)
    for t in range(ntr):
        e1 = O.rel_l2(o1[t], O.type1(coords, cs[t], +1, N=N))
        e2 = O.rel_l2(o2[t], O.type2(coords, fs[t], -1))
        print(f"column FFTs {N} sigma {sigma} transform {t}: type 1 {e1:.2e}, type 2 {e2:.2e}")
        assert e1 <= 10 * eps and e2 <= 10 * eps


@pytest.mark.parametrize("N,sigma,nf", [((31, 127, 16), 2.0, (64, 256, 32)),
                                         ((101, 25, 25), 1.25, (128, 32, 32))],
                         ids=["s2-odd", "s1.25-w10"])
def test_column_fft_several_transforms_per_launch(N, sigma, nf):
    """Three transforms on one plan whose launches take several at once (the
    LDS-tile kernels fuse the batch as far as the LDS allows, so the column
    passes run with a transform index per block and the correction and the
    clear of the unkept columns with ntr > 1, then a tail launch), for type 1,
    type 2 and the type 1 plan's adjoint: every transform meets the oracle bar."""
    eps, M = 1e-5, 3000
    coords = coord_np(I.uniform_points(M, 3, 931, np.float32), "f32")
    c = I.complex_normal((3, M), 932, np.complex64)
    f = I.complex_normal((3,) + tuple(reversed(N)), 933, np.complex64)
    opts = {"spread_method": 1, "interp_method": 1}
    if sigma != 2.0:
        # w = 10: bins of 4 x 4 x 4 keep two tiles within the LDS budget
        opts.update(upsampfac=sigma, bin=(4, 4, 4))
    t = torch()
    p1 = B.Plan(1, N, eps, dtype=t.complex64, ntransf=3, **opts)
    p1.setpts(*[dev(a) for a in coords])
    info = p1.info()
    assert tuple(int(info.nf[m]) for m in range(3)) == nf and info.ntransf_chunk >= 2
    o1 = host(p1.type1(dev(c)))
    adj = t.empty((3, M), dtype=t.complex64, device="cuda")
    p1.execute_adjoint(adj, dev(f))
    adj = host(adj)
    p1.close()
    o2, info2 = run_type2(coords, f, N, eps, "f32", ntransf=3, **opts)
    assert info2.ntransf_chunk >= 2
    for k in range(3):
        e1 = O.rel_l2(o1[k], O.type1(coords, c[k], +1, N=N))
        r2 = O.type2(coords, f[k], -1)
        e2 = O.rel_l2(o2[k], r2)
        ea = O.rel_l2(adj[k], r2)
        print(f"column FFTs, 3 transforms, {N} sigma {sigma} transform {k}: type 1 {e1:.2e}, "
              f"type 2 {e2:.2e}, adjoint {ea:.2e}")
        assert e1 <= 10 * eps and e2 <= 10 * eps and ea <= 10 * eps


def test_column_fft_modes_in_fft_order():
    """The column passes that read or write the mode arrays themselves keep
    the caller's mode order: modeord 1 (FFT order) gives the modeord 0 result
    permuted, for type 1 and type 2 (odd and even N on a 64 x 256 x 32 grid)."""
    N = (31, 127, 16)
    coords = coord_np(I.uniform_points(4000, 3, 911, np.float32), "f32")
    c = I.complex_normal(4000, 912, np.complex64)
    f0, info = run_type1(coords, c, N, 1e-5, "f32")
    assert tuple(int(info.nf[m]) for m in range(3)) == (64, 256, 32)
    f1, _ = run_type1(coords, c, N, 1e-5, "f32", modeord=1)
    perm = [np.concatenate([np.arange(n // 2, n), np.arange(0, n // 2)]) for n in reversed(N)]
    assert np.max(np.abs(f1 - f0[np.ix_(*perm)])) <= 1e-5 * np.max(np.abs(f0))
    ff = I.complex_normal(tuple(reversed(N)), 913, np.complex64)
    c0, _ = run_type2(coords, ff, N, 1e-5, "f32")
    c1, _ = run_type2(coords, ff[np.ix_(*perm)], N, 1e-5, "f32", modeord=1)
    assert np.max(np.abs(c1 - c0)) <= 1e-5 * np.max(np.abs(c0))
    assert O.rel_l2(c0, O.type2(coords, ff, -1)) <= 1e-4


@pytest.mark.parametrize("N,ntr,nf", [((64, 80), 1, (128, 160)), ((47, 143), 3, (96, 288))],
                         ids=["64x80", "47x143-t3"])
def test_column_fft_grids_2d(N, ntr, nf):
    """2D single-precision plans on column-FFT lengths run the y pass on the
    kept x columns only: type 1 and type 2 meet the bar for every transform."""
    eps, M = 1e-5, 20000
    coords = coord_np(I.wrapped_gaussian_points(M, 2, 921, 0.5, np.float32), "f32")
    c = I.complex_normal((ntr, M) if ntr > 1 else M, 922, np.complex64)
    f = I.complex_normal(((ntr,) if ntr > 1 else ()) + tuple(reversed(N)), 923, np.complex64)
    out1, info = run_type1(coords, c, N, eps, "f32", ntransf=ntr)
    assert tuple(int(info.nf[m]) for m in range(2)) == nf
    out2, _ = run_type2(coords, f, N, eps, "f32", ntransf=ntr)
    cs = c.reshape(ntr, M)
    fs = f.reshape((ntr,) + tuple(reversed(N)))
    o1 = out1.reshape((ntr,) + tuple(reversed(N)))
    o2 = out2.reshape(ntr, M)
    for t in range(ntr):
        e1 = O.rel_l2(o1[t], O.type1(coords, cs[t], +1, N=N))
        e2 = O.rel_l2(o2[t], O.type2(coords, fs[t], -1))
        print(f"2D column FFTs {N} transform {t}: type 1 {e1:.2e}, type 2 {e2:.2e}")
        assert e1 <= 10 * eps and e2 <= 10 * eps


@pytest.mark.parametrize("type_", [1, 2])
def test_matrix_core_3d_batched_transforms(type_):
    """Five vectors on one clustered 3D point set through the 3D matrix-core
    kernels as one batched execute (one launch per vector on the once-sorted
    points, the FFTs batched): each equals the same vector run by itself, and
    two of them meet the oracle bar.  The same plan's adjoint runs the other
    direction batched."""
    N = (40, 36, 32)
    M = 120_000
    eps = 1e-6
    coords, _, _ = _inputs(3, N, M, "wrapped_gaussian", "f32", 91)
    c = I.complex_normal((5, M), 92, np.complex64)
    f = I.complex_normal((5,) + tuple(reversed(N)), 93, np.complex64)
    t = torch()
    p = B.Plan(type_, N, eps, dtype=t.complex64, ntransf=5)
    p.setpts(*[dev(a) for a in coords])
    info = p.info()
    assert (info.spread_method if type_ == 1 else info.interp_method) == 3
    batch = host(p.type1(dev(c))) if type_ == 1 else host(p.type2(dev(f)))
    # the adjoint (other direction, opposite sign) of the same plan, batched too
    if type_ == 1:
        adj = t.empty((5, M), dtype=t.complex64, device="cuda")
        p.execute_adjoint(adj, dev(f))
    else:
        adj = t.empty((5,) + tuple(reversed(N)), dtype=t.complex64, device="cuda")
        p.execute_adjoint(dev(c), adj)
    adj = host(adj)
    p.close()
    for k in range(5):
        if type_ == 1:
            one, _ = run_type1(coords, c[k], N, eps, "f32")
            one_adj, _ = run_type2(coords, f[k], N, eps, "f32", isign=-1)
        else:
            one, _ = run_type2(coords, f[k], N, eps, "f32")
            one_adj, _ = run_type1(coords, c[k], N, eps, "f32", isign=+1)
        assert O.rel_l2(batch[k], one) < 1e-5, k
        assert O.rel_l2(adj[k], one_adj) < 1e-5, k
    for k in (0, 3):
        if type_ == 1:
            ref = O.type1(coords, c[k], +1, N=N)
        else:
            ref = O.type2(coords, f[k], -1)
        err = O.rel_l2(batch[k], ref)
        print(f"batched type {type_} vector {k}: rel l2 {err:.3e}")
        assert err <= 10 * eps
