"""Invariants of the bin sort (Sec. 5.1) and of the subproblems (Sec. 5.2),
read back through esn_debug_sort:

* perm is a permutation of the input indices;
* the keys are non-decreasing along the sorted order (the radix sort is also
  stable: equal keys keep the input order);
* bin_start agrees with the keys, the bin counts add up to M;
* the subproblems cover each bin exactly, in order, none longer than maxsub;
* every point's key is the key of its window cell, recomputed here on the
  host from the coordinates (FP64 fold and rescale, fixed point in single
  precision), except at most a few points within rounding of a cell edge;
* the radix sort and the counting sort produce the same key sequence.

Sizes cover both methods (the radix sort for M >= 2^21 by default, forced
below that), one, two and three radix passes, 16- and 32-byte records,
blocked and unblocked 3D cell orders, ragged tiles and single points."""
import numpy as np
import pytest

from paper_1808_06736_amd import binding as B
from paper_1808_06736_amd import inputs as I
from tests.gpu_helpers import dev, torch

pytestmark = pytest.mark.gpu

TWO_PI = 2.0 * np.pi


def _fold_rescale(x, n):
    t = x * (n / TWO_PI)
    t = t - n * np.floor(t / n)
    t = np.where(t < 0, t + n, t)
    t = np.where(t >= n, t - n, t)
    return t


def _host_keys(coords, info, fixed):
    """Window-cell keys of the points, following the plan's binning."""
    dim = len(coords)
    w = info.w
    nf = [int(info.nf[m]) for m in range(3)]
    b = [int(info.bin[m]) for m in range(3)]
    nb = [(nf[m] + b[m] - 1) // b[m] for m in range(3)]
    cells, near = [], np.zeros(coords[0].shape, dtype=bool)
    for m in range(3):
        if m >= dim:
            cells.append(np.zeros(coords[0].shape, dtype=np.int64))
            continue
        t = _fold_rescale(coords[m].astype(np.float64), nf[m])
        if fixed:
            fb = 32 - int(np.ceil(np.log2(nf[m])))
            q = np.rint(np.ldexp(t, fb))
            q = np.where(q >= np.ldexp(float(nf[m]), fb), q - np.ldexp(float(nf[m]), fb), q)
            q = q.astype(np.uint64)
            c = (q >> fb).astype(np.int64)
            fr = q & ((1 << fb) - 1)
            sh = (fr > (1 << (fb - 1))) if (w & 1) else (fr != 0)
        else:
            c = np.floor(t).astype(np.int64)
            f = t - c
            sh = (f > 0.5) if (w & 1) else (f > 0.0)
        k = c + sh.astype(np.int64)
        cells.append(np.where(k >= nf[m], k - nf[m], k))
        # points within rounding of an edge of their cell or of the shift threshold
        frac = t - np.floor(t)
        near |= (np.minimum(frac, 1 - frac) < 1e-6) | (np.abs(frac - 0.5) < 1e-6)
    bx, by, bz = (cells[m] // b[m] for m in range(3))
    lx, ly, lz = (cells[m] - (cells[m] // b[m]) * b[m] for m in range(3))
    cpb = b[0] * b[1] * b[2]
    binid = bx + nb[0] * (by + nb[1] * bz)
    if dim == 3:
        if b[0] % 2 == 0 and b[1] % 2 == 0:
            local = (lx & 1) + 2 * (ly & 1) + 4 * (lz + b[2] * ((lx >> 1) + (b[0] >> 1) * (ly >> 1)))
        else:
            local = lz + b[2] * (lx + b[0] * ly)
    elif dim == 2 and b[0] % (B := (8 if w <= 9 else 4)) == 0 and b[1] % B == 0:
        local = (lx % B) + B * (ly % B) + B * B * ((lx // B) + (b[0] // B) * (ly // B))
    else:
        local = lx + b[0] * ly
    return (binid * cpb + local).astype(np.int64), near


def _check_sort(plan, coords, fixed, stable):
    d = plan.debug_sort()
    info = plan.info()
    M = d["M"]
    perm, key, bs, sub = d["perm"], d["key"].astype(np.int64), d["bin_start"], d["sub"]
    nbins, cpb = d["nbins"], d["cells_per_bin"]
    assert d["method"] in (2, 3)
    # perm is a permutation
    assert np.array_equal(np.sort(perm), np.arange(M, dtype=np.int32))
    # keys non-decreasing; stable order within equal keys (radix)
    assert np.all(np.diff(key) >= 0)
    if stable and M > 1:
        same = np.diff(key) == 0
        assert np.all(np.diff(perm.astype(np.int64))[same] > 0)
    # keys are the points' window-cell keys
    hk, near = _host_keys(coords, info, fixed)
    bad = hk[perm] != key
    assert np.all(near[perm][bad]), f"{bad.sum()} keys differ away from cell edges"
    assert bad.sum() <= max(2, M // 10000)
    # bin starts agree with the keys; counts add up to M
    assert bs.shape == (nbins + 1,) and bs[0] == 0 and bs[-1] == M
    counts = np.diff(bs.astype(np.int64))
    assert np.all(counts >= 0) and counts.sum() == M
    assert np.array_equal(np.bincount(key // cpb, minlength=nbins)[:nbins], counts)
    # subproblems: cover each bin exactly, in order, length <= maxsub
    maxsub = info.maxsubprob
    assert sub.shape[0] == d["nsub"] == info.nsubprob
    assert np.all(sub[:, 2] >= 1) and np.all(sub[:, 2] <= maxsub)
    expect = np.sum((counts + maxsub - 1) // maxsub)
    assert d["nsub"] == expect
    pos = 0
    for i in range(sub.shape[0]):
        bb, st, ln = (int(v) for v in sub[i])
        if st == bs[bb]:
            pos = st
        assert st == pos and bs[bb] <= st and st + ln <= bs[bb + 1]
        pos = st + ln
        if i + 1 == sub.shape[0] or sub[i + 1, 0] != bb:
            assert pos == bs[bb + 1]
    # every nonempty bin has subproblems
    assert set(np.nonzero(counts)[0].tolist()) == set(np.unique(sub[:, 0]).tolist())
    assert info.nbins_nonempty == int(np.count_nonzero(counts))
    return key, perm


CASES = [
    # (name, dim, N, M, kind, prec, sort, opts)
    ("3d_clustered_radix", 3, (128, 128, 128), 2_500_000, "clustered", "f32", 1, {}),
    ("3d_uniform_f64_radix", 3, (60, 48, 40), 2_200_000, "uniform", "f64", 1, {}),
    ("3d_ragged_forced_radix", 3, (40, 45, 36), 123_457, "uniform", "f32", 2, {}),
    ("3d_unblocked_radix", 3, (40, 45, 36), 60_001, "clustered", "f32", 2, {"bin": (5, 3, 4)}),
    ("3d_counting", 3, (40, 45, 36), 60_001, "clustered", "f32", 3, {}),
    ("2d_radix", 2, (1000, 1000), 2_100_000, "uniform", "f32", 1, {}),
    ("2d_f64_forced_radix", 2, (300, 170), 77_777, "clustered", "f64", 2, {}),
    ("2d_unblocked_radix", 2, (300, 170), 50_000, "uniform", "f32", 2, {"bin": (10, 6)}),
    ("1d_radix_one_pass", 1, (1000,), 50_000, "uniform", "f64", 2, {}),
    ("1d_single_point", 1, (100,), 1, "uniform", "f32", 2, {}),
    # 320 x 320 x 288 cells: 25-bit keys, three passes of 9-bit digits
    ("3d_three_passes", 3, (160, 160, 144), 300_000, "uniform", "f32", 2, {"bin": (2, 2, 2)}),
]


@pytest.mark.parametrize("name,dim,N,M,kind,prec,sort,opts", CASES, ids=[c[0] for c in CASES])
def test_sort_invariants(name, dim, N, M, kind, prec, sort, opts):
    print(f"sort case {name}: dim {dim} N {N} M {M} {kind} {prec} sort {sort}", flush=True)
    t = torch()
    dt = np.float32 if prec == "f32" else np.float64
    if kind == "uniform":
        coords = I.uniform_points(M, dim, seed=41 + dim, dtype=dt)
    else:
        coords = I.wrapped_gaussian_points(M, dim, seed=43 + dim, dtype=dt)
    cdt = t.complex64 if prec == "f32" else t.complex128
    eps = 1e-6 if prec == "f32" else 1e-9
    plan = B.Plan(1, N, eps, dtype=cdt, sort=sort, **opts)
    plan.setpts(*[dev(a) for a in coords])
    t.cuda.synchronize()
    d = plan.debug_sort()
    if sort == 1:
        assert d["method"] == (2 if M >= (1 << 21) else 3)
    else:
        assert d["method"] == sort
    _check_sort(plan, coords, fixed=(prec == "f32"), stable=(d["method"] == 2))
    plan.close()


@pytest.mark.parametrize("dim,N,M,prec", [(3, (40, 45, 36), 200_000, "f32"),
                                          (2, (300, 170), 150_001, "f64")])
def test_radix_and_counting_sorts_agree(dim, N, M, prec):
    """The two sort methods order the same points into the same key sequence
    (the counting sort leaves the order within a cell free)."""
    t = torch()
    dt = np.float32 if prec == "f32" else np.float64
    coords = I.wrapped_gaussian_points(M, dim, seed=47, dtype=dt)
    cdt = t.complex64 if prec == "f32" else t.complex128
    keys = {}
    for sort in (2, 3):
        plan = B.Plan(1, N, 1e-6 if prec == "f32" else 1e-9, dtype=cdt, sort=sort)
        plan.setpts(*[dev(a) for a in coords])
        keys[sort] = _check_sort(plan, coords, fixed=(prec == "f32"), stable=(sort == 2))
        plan.close()
    k2, p2 = keys[2]
    k3, p3 = keys[3]
    assert np.array_equal(k2, k3)
    # same points per key: the stable order is the counting order sorted per key
    order3 = np.lexsort((p3, k3))
    assert np.array_equal(p3[order3], p2)


def test_radix_sort_repeated_setpts_reuses_scratch():
    """setpts twice on one plan (larger then smaller point set): the second sort
    starts from fresh counters and status words."""
    t = torch()
    plan = B.Plan(1, (64, 64, 64), 1e-6, sort=2)
    for M, seed in ((300_000, 3), (70_001, 4)):
        coords = I.uniform_points(M, 3, seed=seed, dtype=np.float32)
        plan.setpts(*[dev(a) for a in coords])
        t.cuda.synchronize()
        _check_sort(plan, coords, fixed=True, stable=True)
    plan.close()
