"""esn_setpts_noalloc (the bin sort's scratch in a static device array, no
allocation) against esn_setpts, through the C ABI: two calls in a row on one
plan, the second with fewer points.  After each, the sorted records, keys,
bin starts and subproblems equal those of esn_setpts on another plan
(integer work: bit for bit), and a type 1 transform from the sorted points
meets the oracle bar and agrees with the other plan's.  The calls leave the
device's free memory and the plan's device bytes unchanged; sizes beyond the
plan's room are refused."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1808_06736_amd import binding as B
from paper_1808_06736_amd import inputs as I
from tests.gpu_helpers import dev, host, torch

pytestmark = pytest.mark.gpu


def _oracle_err(coords, c, f, N, seed):
    modes = [I.sample_modes(n, 10, seed=seed + m) for m, n in enumerate(N)]
    ref = O.type1(coords, c, +1, modes=modes)
    idx = np.ix_(*[m + n // 2 for m, n in zip(reversed(modes), reversed(N))])
    return O.rel_l2(f[idx], ref)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_setpts_noalloc_matches_setpts_on_two_calls(prec):
    t = torch()
    N = (64, 48, 40)
    eps = 1e-6 if prec == "f32" else 1e-9
    cdt = t.complex64 if prec == "f32" else t.complex128
    rdt = np.float32 if prec == "f32" else np.float64
    cnp = np.complex64 if prec == "f32" else np.complex128
    sets = [I.wrapped_gaussian_points(400_000, 3, 81, 0.3, rdt),
            I.uniform_points(123_457, 3, 82, rdt)]
    ref = B.Plan(1, N, eps, dtype=cdt, sort=2)
    na = B.Plan(1, N, eps, dtype=cdt, sort=2)
    na.setpts(*[dev(a) for a in sets[0]])       # room for the larger set (allocates)
    t.cuda.synchronize()
    room = na.info().device_bytes
    for k, coords in enumerate(sets):
        M = coords[0].size
        print(f"no-alloc call {k}: {prec}, M {M}", flush=True)
        xs = [dev(a) for a in coords]
        c = dev(I.complex_normal(M, 90 + k, cnp))
        t.cuda.synchronize()
        free0 = t.cuda.mem_get_info()[0]
        st = B.lib().esn_setpts_noalloc(na.handle, M, B.ESN_SINGLE if prec == "f32" else B.ESN_DOUBLE,
                                        *[B.vp(a.data_ptr()) for a in xs])
        assert st == 0, B.strerror(st)
        na.M = M
        t.cuda.synchronize()
        if k > 0:          # the first call looked up the static array's address
            assert t.cuda.mem_get_info()[0] == free0
        assert na.info().device_bytes == room
        ref.setpts(*xs)
        dn, dr = na.debug_sort(), ref.debug_sort()
        assert dn["method"] == dr["method"] == 2 and dn["M"] == M
        for name in ("perm", "key", "bin_start", "sub"):
            assert np.array_equal(dn[name], dr[name]), name
        f_na = host(na.type1(c))
        f_ref = host(ref.type1(c))
        assert O.rel_l2(f_na, f_ref) < (1e-5 if prec == "f32" else 1e-12)
        err = _oracle_err(coords, host(c), f_na, N, seed=95 + 3 * k)
        print(f"  oracle rel l2 {err:.2e} (eps {eps:g})", flush=True)
        assert err <= 10 * eps
    # more points than the plan holds room for: refused, nothing allocated
    big = [dev(a) for a in I.uniform_points(400_001, 3, 83, rdt)]
    st = B.lib().esn_setpts_noalloc(na.handle, 400_001, B.ESN_SINGLE if prec == "f32" else B.ESN_DOUBLE,
                                    *[B.vp(a.data_ptr()) for a in big])
    assert st == B.ESN_ERR_BAD_ARG
    assert na.info().device_bytes == room
    ref.close()
    na.close()


def test_setpts_noalloc_refuses_more_than_its_scratch():
    """A plan with room for 6e6 single-precision points: the sort's scratch for
    them exceeds the 128 MiB static array, so the call is refused."""
    t = torch()
    M = 6_000_000
    xs = [t.zeros(M, dtype=t.float32, device="cuda") for _ in range(3)]
    p = B.Plan(1, (32, 32, 32), 1e-6, sort=2)
    p.setpts(*xs)
    st = B.lib().esn_setpts_noalloc(p.handle, M, B.ESN_SINGLE, *[B.vp(a.data_ptr()) for a in xs])
    assert st == B.ESN_ERR_BAD_ARG
    # within the limit the same plan sorts without allocating
    st = B.lib().esn_setpts_noalloc(p.handle, 1_000_000, B.ESN_SINGLE,
                                    *[B.vp(a.data_ptr()) for a in xs])
    assert st == 0
    p.close()
