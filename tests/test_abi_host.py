"""Host-side checks of the C-ABI library: it loads without a GPU, exports every
symbol the header declares, and its plan arithmetic (no GPU calls) follows the
paper's rules:
* eq. (params): w = ceil(log10(1/eps)) + 1 and beta = 2.30 w;
* Sec. 3.1: n = smallest 2^a 3^b 5^c >= max(2N, 2w);
* Sec. 3.1 after eq. (quad): p >= 1.5 w + 2 positive Gauss-Legendre nodes.
The quadrature itself is pinned against numpy's Gauss-Legendre rule, scipy's
adaptive quadrature of the kernel's Fourier integral, and the closed-form
Fourier transform of the Kaiser-Bessel kernel (eqs. (KB), (KBhat)) computed
with the same Gauss-Legendre rule.
"""
import math
import os
import re

import numpy as np
import pytest

from paper_1808_06736_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


def header_symbols():
    text = open(os.path.join(ROOT, "include", "esnufft.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(esn_\w+)\s*\(", text)))


def test_library_loads_and_exports_header_symbols():
    L = B.lib()
    syms = header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(L, s), f"missing export {s}"
    # the binding wraps exactly the declared entry points
    assert set(B.exported_symbols()) >= set(syms) - set()


def test_strerror_and_default_opts():
    assert B.strerror(0) == "success"
    assert "NaN" in B.strerror(4)
    o = B.esn_default_opts()
    assert o.chkbnds == 1 and o.sort == 1 and o.upsampfac == 2.0 and o.modeord == 0


def _params(eps, prec=B.ESN_DOUBLE, dim=1, N=(100, 1, 1), sigma=2.0):
    st, p = B.esn_choose_params(eps, prec, dim, N, upsampfac=sigma)
    return st, p


@pytest.mark.parametrize("digits", range(1, 16))
def test_width_rule(digits):
    eps = 10.0 ** (-digits)
    st, p = _params(eps)
    assert st == 0
    assert p.w == max(2, digits + 1)
    assert abs(p.beta - 2.30 * p.w) < 1e-12
    assert p.nquad == math.ceil(1.5 * p.w + 2)
    # between powers of ten the width rounds up
    st, p2 = _params(eps * 3.0)
    assert p2.w == max(2, digits + 1)


def test_paper_width_examples():
    """Widths printed in the paper's parallel scaling discussion (Sec. 6):
    eps = 1e-12 touches 13^3 fine grid points, eps = 1e-3 touches 4^3."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "paper_widths.txt"))
            if l.strip() and not l.startswith("#")]
    assert rows
    for eps, dim, touched in rows:
        st, p = _params(float(eps), dim=int(dim), N=(50, 50, 50))
        assert p.w ** int(dim) == int(touched)


def _smooth(n):
    for q in (2, 3, 5):
        while n % q == 0:
            n //= q
    return n == 1


@pytest.mark.parametrize("N", [1, 2, 3, 7, 64, 100, 128, 129, 160, 255, 256, 999, 1000, 4097])
@pytest.mark.parametrize("eps", [1e-2, 1e-6, 1e-12])
def test_fine_grid_rule(N, eps):
    st, p = _params(eps, dim=3, N=(N, N + 1, 5))
    for m, Nm in enumerate((N, N + 1, 5)):
        n = p.nf[m]
        assert _smooth(n) and n >= 2 * Nm and n >= 2 * p.w
        # smallest such size
        assert not any(_smooth(k) for k in range(max(2 * Nm, 2 * p.w), n))


def test_status_codes():
    assert _params(1e-7, prec=B.ESN_SINGLE)[0] == B.ESN_WARN_EPS_TOO_SMALL
    assert _params(1e-6, prec=B.ESN_SINGLE)[0] == 0
    assert _params(1e-17)[0] == B.ESN_WARN_EPS_TOO_SMALL
    assert _params(1e-17)[1].w == 16
    assert _params(0.0)[0] == B.ESN_ERR_BAD_ARG
    assert _params(1e-6, dim=4)[0] == B.ESN_ERR_BAD_ARG
    assert _params(1e-6, N=(0, 1, 1))[0] == B.ESN_ERR_BAD_ARG
    st, _ = B.esn_choose_params(1e-6, B.ESN_DOUBLE, 1, (10, 1, 1), upsampfac=1.25)
    assert st == 0
    for sigma in (1.5, 1.0, 3.0):
        st, _ = B.esn_choose_params(1e-6, B.ESN_DOUBLE, 1, (10, 1, 1), upsampfac=sigma)
        assert st == B.ESN_ERR_BAD_ARG
    o = B.esn_default_opts()
    o.upsampfac = 1.25   # type 3 runs at sigma = 2 only, refused before any GPU use
    assert B.esn_makeplan(3, 2, None, 1, 1, 1e-6, B.ESN_DOUBLE, opts=o)[0] == B.ESN_ERR_BAD_ARG
    # bad args fail before any GPU use, type 3 ones included
    assert B.esn_makeplan(4, 1, (10,), 1, 1, 1e-6, B.ESN_DOUBLE)[0] == B.ESN_ERR_BAD_ARG
    assert B.esn_makeplan(3, 4, (10,), 1, 1, 1e-6, B.ESN_DOUBLE)[0] == B.ESN_ERR_BAD_ARG
    assert B.esn_makeplan(3, 2, None, 0, 1, 1e-6, B.ESN_DOUBLE)[0] == B.ESN_ERR_BAD_ARG
    assert B.esn_makeplan(3, 2, None, 1, 0, 1e-6, B.ESN_DOUBLE)[0] == B.ESN_ERR_BAD_ARG
    assert B.esn_makeplan(1, 1, (10,), 0, 1, 1e-6, B.ESN_DOUBLE)[0] == B.ESN_ERR_BAD_ARG
    assert B.esn_makeplan(1, 1, (10,), 1, 0, 1e-6, B.ESN_DOUBLE)[0] == B.ESN_ERR_BAD_ARG
    assert B.esn_makeplan(1, 1, (0,), 1, 1, 1e-6, B.ESN_DOUBLE)[0] == B.ESN_ERR_BAD_ARG


@pytest.mark.parametrize("p", [1, 2, 5, 11, 13, 17, 26])
def test_gauss_legendre_matches_numpy(p):
    q, w = B.esn_gauss_legendre(p)
    x, wn = np.polynomial.legendre.leggauss(2 * p)
    pos = x > 0
    order = np.argsort(-x[pos])
    assert np.max(np.abs(q - x[pos][order])) < 1e-14
    assert np.max(np.abs(w - wn[pos][order])) < 1e-14
    assert abs(2 * np.sum(w) - 2.0) < 1e-14
    # exact on even monomials up to degree 4p - 2
    for m in range(0, 2 * p):
        assert abs(2 * np.sum(w * q ** (2 * m)) - 2.0 / (2 * m + 1)) < 1e-13


def _phi_hat_quad(beta, xi):
    """scipy adaptive quadrature of int_{-1}^{1} phi(z) cos(xi z) dz."""
    from scipy.integrate import quad
    f = lambda z: math.exp(beta * (math.sqrt(max(1 - z * z, 0.0)) - 1.0)) * math.cos(xi * z)
    return 2 * quad(f, 0, 1, limit=400, epsabs=1e-15, epsrel=1e-13)[0]


@pytest.mark.parametrize("eps,N", [(1e-3, 64), (1e-6, 128), (1e-6, 1000), (1e-9, 301),
                                   (1e-12, 200)])
def test_correction_factors_against_scipy_quad(eps, N):
    st, p = _params(eps, N=(N, 1, 1))
    nf = p.nf[0]
    pk = B.esn_correction_factors(p.w, p.beta, p.nquad, nf, N)
    alpha = math.pi * p.w / nf
    ks = sorted(set([0, 1, N // 4, N // 3, N // 2]))
    for k in ks:
        ref = 2.0 / (p.w * _phi_hat_quad(p.beta, alpha * k))   # eq. (pk1)
        assert abs(pk[k] - ref) < eps * abs(ref), (k, pk[k], ref)


@pytest.mark.parametrize("w", [4, 7, 10, 13])
def test_quadrature_machinery_on_kaiser_bessel(w):
    """The same Gauss-Legendre rule applied to the KB kernel (eq. (KB)) must
    reproduce its closed-form transform (eq. (KBhat)) over |xi| <= pi w / 2."""
    from scipy.special import i0
    beta = 2.30 * w
    q, wq = B.esn_gauss_legendre(math.ceil(1.5 * w + 2))
    for xi in np.linspace(0, math.pi * w / 2, 7):
        kb = i0(beta * np.sqrt(1 - q * q)) / i0(beta)
        approx = 2 * np.sum(wq * kb * np.cos(xi * q))
        s = math.sqrt(beta * beta - xi * xi)
        exact = 2.0 / i0(beta) * math.sinh(s) / s
        assert abs(approx - exact) < 10 ** (-(w - 1)) * abs(exact)


@pytest.mark.parametrize("w", [7, 10, 13, 16])
def test_phi_hat_semicircle_asymptote(w):
    """eq. (EShat1): phi^(rho beta) ~ sqrt(2 pi / beta) (1 - rho^2)^(-3/4)
    exp(beta (sqrt(1 - rho^2) - 1)) up to a relative O(1/beta); and phi^ decreases
    monotonically on the usable band |xi| <= pi w / 4 (Remark r:heur's premise)."""
    beta = 2.30 * w
    nf = 1000
    pk = B.esn_correction_factors(w, beta, math.ceil(1.5 * w + 2), nf, nf - 1)
    alpha = math.pi * w / nf
    k = np.arange(len(pk))
    phihat = 2.0 / (w * pk)
    xi = alpha * k
    assert np.all(np.diff(phihat[xi <= math.pi * w / 4]) < 0)
    for rho in (0.0, 0.3, 0.6):
        kk = int(round(rho * beta / alpha))
        r = alpha * kk / beta
        asym = math.sqrt(2 * math.pi / beta) * (1 - r * r) ** -0.75 * math.exp(
            beta * (math.sqrt(1 - r * r) - 1))
        assert abs(phihat[kk] / asym - 1) < 3.0 / beta


def _phi(beta, z):
    """eq. (ES): exp(beta (sqrt(1 - z^2) - 1)) on |z| <= 1, 0 outside."""
    z = np.asarray(z, dtype=float)
    return np.where(np.abs(z) <= 1, np.exp(beta * (np.sqrt(np.maximum(1 - z * z, 0)) - 1)), 0.0)


@pytest.mark.parametrize("w", range(2, 17))
def test_kernel_poly_table_matches_kernel(w):
    """Sec. 5.3: w intervals, degree w + 3.  The table reproduces phi on every
    interval to well below the tolerance the width is chosen for
    (eps = 10^-(w-1); FP64 rounding bounds it at w = 15, 16), and a point's w
    window weights (window cells l0 .. l0 + w - 1, l0 = ceil(t - w/2)) come out
    of one shared local coordinate."""
    beta = 2.30 * w
    c = B.esn_kernel_poly(w, beta)
    assert c.shape == (w, w + 4)
    t = np.linspace(-1, 1, 2001)
    err = 0.0
    for k in range(w):
        z = (k + (t + 1) / 2 - w / 2) * (2 / w)
        approx = np.polynomial.polynomial.polyval(t, c[k])
        err = max(err, float(np.max(np.abs(approx - _phi(beta, z)))))
    assert err <= max(0.1 * 10.0 ** (-(w - 1)), 1e-14), err
    # window weights of a few points from the definition of the window
    for tp in (3.0, 3.25, 3.5, 3.5 + 1e-9, 3.75, 3.999):
        l0 = math.ceil(tp - w / 2)
        direct = _phi(beta, (l0 + np.arange(w) - tp) / (w / 2))
        u = l0 - tp + w / 2                  # in [0, 1)
        tt = 2 * u - 1
        table = np.array([np.polynomial.polynomial.polyval(tt, c[k]) for k in range(w)])
        assert np.max(np.abs(table - direct)) <= max(0.1 * 10.0 ** (-(w - 1)), 1e-14)


def test_kernel_poly_bad_args():
    for w, beta in ((1, 2.3), (17, 39.1), (7, 0.0)):
        with pytest.raises(B.EsnError):
            B.esn_kernel_poly(w, beta)
    o = B.esn_default_opts()
    assert o.kerevalmeth == 0
    o.kerevalmeth = 3   # rejected before any GPU use
    assert B.esn_makeplan(1, 1, (10,), 1, 1, 1e-6, B.ESN_DOUBLE, opts=o)[0] == B.ESN_ERR_BAD_ARG


def _phi_hat_gl(beta, xi, nodes=600):
    """int_{-1}^{1} phi(z) cos(xi z) dz by a 600-node Gauss-Legendre rule."""
    x, wq = np.polynomial.legendre.leggauss(nodes)
    phi = np.exp(beta * (np.sqrt(1 - x * x) - 1))
    return np.cos(np.outer(np.atleast_1d(xi), x)) @ (wq * phi)


def _aliasing_bound(w, beta, sigma):
    """eq. (epsest) for the ES kernel in scaled frequency u = k/n, |u| <= 1/(2 sigma):
    max_u sum_{0 < |m| <= 20} |phi^(pi w (u + m))| / min_u |phi^(pi w u)|."""
    us = np.linspace(0, 0.5 / sigma, 17)
    ms = np.array([m for m in range(-20, 21) if m])
    num = max(np.sum(np.abs(_phi_hat_gl(beta, math.pi * w * (u + ms)))) for u in us)
    return num / abs(_phi_hat_gl(beta, math.pi * w * 0.5 / sigma)[0])


def test_low_upsampling_rule():
    """sigma = 5/4: beta from eq. (gam) with the safety factor that gives 2.30 at
    sigma = 2; w from the rate of eq. (ESerr).  The aliasing bound of eq. (epsest)
    at the chosen w stays within 5 eps for eps = 1e-1 .. 1e-8 (the sigma = 2 rule
    keeps it within 2 to 9 eps), and one width less would exceed eps."""
    gam = 2.30 / (math.pi * 0.75)                      # sigma = 2: beta / w = 2.30
    assert abs(gam - 0.976) < 1e-3
    for digits in range(1, 9):
        eps = 10.0 ** -digits
        st, p = _params(eps, N=(200, 1, 1), sigma=1.25)
        assert st == 0
        assert abs(p.beta / p.w - 0.976 * math.pi * 0.6) < 1e-12
        bound = _aliasing_bound(p.w, p.beta, 1.25)
        assert bound <= 5 * eps, (eps, p.w, bound)
        if p.w > 2:
            w1 = p.w - 1
            assert _aliasing_bound(w1, 0.976 * math.pi * 0.6 * w1, 1.25) > eps
    # the same bound for the sigma = 2 rule of eq. (params), for comparison
    for digits in range(1, 13):
        st, p = _params(10.0 ** -digits, N=(200, 1, 1))
        assert 1.0 <= _aliasing_bound(p.w, p.beta, 2.0) / 10.0 ** -digits <= 10.0


@pytest.mark.parametrize("N", [1, 7, 64, 100, 129, 1000])
@pytest.mark.parametrize("eps", [1e-2, 1e-6])
def test_low_upsampling_fine_grid_and_factors(N, eps):
    st, p = _params(eps, dim=1, N=(N, 1, 1), sigma=1.25)
    n = p.nf[0]
    assert _smooth(n) and n >= 1.25 * N and n >= 2 * p.w
    assert not any(_smooth(k) for k in range(max(math.ceil(1.25 * N), 2 * p.w), n))
    pk = B.esn_correction_factors(p.w, p.beta, p.nquad, n, N)
    alpha = math.pi * p.w / n
    for k in sorted(set([0, N // 3, N // 2])):
        ref = 2.0 / (p.w * _phi_hat_quad(p.beta, alpha * k))   # eq. (pk1)
        assert abs(pk[k] - ref) < 0.01 * eps * abs(ref)


def test_toeplitz_bad_args_fail_before_gpu_use():
    for dim, N, isign, M in ((4, (8,), 1, 10), (1, (0,), 1, 10), (1, (8,), 0, 10),
                             (1, (8,), 1, -1)):
        st, h = B.esn_toeplitz_makeplan(dim, N, isign, 1e-6, B.ESN_DOUBLE, M, B.ESN_DOUBLE,
                                        [None])
        assert st == B.ESN_ERR_BAD_ARG and not h.value
    assert B.esn_toeplitz_apply(None, None, None) == B.ESN_ERR_BAD_ARG
    assert B.esn_toeplitz_destroy(None) == 0
