"""Pins of the oracle's Wigner-d against closed forms, textbook special cases,
high-precision Jacobi polynomials (Eq. 22) and unitarity.  CPU only."""
import math

import numpy as np
import pytest
import scipy.special as sp

BETAS = [1e-3, 0.05, 0.7, 1.3, math.pi / 2, 2.2, 3.0, math.pi - 1e-3]


@pytest.mark.parametrize("b", BETAS)
def test_closed_forms_low_degree(oracle, b):
    """d^1 and d^2 entries in closed form (Eq. 27 plus the index symmetries)."""
    L = 4
    d = lambda m, n: oracle.wigner_d(L, m, n, b)
    cb, sb = math.cos(b), math.sin(b)
    assert d(1, 1)[1] == pytest.approx((1 + cb) / 2, abs=1e-15)
    assert d(1, 0)[1] == pytest.approx(-sb / math.sqrt(2), abs=1e-15)
    assert d(1, -1)[1] == pytest.approx((1 - cb) / 2, abs=1e-15)
    assert d(0, 0)[1] == pytest.approx(cb, abs=1e-15)
    assert d(0, 1)[1] == pytest.approx(sb / math.sqrt(2), abs=1e-15)
    assert d(2, 0)[2] == pytest.approx(math.sqrt(3 / 8) * sb * sb, abs=1e-15)
    assert d(2, 1)[2] == pytest.approx(-(1 + cb) * sb / 2, abs=1e-15)
    assert d(2, -1)[2] == pytest.approx(-(1 - cb) * sb / 2, abs=1e-15)
    assert d(0, 0)[0] == 1.0


@pytest.mark.parametrize("l", [3, 10, 57])
def test_extreme_orders(oracle, l):
    """d^l_{ll} = cos^{2l}(b/2), d^l_{l,-l} = sin^{2l}(b/2)."""
    for b in [0.3, 1.1, 2.5]:
        assert oracle.wigner_d(l + 1, l, l, b)[l] == pytest.approx(math.cos(b / 2) ** (2 * l), rel=1e-13)
        assert oracle.wigner_d(l + 1, l, -l, b)[l] == pytest.approx(math.sin(b / 2) ** (2 * l), rel=1e-13)


def test_poles(oracle):
    """Eqs. 28-29 at the poles, and continuity of the recursion next to them."""
    L = 12
    for m in range(-3, 4):
        for n in range(-3, 4):
            d0 = oracle.wigner_d(L, m, n, 0.0)
            dpi = oracle.wigner_d(L, m, n, math.pi)
            l0 = max(abs(m), abs(n))
            for l in range(l0, L):
                assert d0[l] == (1.0 if m == n else 0.0)
                assert dpi[l] == ((-1.0) ** (l + m) if m == -n else 0.0)
            # just off the poles the generic path must agree to O(beta)
            assert np.allclose(oracle.wigner_d(L, m, n, 1e-9)[l0:], d0[l0:], atol=1e-7)
            assert np.allclose(oracle.wigner_d(L, m, n, math.pi - 1e-9)[l0:], dpi[l0:], atol=1e-7)


@pytest.mark.parametrize("b", [0.01, 0.4, 1.2, 2.9])
def test_legendre_special_cases(oracle, b):
    """d^l_{00} = P_l(cos b); d^l_{m0} = sqrt((l-m)!/(l+m)!) P_l^m(cos b) with Condon-Shortley phase."""
    L = 60
    x = math.cos(b)
    d00 = oracle.wigner_d(L, 0, 0, b)
    assert np.allclose(d00, sp.eval_legendre(np.arange(L), x), atol=2e-15)
    for m in [1, 2, 5, 13]:
        d = oracle.wigner_d(L, m, 0, b)
        ell = np.arange(m, L)
        norm = np.exp(0.5 * (sp.gammaln(ell - m + 1) - sp.gammaln(ell + m + 1)))
        ref = norm * sp.lpmv(m, ell, x)          # scipy includes the Condon-Shortley phase
        assert np.allclose(d[m:], ref, atol=1e-13), np.max(np.abs(d[m:] - ref))


def test_scalar_harmonics_match_scipy(oracle):
    """Eq. 1: Y_lm(theta, phi) = sqrt((2l+1)/4pi) e^{i m phi} d^l_{m0}(theta)."""
    L = 24
    for th in [0.2, 1.0, 2.6]:
        for m in [-7, -1, 0, 3, 11]:
            d = oracle.wigner_d(L, m, 0, th)
            for l in range(abs(m), L):
                y = math.sqrt((2 * l + 1) / (4 * math.pi)) * d[l] * np.exp(1j * m * 0.37)
                ref = sp.sph_harm_y(l, m, th, 0.37)
                assert abs(y - ref) < 1e-13


def _jacobi_d(l, m, n, b):
    """Eq. 22 at 50 digits (factorial denominator read as (s+mu)!(s+nu)!)."""
    import mpmath as mp
    mp.mp.dps = 50
    mu, nu = abs(m - n), abs(m + n)
    s = l - (mu + nu) // 2
    zeta = 1 if n >= m else (-1) ** (n - m)
    pref = mp.sqrt(mp.factorial(s) * mp.factorial(s + mu + nu) /
                   (mp.factorial(s + mu) * mp.factorial(s + nu)))
    bb = mp.mpf(b)
    return zeta * pref * mp.sin(bb / 2) ** mu * mp.cos(bb / 2) ** nu * mp.jacobi(s, mu, nu, mp.cos(bb))


@pytest.mark.parametrize("l,m,n,b", [
    (7, 3, -2, 0.9), (40, 0, 0, 0.05), (40, 17, 2, 1.7), (120, 60, -3, 0.4),
    (300, 5, 2, 0.02), (300, 150, -2, 3.1), (300, 299, 0, 1.5), (250, -40, 2, 2.0)])
def test_jacobi_high_precision(oracle, l, m, n, b):
    d = oracle.wigner_d(l + 1, m, n, b)[l]
    ref = float(_jacobi_d(l, m, n, b))
    assert abs(d - ref) < 1e-13, (d, ref)


@pytest.mark.parametrize("n", [0, 2, -2, 5])
@pytest.mark.parametrize("b", [7.7e-4, 0.05, 1.0, math.pi / 2, 3.14])
def test_unitarity_and_orthogonality(oracle, n, b):
    """sum_m d^l_{mn}^2 = 1 (the addition theorem) and sum_m d_{mn} d_{mn'} = delta."""
    L = 600
    D = np.array([oracle.wigner_d(L, m, n, b) for m in range(-(L - 1), L)])   # [m][l]
    l = np.arange(abs(n), L)
    s = (D[:, abs(n):] ** 2).sum(axis=0)
    assert np.max(np.abs(s - 1.0)) < 5e-13
    D2 = np.array([oracle.wigner_d(L, m, n + 1, b) for m in range(-(L - 1), L)])
    cross = (D[:, abs(n) + 1:] * D2[:, abs(n) + 1:]).sum(axis=0)
    assert np.max(np.abs(cross)) < 5e-13
    del l


@pytest.mark.slow
def test_unitarity_high_degree(oracle):
    """Unitarity at l up to 2047 for a polar, a mid and an equatorial colatitude."""
    L = 2048
    for b in [math.pi / 4095, 0.8, math.pi / 2]:
        acc = np.zeros(L)
        for m in range(-(L - 1), L):
            acc += oracle.wigner_d(L, m, 0, b) ** 2
        assert np.max(np.abs(acc - 1.0)) < 2e-12


def test_index_symmetries(oracle):
    """d^l_{mn} = (-1)^{m-n} d^l_{nm} = d^l_{-n,-m}."""
    L = 50
    for (m, n) in [(3, 1), (-4, 2), (7, -7), (0, 5)]:
        a = oracle.wigner_d(L, m, n, 1.1)
        b = oracle.wigner_d(L, n, m, 1.1)
        c = oracle.wigner_d(L, -n, -m, 1.1)
        assert np.allclose(a, (-1) ** (m - n) * b, atol=1e-15)
        assert np.allclose(a, c, atol=1e-15)
