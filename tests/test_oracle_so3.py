"""Pins of the oracle's Wigner (SO(3)) transforms at n != 0.  CPU only.

Two independent routes fix what the oracle's so3_inverse / so3_forward must
return for every slice n, not only n = 0:

* Sec. 2.3, the slice identities: after the gamma analysis
  f_n = (1/(2N-1)) sum_k f(gamma_k) e^{-i n gamma_k}, slice n of the inverse
  is the inverse spin SHT at spin -n of (-1)^n sqrt((2l+1)/(16 pi^3)) flmn, and
  the forward of slice n is (-1)^n sqrt(4 pi/(2l+1)) times the forward spin
  SHT at spin -n of the gamma integral of f (weight 2 pi/(2N-1)).  The spin
  SHTs are the oracle's, themselves pinned by scipy's Y_lm, the spin-raising
  relation and exact round trips; the gamma analysis is written here.
* Eq. 13 with D^* = e^{i m alpha} d^l_{mn}(beta) e^{i n gamma} (Eq. 10) summed by
  brute force over every sample, d taken from the Jacobi form (Eq. 22) at 40
  digits, and the forward of such band-limited samples returning the
  coefficients.

Each test also evaluates the two plausible mistakes that a round trip cannot
see (n and -n swapped in both directions; the sign of the gamma phase flipped
in both directions) and asserts that they would miss the reference by far more
than the tolerance, so the pins are sensitive to them.
"""
import math

import numpy as np
import pytest

from paper_2311_14670_amd.synth import flmn_gaussian, map_gaussian


def _gammas(N):
    return 2 * np.pi * np.arange(2 * N - 1) / (2 * N - 1)


def _gamma_analysis(f, N, n, weight):
    """weight * sum_k f[k] e^{-i n gamma_k} over the leading (gamma) axis."""
    ph = np.exp(-1j * n * _gammas(N))
    return weight * np.tensordot(ph, f, axes=(0, 0))


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("L,N", [(8, 3), (10, 4), (12, 5)])
def test_so3_inverse_slice_is_spin_minus_n_sht(oracle, L, N):
    flmn = flmn_gaussian(L, N, seed=100 + L + N)
    f = oracle.so3_inverse(flmn, L, N)
    ell = np.arange(L)[:, None]
    scale = np.sqrt((2 * ell + 1) / (16 * np.pi ** 3))
    worst = 0.0
    for n in range(-(N - 1), N):
        fn = _gamma_analysis(f, N, n, 1.0 / (2 * N - 1))
        ref = oracle.s2_inverse((-1.0) ** n * scale * flmn[n + N - 1], L, -n)
        worst = max(worst, _rel(fn, ref))
        if n != 0:
            # n <-> -n in both directions: slice n would carry the spin +n transform
            wrong = oracle.s2_inverse((-1.0) ** n * scale * flmn[n + N - 1], L, n)
            assert _rel(wrong, ref) > 1e-2
            # gamma phase flipped in both directions: slice n would hold slice -n's content
            flipped = _gamma_analysis(f, N, -n, 1.0 / (2 * N - 1))
            assert _rel(flipped, ref) > 1e-2
    assert worst < 1e-13, worst


@pytest.mark.parametrize("L,N", [(8, 3), (10, 4), (12, 5)])
def test_so3_forward_slice_is_spin_minus_n_sht(oracle, L, N):
    """Holds for arbitrary (not band-limited) samples: both sides are the exact
    integrals of the MW interpolant."""
    f = map_gaussian((2 * N - 1, L, 2 * L - 1), seed=200 + L + N)
    flmn = oracle.so3_forward(f, L, N)
    ell = np.arange(L)[:, None]
    scale = np.sqrt(4 * np.pi / (2 * ell + 1))
    worst = 0.0
    for n in range(-(N - 1), N):
        fn = _gamma_analysis(f, N, n, 2 * np.pi / (2 * N - 1))
        ref = (-1.0) ** n * scale * oracle.s2_forward(fn, L, -n)
        worst = max(worst, _rel(flmn[n + N - 1], ref))
        if n != 0:
            wrong = (-1.0) ** n * scale * oracle.s2_forward(fn, L, n)
            assert _rel(wrong, ref) > 1e-2
            flipped = (-1.0) ** n * scale * oracle.s2_forward(
                _gamma_analysis(f, N, -n, 2 * np.pi / (2 * N - 1)), L, -n)
            assert _rel(flipped, ref) > 1e-2
    assert worst < 1e-13, worst


# ------------------------------------------------------------------ brute force
def _jacobi_d(l, m, n, b):
    """Eq. 22 at 40 digits (factorial denominator read as (s+mu)!(s+nu)!)."""
    import mpmath as mp
    mp.mp.dps = 40
    mu, nu = abs(m - n), abs(m + n)
    s = l - (mu + nu) // 2
    zeta = 1 if n >= m else (-1) ** (n - m)
    pref = mp.sqrt(mp.factorial(s) * mp.factorial(s + mu + nu) /
                   (mp.factorial(s + mu) * mp.factorial(s + nu)))
    bb = mp.mpf(b)
    return float(zeta * pref * mp.sin(bb / 2) ** mu * mp.cos(bb / 2) ** nu * mp.jacobi(s, mu, nu, mp.cos(bb)))


def _mw_betas(L):
    return [(2 * t + 1) * math.pi / (2 * L - 1) for t in range(L)]


def _brute_matrix(L, N, n_sign=1, gamma_sign=1):
    """Dense Eq. 13 operator [(k,t,p)] x [(n,l,m)]: (2l+1)/(8 pi^2) e^{i m alpha_p}
    d^l_{m, n_sign*n}(beta_t) e^{i gamma_sign n gamma_k}.  n_sign = gamma_sign = 1
    is the paper's definition; -1 plants the mistakes the pins must catch."""
    G, M = 2 * N - 1, 2 * L - 1
    betas = _mw_betas(L)
    alphas = 2 * np.pi * np.arange(M) / M
    gammas = _gammas(N)
    A = np.zeros((G, L, M, G, L, M), dtype=np.complex128)
    for n in range(-(N - 1), N):
        for l in range(L):
            if l < abs(n):
                continue
            for m in range(-l, l + 1):
                d = np.array([_jacobi_d(l, m, n_sign * n, b) for b in betas])       # [t]
                col = ((2 * l + 1) / (8 * np.pi ** 2)
                       * np.exp(1j * gamma_sign * n * gammas)[:, None, None]
                       * d[None, :, None]
                       * np.exp(1j * m * alphas)[None, None, :])
                A[:, :, :, n + N - 1, l, m + L - 1] = col
    return A.reshape(G * L * M, G * L * M)


@pytest.mark.parametrize("L,N", [(5, 2), (6, 3)])
def test_so3_brute_force_jacobi(oracle, L, N):
    flmn = flmn_gaussian(L, N, seed=300 + L + N)
    A = _brute_matrix(L, N)
    ref = (A @ flmn.reshape(-1)).reshape(2 * N - 1, L, 2 * L - 1)
    f = oracle.so3_inverse(flmn, L, N)
    assert np.max(np.abs(f - ref)) / np.max(np.abs(ref)) < 1e-13
    # the forward of band-limited samples returns their coefficients
    back = oracle.so3_forward(ref, L, N)
    assert np.max(np.abs(back - flmn)) / np.max(np.abs(flmn)) < 1e-13
    # sensitivity: either planted mistake moves the samples by O(1)
    for ns, gs in [(-1, 1), (1, -1), (-1, -1)]:
        wrong = (_brute_matrix(L, N, ns, gs) @ flmn.reshape(-1)).reshape(ref.shape)
        assert _rel(wrong, ref) > 1e-2
        # and the oracle's forward does not invert the mistaken operator
        assert _rel(oracle.so3_forward(wrong, L, N), flmn) > 1e-2
