"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Holds no transform arithmetic: only random draws, shapes and band-limit masks.
The paper measures on random band-limited coefficients with the distribution
unstated (Sec. 6.3); these Gaussian draws stand in for them.

Recipe: ``numpy.random.default_rng(seed)``; draw the real parts, then the
imaginary parts, each with ``standard_normal(shape)``; optionally scale both by
``1/(1+l)``; zero every entry with ``l < max(|m|, |s|)`` (SO(3):
``l < max(|m|, |n|)``).  A second array (e.g. a gradient target) is drawn next
from the same generator.
"""
import numpy as np

__all__ = ["coeff_mask", "flm_gaussian", "flmn_gaussian", "map_gaussian", "serving_trace"]


def coeff_mask(L, spin=0):
    """Boolean [L, 2L-1] mask of valid (l, m) for spin s: l >= max(|m|, |s|)."""
    ell = np.arange(L)[:, None]
    m = np.arange(-(L - 1), L)[None, :]
    return (ell >= np.abs(m)) & (ell >= abs(spin))


def flm_gaussian(L, spin=0, seed=0, batch=None, scale=None, rng=None):
    """complex128 coefficients [batch?][L][2L-1], iid N(0,1) real and imaginary parts.

    scale: None or "inv1pl" (both parts multiplied by 1/(1+l))."""
    rng = np.random.default_rng(seed) if rng is None else rng
    shape = (L, 2 * L - 1) if batch is None else (batch, L, 2 * L - 1)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    out = re + 1j * im
    if scale == "inv1pl":
        out *= (1.0 / (1.0 + np.arange(L)))[:, None]
    elif scale is not None:
        raise ValueError(scale)
    out *= coeff_mask(L, spin)
    return out


def flmn_gaussian(L, N, seed=0, batch=None, rng=None):
    """complex128 Wigner coefficients [batch?][2N-1][L][2L-1], zero for l < max(|m|,|n|)."""
    rng = np.random.default_rng(seed) if rng is None else rng
    shape = (2 * N - 1, L, 2 * L - 1) if batch is None else (batch, 2 * N - 1, L, 2 * L - 1)
    out = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ell = np.arange(L)[None, :, None]
    m = np.arange(-(L - 1), L)[None, None, :]
    n = np.arange(-(N - 1), N)[:, None, None]
    out *= (ell >= np.abs(m)) & (ell >= np.abs(n))
    return out


def map_gaussian(shape, seed=0, rng=None):
    """complex128 array of the given shape with iid N(0,1) real and imaginary parts."""
    rng = np.random.default_rng(seed) if rng is None else rng
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def serving_trace(n_requests=10000, seed=3, rate=1.0, lmin=64, lmax=4096, so3_lmax=512,
                  so3_frac=0.2, healpix_frac=0.5):
    """Poisson arrival trace of mixed transform requests.

    Each request: arrival time (s, rate in requests/s), kind ('s2' or 'so3'),
    L (log-uniform in [lmin, lmax], rounded to even), spin in {0, 2},
    sampling ('mw' or 'healpix' with nside = L/2) and N in {1, 4, 8} for SO(3)
    (L log-uniform in [lmin, so3_lmax])."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps)
    reqs = []
    for i in range(n_requests):
        if rng.random() < so3_frac:
            L = int(round(np.exp(rng.uniform(np.log(lmin), np.log(so3_lmax))) / 2.0)) * 2
            reqs.append(dict(t=float(t[i]), kind="so3", L=max(L, 2), spin=0, sampling="mw",
                             N=int(rng.choice([1, 4, 8]))))
        else:
            L = int(round(np.exp(rng.uniform(np.log(lmin), np.log(lmax))) / 2.0)) * 2
            samp = "healpix" if rng.random() < healpix_frac else "mw"
            reqs.append(dict(t=float(t[i]), kind="s2", L=max(L, 2), spin=int(rng.choice([0, 2])),
                             sampling=samp, N=1))
    return reqs
