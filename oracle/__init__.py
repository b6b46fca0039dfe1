"""CPU oracle for the spin spherical-harmonic and Wigner transforms.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.  The heavy
lifting is plain C (``s2oracle.c``: direct sums, Wigner-d by a recursion in
degree l, exact Gauss-Legendre quadrature for the MW forward transform); this
module only marshals numpy arrays through ctypes.

Arrays are numpy ``complex128``.  Layouts:
  * spherical-harmonic coefficients ``flm[l, m + L - 1]`` (zeros for
    ``l < max(|m|, |s|)``);
  * MW maps ``f[t, p]`` with ``theta_t = (2t+1) pi/(2L-1)``,
    ``phi_p = 2 pi p/(2L-1)`` (paper Sec. 4.2, MW);
  * HEALPix maps as the RING-ordered pixel vector;
  * DH maps ``f[t, p]`` with ``theta_t = (2t+1) pi/(4L)``, t < 2L, and GL maps
    ``f[t, p]`` with ``cos(theta_t)`` the roots of P_L (theta ascending), both
    with ``phi_p = 2 pi p/(2L-1)`` (Sec. 4.2, DH and GL sampling theorems);
  * MWSS maps ``f[t, p]`` with ``theta_t = pi t/L``, t = 0..L (both poles), and
    ``phi_p = 2 pi p/(2L)`` (Sec. 4.2, MW with symmetric sampling);
  * Wigner coefficients ``flmn[n + N - 1, l, m + L - 1]`` and SO(3) maps
    ``f[k, t, p]`` with ``gamma_k = 2 pi k/(2N-1)`` (Sec. 4.5).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "s2oracle.c")
_LIB = os.path.join(_HERE, "_s2oracle.so")
_lib = None

MW, HEALPIX, DH, GL, MWSS = 0, 1, 2, 3, 4


def build(force=True):
    """Compile the oracle with gcc (-O3, OpenMP)."""
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lp = ctypes.POINTER(ctypes.c_longlong)
    i = ctypes.c_int
    lib.or_mw_thetas.argtypes = [i, dp]
    lib.or_healpix_rings.argtypes = [i, dp, ip, lp, ip]
    lib.or_gauss_legendre.argtypes = [i, dp, dp]
    lib.or_wigner_d_ell.argtypes = [i, i, i, ctypes.c_double, dp]
    lib.or_s2_inverse.argtypes = [i, i, i, i, dp, dp, i, ip]
    lib.or_s2_forward.argtypes = [i, i, i, i, dp, dp, i, ip]
    lib.or_s2_inverse_adjoint.argtypes = [i, i, i, i, dp, dp, i, ip]
    lib.or_so3_inverse.argtypes = [i, i, dp, dp]
    lib.or_so3_forward.argtypes = [i, i, dp, dp]
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _sel(sel):
    if sel is None:
        return -1, None
    arr = np.ascontiguousarray(np.asarray(sel, dtype=np.int32))
    return int(arr.size), arr


# ----------------------------------------------------------------- geometry
def mw_thetas(L):
    """MW colatitudes theta_t = (2t+1) pi/(2L-1), t < L (Sec. 4.2)."""
    out = np.empty(L)
    _load().or_mw_thetas(L, _dp(out))
    return out


def healpix_rings(nside):
    """HEALPix RING geometry: (theta, nphi, start, shift) per ring."""
    nr = 4 * nside - 1
    th = np.empty(nr)
    nphi = np.empty(nr, dtype=np.int32)
    start = np.empty(nr, dtype=np.int64)
    shift = np.empty(nr, dtype=np.int32)
    _load().or_healpix_rings(nside, _dp(th), _ip(nphi),
                             start.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), _ip(shift))
    return th, nphi, start, shift


def healpix_phis(nside):
    """Longitude of every RING-ordered pixel: phi_j = (pi/nphi)(2j + shift)."""
    th, nphi, start, shift = healpix_rings(nside)
    out = np.empty(12 * nside * nside)
    for r in range(th.size):
        j = np.arange(nphi[r])
        out[start[r]:start[r] + nphi[r]] = np.pi * (2 * j + shift[r]) / nphi[r]
    return out


def gauss_legendre(n):
    x = np.empty(n)
    w = np.empty(n)
    _load().or_gauss_legendre(n, _dp(x), _dp(w))
    return x, w


def dh_nodes(L):
    """DH colatitudes (2t+1) pi/(4L), t < 2L, and theta weights w_t with
    sum_t w_t g(theta_t) = int_0^pi g sin(theta) for g of degree < 2L in cos(theta)."""
    th, w = np.empty(2 * L), np.empty(2 * L)
    _load().or_dh_nodes(L, _dp(th), _dp(w))
    return th, w


def gl_nodes(L):
    """GL colatitudes (cos(theta) = roots of P_L, theta ascending) and weights in cos(theta)."""
    th, w = np.empty(L), np.empty(L)
    _load().or_gl_nodes(L, _dp(th), _dp(w))
    return th, w


def num_rings(L, sampling, nside=0):
    return {MW: L, DH: 2 * L, GL: L, MWSS: L + 1}.get(sampling, 4 * nside - 1)


def ring_length(L, sampling):
    """Samples per ring of the equiangular-phi samplings."""
    return 2 * L if sampling == MWSS else 2 * L - 1


def map_size(L, sampling, nside=0):
    if sampling == HEALPIX:
        return 12 * nside * nside
    return num_rings(L, sampling) * ring_length(L, sampling)


# ----------------------------------------------------------------- Wigner d
def wigner_d(L, m, n, beta):
    """d^l_{mn}(beta) for l = 0..L-1 (independent l-recursion)."""
    out = np.empty(L)
    _load().or_wigner_d_ell(L, int(m), int(n), float(beta), _dp(out))
    return out


# ----------------------------------------------------------------- S2 transforms
def s2_inverse(flm, L, spin=0, sampling=MW, nside=0, rings=None):
    """Inverse spin SHT by direct summation (Eqs. 4, 32-33).

    Returns the MW / DH / GL map [rings, 2L-1] or the HEALPix pixel vector, or,
    with ``rings``, the concatenated samples of the selected rings."""
    flm = _c128(flm)
    assert flm.shape == (L, 2 * L - 1)
    lib = _load()
    nsel, sel = _sel(rings)
    if sampling != HEALPIX:
        nout = (num_rings(L, sampling) if nsel < 0 else nsel) * ring_length(L, sampling)
    else:
        _, nphi, _, _ = healpix_rings(nside)
        nout = int(nphi.sum()) if nsel < 0 else int(nphi[np.asarray(rings)].sum())
    f = np.empty(nout, dtype=np.complex128)
    lib.or_s2_inverse(L, spin, sampling, nside, _dp(flm.view(np.float64)), _dp(f.view(np.float64)),
                      nsel, _ip(sel) if sel is not None else None)
    if sampling != HEALPIX and nsel < 0:
        return f.reshape(num_rings(L, sampling), ring_length(L, sampling))
    return f


def s2_forward(f, L, spin=0, sampling=MW, nside=0, ms=None):
    """Forward spin SHT: exact MW transform (GL route), HEALPix quadrature, or the
    DH / GL sampling theorems' quadratures (exact for band-limited maps).

    With ``ms`` only those order columns are computed (others are zero)."""
    f = _c128(f).reshape(-1)
    assert f.size == map_size(L, sampling, nside)
    flm = np.empty((L, 2 * L - 1), dtype=np.complex128)
    nsel, sel = _sel(ms)
    _load().or_s2_forward(L, spin, sampling, nside, _dp(f.view(np.float64)), _dp(flm.view(np.float64)),
                          nsel, _ip(sel) if sel is not None else None)
    return flm


def s2_inverse_adjoint(g, L, spin=0, sampling=MW, nside=0, ms=None):
    """Hermitian adjoint of the inverse SHT: sum_{t,p} g conj(sY_lm)."""
    g = _c128(g).reshape(-1)
    assert g.size == map_size(L, sampling, nside)
    out = np.empty((L, 2 * L - 1), dtype=np.complex128)
    nsel, sel = _sel(ms)
    _load().or_s2_inverse_adjoint(L, spin, sampling, nside, _dp(g.view(np.float64)),
                                  _dp(out.view(np.float64)), nsel, _ip(sel) if sel is not None else None)
    return out


# ----------------------------------------------------------------- real signals
def hermitian_complete(flm, L):
    """Coefficients of a real spin-0 signal from their orders m >= 0: the
    Hermitian symmetry of Sec. 2.1, flm[l, -m] = (-1)^m conj(flm[l, m]), with
    order 0 taken real.  The orders m < 0 of the input are not read."""
    out = np.array(_c128(flm), copy=True)
    assert out.shape == (L, 2 * L - 1)
    for m in range(1, L):
        out[:, L - 1 - m] = (-1.0) ** m * np.conj(out[:, L - 1 + m])
    out[:, L - 1] = out[:, L - 1].real
    return out


def s2_inverse_real(flm, L, sampling=MW, nside=0, rings=None):
    """Real map of a spin-0 signal given by its orders m >= 0: the inverse SHT
    of the Hermitian completion (a real map up to rounding), real part."""
    return s2_inverse(hermitian_complete(flm, L), L, 0, sampling, nside, rings=rings).real


def s2_forward_real(f, L, sampling=MW, nside=0, ms=None):
    """Forward SHT of a real map (the complex transform of the same samples)."""
    return s2_forward(np.asarray(f, dtype=np.float64).astype(np.complex128), L, 0, sampling, nside, ms=ms)


# ----------------------------------------------------------------- SO(3) transforms
def so3_inverse(flmn, L, N):
    """Inverse Wigner transform (Eq. 13), MW in (beta, alpha), 2N-1 gammas."""
    flmn = _c128(flmn)
    assert flmn.shape == (2 * N - 1, L, 2 * L - 1)
    f = np.empty((2 * N - 1, L, 2 * L - 1), dtype=np.complex128)
    _load().or_so3_inverse(L, N, _dp(flmn.view(np.float64)), _dp(f.view(np.float64)))
    return f


def so3_forward(f, L, N):
    """Forward Wigner transform (Eq. 14), exact for MW sampling."""
    f = _c128(f)
    assert f.shape == (2 * N - 1, L, 2 * L - 1)
    flmn = np.empty((2 * N - 1, L, 2 * L - 1), dtype=np.complex128)
    _load().or_so3_forward(L, N, _dp(f.view(np.float64)), _dp(flmn.view(np.float64)))
    return flmn
