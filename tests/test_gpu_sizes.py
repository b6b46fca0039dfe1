"""GPU parity beyond the small cases: sizes spanning several workgroups with
ragged tails (full oracle comparison), and the benchmark's full sizes in the
benchmark's launch configuration (oracle on sampled rings / orders, plus the
round-trip property that holds at any size)."""
import numpy as np
import pytest
import torch

import oracle
from conftest import fp64_err
from paper_2311_14670_amd.synth import flm_gaussian, flmn_gaussian, map_gaussian, coeff_mask

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(x):
    torch.cuda.synchronize()
    return x.cpu().numpy()


@pytest.fixture(scope="module")
def binding():
    from paper_2311_14670_amd import binding as b
    b.load_library()
    return b


# --------------------------------------------------------------- several tiles, full oracle
@pytest.mark.parametrize("L,spin", [(200, 0), (131, 2), (97, -3)])
def test_mw_multi_tile(binding, L, spin):
    flm = flm_gaussian(L, spin, seed=10, scale="inv1pl")
    plan = binding.Plan(L, spin=spin)
    f = host(plan.inverse(dev(flm)))
    assert fp64_err(f, oracle.s2_inverse(flm, L, spin)) < 1e-12
    g = map_gaussian((L, 2 * L - 1), seed=11)
    a = host(plan.forward(dev(g)))
    assert fp64_err(a, oracle.s2_forward(g, L, spin)) < 1e-12
    adj = host(plan.inverse_adjoint(dev(g)))
    assert fp64_err(adj, oracle.s2_inverse_adjoint(g, L, spin)) < 1e-12


@pytest.mark.parametrize("nside,L,spin", [(32, 64, 0), (24, 50, 2)])
def test_healpix_multi_tile(binding, nside, L, spin):
    flm = flm_gaussian(L, spin, seed=12)
    plan = binding.Plan(L, spin=spin, sampling="healpix", nside=nside)
    f = host(plan.inverse(dev(flm)))
    assert fp64_err(f, oracle.s2_inverse(flm, L, spin, oracle.HEALPIX, nside)) < 1e-12
    g = map_gaussian(12 * nside * nside, seed=13)
    a = host(plan.forward(dev(g)))
    assert fp64_err(a, oracle.s2_forward(g, L, spin, oracle.HEALPIX, nside)) < 1e-12


_SAMP = {"dh": oracle.DH, "gl": oracle.GL, "mwss": oracle.MWSS}


@pytest.mark.parametrize("sampling,L,spin", [("dh", 130, 0), ("gl", 150, 2), ("mwss", 140, -2)])
def test_dh_gl_multi_tile(binding, sampling, L, spin):
    samp = _SAMP[sampling]
    flm = flm_gaussian(L, spin, seed=19, scale="inv1pl")
    plan = binding.Plan(L, spin=spin, sampling=sampling)
    f = host(plan.inverse(dev(flm)))
    assert fp64_err(f, oracle.s2_inverse(flm, L, spin, samp)) < 1e-12
    assert fp64_err(host(plan.forward(dev(f))), flm) < 1e-12     # sampling theorem: exact round trip


@pytest.mark.parametrize("sampling,L", [("dh", 1024), ("gl", 2048), ("mwss", 2048)])
def test_dh_gl_full_size_sampled(binding, sampling, L):
    samp = _SAMP[sampling]
    flm = flm_gaussian(L, 0, seed=20, scale="inv1pl")
    plan = binding.Plan(L, sampling=sampling)
    f = plan.inverse(dev(flm))
    nr = oracle.num_rings(L, samp)
    rings = np.array(sorted({0, 1, nr // 3, nr // 2, nr - 2, nr - 1}))
    fr = host(f)[rings].ravel()
    assert fp64_err(fr, oracle.s2_inverse(flm, L, 0, samp, rings=rings)) < 1e-11
    assert fp64_err(host(plan.forward(f)), flm) < 1e-11


def test_so3_multi_tile(binding):
    L, N = 72, 4
    flmn = flmn_gaussian(L, N, seed=14)
    plan = binding.Plan(L, N=N)
    f = host(plan.so3_inverse(dev(flmn)))
    assert fp64_err(f, oracle.so3_inverse(flmn, L, N)) < 1e-12
    back = host(plan.so3_forward(dev(f)))
    assert fp64_err(back, flmn) < 1e-12


def test_batch_with_ragged_sizes(binding):
    """Batch 5 through a plan sized for 8, against per-map oracle results."""
    L, spin = 70, 1
    flm = flm_gaussian(L, spin, seed=15, batch=5)
    plan = binding.Plan(L, spin=spin, max_batch=8)
    f = host(plan.inverse(dev(flm)))
    for b in range(5):
        assert fp64_err(f[b], oracle.s2_inverse(flm[b], L, spin)) < 1e-12
    a = host(plan.forward(dev(f)))
    assert fp64_err(a, flm) < 1e-12


@pytest.mark.parametrize("L", [2, 3, 9])
def test_smallest_bandlimits(binding, L):
    for spin in range(-(L - 1), L):
        tol = 1e-13 if abs(spin) <= 3 else 1e-12      # as the sibling parity tests (stable-direction remedy)
        flm = flm_gaussian(L, spin, seed=16)
        plan = binding.Plan(L, spin=spin)
        f = host(plan.inverse(dev(flm)))
        assert fp64_err(f, oracle.s2_inverse(flm, L, spin)) < tol, spin
        assert fp64_err(host(plan.forward(dev(f))), flm) < tol, spin


def test_batch_larger_than_plan_is_rejected(binding):
    plan = binding.Plan(16, max_batch=2)
    x = torch.zeros((3, 16, 31), dtype=torch.complex128, device="cuda")
    with pytest.raises(binding.S2Error):
        plan.inverse(x)


# --------------------------------------------------------------- full sizes, sampled
def _sample_rings(L):
    """One ring in every 64-ring block of the inverse sweep (its lanes), at an
    offset that moves from block to block, plus both sides of the first and the
    middle block boundaries and the last rings (south pole included).  Every
    sampled ring sums the partials of every degree block."""
    rings = {64 * k + (23 * k + 5) % 64 for k in range((L + 63) // 64)}
    rings |= {0, 1, 63, 64, L // 2 - 1, L // 2, L - 3, L - 2, L - 1}
    return np.array(sorted(r for r in rings if 0 <= r < L))


def _sample_orders(L):
    """Orders at both ends of the 8-degree chunks and the 64-degree lane groups
    (where chunks start and lane groups change), spread over the whole range and
    both signs, plus the extremes.  Every sampled order's column holds every
    degree, so it sums every ring block and degree group of the forward sweep."""
    ms = {0, 1, -1, 2, 7, 8, -8, L - 2, L - 1, -(L - 1), L // 2, -(L // 3)}
    step = max(64, (L // 8) // 64 * 64)
    for j in range(64, L, step):
        ms |= {j - 1, j, -(j + 7)}
    return np.array(sorted(m for m in ms if -L < m < L))


# L = 2049 and 4096: the ring DFT length 2L - 1 (4097 = 17 x 241, 8191 prime) needs a
# Bluestein convolution of 16384 points, run as two LDS-resident halves
@pytest.mark.parametrize("L,spin", [(2048, 0), (1024, 2), (2049, 0), (4096, 0), (2100, 2)])
def test_mw_full_size_sampled(binding, L, spin):
    flm = flm_gaussian(L, spin, seed=1, scale="inv1pl")
    plan = binding.Plan(L, spin=spin)                # benchmark configuration: batch 1
    x = dev(flm)
    f = plan.inverse(x)
    rings = _sample_rings(L)
    fr = host(f)[rings].ravel()
    assert fp64_err(fr, oracle.s2_inverse(flm, L, spin, rings=rings)) < 1e-11
    back = host(plan.forward(f))
    assert fp64_err(back, flm) < 1e-11                 # holds at any size
    g = map_gaussian((L, 2 * L - 1), seed=17)
    a = host(plan.forward(dev(g)))
    ms = _sample_orders(L)
    ref = oracle.s2_forward(g, L, spin, ms=ms)
    cols = ms + L - 1
    assert fp64_err(a[:, cols], ref[:, cols]) < 1e-11
    assert np.all(a[~coeff_mask(L, spin)] == 0)


@pytest.mark.parametrize("nside,L", [(1024, 2048), (1100, 2200)])
def test_healpix_full_size_sampled(binding, nside, L):
    spin = 0                                         # nside 1100: cap rings up to 4396 points (split Bluestein)
    flm = flm_gaussian(L, spin, seed=18, scale="inv1pl")
    plan = binding.Plan(L, spin=spin, sampling="healpix", nside=nside)
    f = host(plan.inverse(dev(flm)))
    theta, nphi, start, _ = oracle.healpix_rings(nside)
    rings = np.array([0, 1, nside - 1, nside, 2 * nside - 1, 3 * nside, 4 * nside - 2])
    fr = np.concatenate([f[start[r]:start[r] + nphi[r]] for r in rings])
    assert fp64_err(fr, oracle.s2_inverse(flm, L, spin, oracle.HEALPIX, nside, rings=rings)) < 1e-11
    a = host(plan.forward(dev(f)))
    ms = _sample_orders(L)
    ref = oracle.s2_forward(f, L, spin, oracle.HEALPIX, nside, ms=ms)
    cols = ms + L - 1
    assert fp64_err(a[:, cols], ref[:, cols]) < 1e-11


def test_empty_batch_is_a_no_op(binding):
    plan = binding.Plan(16, max_batch=4)
    x = torch.zeros((0, 16, 31), dtype=torch.complex128, device="cuda")
    for fn in (plan.inverse, plan.forward, plan.inverse_adjoint, plan.forward_adjoint):
        y = fn(x)
        assert y.shape == (0, 16, 31)
    assert plan.inverse_real(x).shape == (0, 16, 31)
    assert plan.forward_real(torch.zeros((0, 16, 31), dtype=torch.float64, device="cuda")).shape == (0, 16, 31)
    so3 = binding.Plan(8, N=2)
    assert so3.so3_inverse(torch.zeros((0, 3, 8, 15), dtype=torch.complex128, device="cuda")).shape == (0, 3, 8, 15)


@pytest.mark.parametrize("nside,L", [(1, 2), (1, 4), (2, 3)])
def test_smallest_healpix(binding, nside, L):
    """nside 1: 12 pixels on 3 rings (4 pixels each); band-limits above what the
    grid resolves are still computed as defined (the quadrature of Eq. 19)."""
    for spin in range(-(L - 1), L):
        flm = flm_gaussian(L, spin, seed=19)
        plan = binding.Plan(L, spin=spin, sampling="healpix", nside=nside)
        f = host(plan.inverse(dev(flm)))
        assert fp64_err(f, oracle.s2_inverse(flm, L, spin, oracle.HEALPIX, nside)) < 1e-12, spin
        g = map_gaussian(12 * nside * nside, seed=20)
        a = host(plan.forward(dev(g)))
        assert fp64_err(a, oracle.s2_forward(g, L, spin, oracle.HEALPIX, nside)) < 1e-12, spin


# --------------------------------------------------------------- mirror-ring sweep (spin 0, symmetric grids)
# forced on at sizes of a few tiles: odd ring counts put the equator in a pair of
# its own, ragged last tiles, and every path that runs the inverse sweep
@pytest.mark.parametrize("sampling,L,nside", [("dh", 70, 0), ("gl", 131, 0), ("gl", 64, 0), ("mwss", 130, 0),
                                              ("mwss", 65, 0), ("healpix", 100, 48)])
def test_mirror_ring_sweep(binding, monkeypatch, sampling, L, nside):
    samp = {"dh": oracle.DH, "gl": oracle.GL, "mwss": oracle.MWSS, "healpix": oracle.HEALPIX}[sampling]
    monkeypatch.setenv("S2MI_RING_PAIRING", "1")
    plan = binding.Plan(L, sampling=sampling, nside=nside, max_batch=2)
    nreg = plan.info["nrings"] - (2 if sampling == "mwss" else 0)
    assert plan.info["swept_rings"] == (nreg + 1) // 2
    flm = flm_gaussian(L, 0, seed=21, batch=2, scale="inv1pl")
    f = host(plan.inverse(dev(flm)))
    for b in range(2):
        assert fp64_err(f[b].ravel(), oracle.s2_inverse(flm[b], L, 0, samp, nside).ravel()) < 1e-12
    fr = host(plan.inverse_real(dev(flm[0])))
    assert fp64_err(fr.ravel(), oracle.s2_inverse_real(flm[0], L, samp, nside).ravel()) < 1e-12
    # forward sweep over the northern rings (degree groups of one parity)
    gm = map_gaussian((2,) + tuple(plan.map_shape), seed=24)
    a = host(plan.forward(dev(gm)))
    for b in range(2):
        assert fp64_err(a[b], oracle.s2_forward(gm[b], L, 0, samp, nside)) < 1e-12
    assert np.all(a[:, ~coeff_mask(L, 0)] == 0)
    gr = np.random.default_rng(25).standard_normal(plan.map_shape)
    assert fp64_err(host(plan.forward_real(dev(gr))), oracle.s2_forward_real(gr, L, samp, nside)) < 1e-12
    # adjoints: the forward's (an inverse-type sweep) and the inverse's (a forward-type sweep)
    g = flm_gaussian(L, 0, seed=22)
    x = map_gaussian(plan.map_shape, seed=23)
    lhs = np.vdot(g, oracle.s2_forward(x, L, 0, samp, nside))
    rhs = np.vdot(host(plan.forward_adjoint(dev(g))), x)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    assert fp64_err(host(plan.inverse_adjoint(dev(x))), oracle.s2_inverse_adjoint(x, L, 0, samp, nside)) < 1e-12
    monkeypatch.setenv("S2MI_RING_PAIRING", "0")
    ref_plan = binding.Plan(L, sampling=sampling, nside=nside, max_batch=2)
    assert ref_plan.info["swept_rings"] == nreg
    assert fp64_err(f, host(ref_plan.inverse(dev(flm)))) < 1e-13
    assert fp64_err(a, host(ref_plan.forward(dev(gm)))) < 1e-13
