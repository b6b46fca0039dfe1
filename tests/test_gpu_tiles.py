"""Order tiles of the FP64 sweeps.  A plan may run the orders of each recursion run
in tiles (separate slices of the sweep's grid), each tile below the top starting
from the recursion state stored at plan creation.  That state equals the one the
uninterrupted sweep holds up to exact powers of two, so tiled and untiled sweeps
must agree bit for bit; both must match the oracle."""
import numpy as np
import pytest
import torch

import oracle
from conftest import fp64_err
from paper_2311_14670_amd.synth import flm_gaussian, flmn_gaussian, map_gaussian

pytestmark = pytest.mark.gpu

_SAMP = {"mw": oracle.MW, "healpix": oracle.HEALPIX, "dh": oracle.DH, "gl": oracle.GL, "mwss": oracle.MWSS}


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


def _plans(binding, monkeypatch, tiles, **kw):
    monkeypatch.setenv("S2MI_ORDER_TILES", "1")
    ref = binding.Plan(**kw)
    monkeypatch.setenv("S2MI_ORDER_TILES", str(tiles))
    plan = binding.Plan(**kw)
    monkeypatch.delenv("S2MI_ORDER_TILES")
    assert ref.info["order_tiles"] == 1
    return ref, plan


# spin 0 and high spins (continuation below m = 0 for n != 0), the mirror-ring
# sweeps of the symmetric grids (cuts at whole 128-degree groups), ragged L
CASES = [("mw", 256, 0, 0), ("mw", 200, 2, 0), ("mw", 161, -5, 0), ("healpix", 256, 0, 128),
         ("dh", 200, 0, 0), ("mwss", 192, 1, 0), ("gl", 300, 0, 0), ("healpix", 130, 3, 64)]


@pytest.mark.parametrize("tiles", [3, 8])
@pytest.mark.parametrize("sampling,L,spin,nside", CASES)
def test_tiles_match_untiled_and_oracle(binding, monkeypatch, sampling, L, spin, nside, tiles):
    ref, plan = _plans(binding, monkeypatch, tiles, L=L, spin=spin, sampling=sampling, nside=nside)
    nt = plan.info["order_tiles"]
    assert 1 < nt <= tiles
    samp = _SAMP[sampling]
    flm = flm_gaussian(L, spin, seed=31, scale="inv1pl")
    f = host(plan.inverse(dev(flm)))
    assert np.array_equal(f, host(ref.inverse(dev(flm))))
    assert fp64_err(f, oracle.s2_inverse(flm, L, spin, samp, nside)) < 1e-12
    g = map_gaussian(plan.map_shape, seed=32)
    a = host(plan.forward(dev(g)))
    assert np.array_equal(a, host(ref.forward(dev(g))))
    assert fp64_err(a, oracle.s2_forward(g, L, spin, samp, nside)) < 1e-12
    # adjoints: the inverse's is a forward-type sweep, the forward's an inverse-type one
    adj = host(plan.inverse_adjoint(dev(g)))
    assert np.array_equal(adj, host(ref.inverse_adjoint(dev(g))))
    assert fp64_err(adj, oracle.s2_inverse_adjoint(g, L, spin, samp, nside)) < 1e-12
    fa = host(plan.forward_adjoint(dev(flm)))
    assert np.array_equal(fa, host(ref.forward_adjoint(dev(flm))))
    if spin == 0:
        fr = host(plan.inverse_real(dev(flm)))
        assert np.array_equal(fr, host(ref.inverse_real(dev(flm))))
        assert fp64_err(fr.ravel(), oracle.s2_inverse_real(flm, L, samp, nside).ravel()) < 1e-12
        gr = np.random.default_rng(33).standard_normal(plan.map_shape)
        ar = host(plan.forward_real(dev(gr)))
        assert np.array_equal(ar, host(ref.forward_real(dev(gr))))
        assert fp64_err(ar, oracle.s2_forward_real(gr, L, samp, nside)) < 1e-12


@pytest.mark.parametrize("L,N", [(130, 3), (192, 5)])
def test_tiles_so3(binding, monkeypatch, L, N):
    ref, plan = _plans(binding, monkeypatch, 4, L=L, N=N)
    assert plan.info["order_tiles"] > 1
    flmn = flmn_gaussian(L, N, seed=34)
    f = host(plan.so3_inverse(dev(flmn)))
    assert np.array_equal(f, host(ref.so3_inverse(dev(flmn))))
    assert fp64_err(f, oracle.so3_inverse(flmn, L, N)) < 1e-12
    g = map_gaussian((2 * N - 1, L, 2 * L - 1), seed=35)
    a = host(plan.so3_forward(dev(g)))
    assert np.array_equal(a, host(ref.so3_forward(dev(g))))
    assert fp64_err(a, oracle.so3_forward(g, L, N)) < 1e-12


def test_tiles_batched_and_noalloc(binding, monkeypatch):
    """A tiled plan over a batch (each map's runs share the state tables) and through
    the entry point that allocates nothing."""
    L, spin = 240, 2
    ref, plan = _plans(binding, monkeypatch, 5, L=L, spin=spin, max_batch=3)
    flm = flm_gaussian(L, spin, seed=36, batch=3)
    f = host(plan.inverse(dev(flm)))
    assert np.array_equal(f, host(ref.inverse(dev(flm))))
    assert np.array_equal(f, host(plan.inverse_noalloc(dev(flm))))
    for b in range(3):
        assert fp64_err(f[b], oracle.s2_inverse(flm[b], L, spin)) < 1e-12


@pytest.mark.parametrize("L,spin", [(1024, 0), (1024, 2), (512, 0)])
def test_default_tiling_at_size(binding, L, spin):
    """The plans the library tiles by itself (grids under two waves per SIMD) at the
    sizes where it matters: sampled rings and orders against the oracle, and the
    round trip."""
    plan = binding.Plan(L, spin=spin)
    assert plan.info["order_tiles"] > 1
    flm = flm_gaussian(L, spin, seed=37, scale="inv1pl")
    x = dev(flm)
    f = plan.inverse(x)
    rings = np.array(sorted({0, 1, 63, 64, 127, 200, L // 2, L - 2, L - 1} | set(range(5, L, 97))))
    assert fp64_err(host(f)[rings].ravel(), oracle.s2_inverse(flm, L, spin, rings=rings)) < 1e-11
    assert fp64_err(host(plan.forward(f)), flm) < 1e-11
    g = map_gaussian((L, 2 * L - 1), seed=38)
    a = host(plan.forward(dev(g)))
    ms = np.array(sorted({0, 1, -1, 63, 64, 127, 128, -129, 320, -321, 511, 512, L - 1, -(L - 1)}
                         & set(range(-(L - 1), L))))
    cols = ms + L - 1
    assert fp64_err(a[:, cols], oracle.s2_forward(g, L, spin, ms=ms)[:, cols]) < 1e-11


@pytest.mark.parametrize("sampling,L,nside", [("gl", 300, 0), ("healpix", 384, 192), ("mwss", 260, 0)])
def test_tiles_mirror_ring_sweeps(binding, monkeypatch, sampling, L, nside):
    """The mirror-ring sweeps (spin 0, N/S-symmetric grids: northern rings only,
    forward l-groups of one parity) under tiles."""
    monkeypatch.setenv("S2MI_RING_PAIRING", "1")
    ref, plan = _plans(binding, monkeypatch, 8, L=L, sampling=sampling, nside=nside)
    assert plan.info["order_tiles"] > 1
    assert plan.info["swept_rings"] < plan.info["nrings"]
    samp = _SAMP[sampling]
    flm = flm_gaussian(L, 0, seed=39, scale="inv1pl")
    f = host(plan.inverse(dev(flm)))
    assert np.array_equal(f, host(ref.inverse(dev(flm))))
    assert fp64_err(f, oracle.s2_inverse(flm, L, 0, samp, nside)) < 1e-12
    g = map_gaussian(plan.map_shape, seed=40)
    a = host(plan.forward(dev(g)))
    assert np.array_equal(a, host(ref.forward(dev(g))))
    assert fp64_err(a, oracle.s2_forward(g, L, 0, samp, nside)) < 1e-12
    gr = np.random.default_rng(41).standard_normal(plan.map_shape)
    ar = host(plan.forward_real(dev(gr)))
    assert np.array_equal(ar, host(ref.forward_real(dev(gr))))
