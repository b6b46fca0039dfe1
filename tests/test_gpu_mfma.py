"""Matrix-core contraction path (precision FP32 and split BF16): the Wigner-d
recursion, quadrature weights and phi-DFTs stay FP64; the per-order products
run on MFMA with fp32 accumulation.  Results are compared with the FP64 oracle
at tolerances derived from the arithmetic:

  FP32        operands rounded to fp32 (2^-24 relative) and fp32 sums over
              K <= L terms (~sqrt(K) 2^-24 in rms): rel-L2 <= 2e-5 at L <= 256.
  split BF16  |x - hi - lo| <= 2^-16 |x| per operand and the dropped lo*lo
              term <= 2^-16 of the product: <= 3 2^-16 per product, rel-L2
              <= 2e-4.

The same bounds hold at L = 2048: the fp32 accumulation error grows like
sqrt(K) 2^-24 ~ 3e-6 at K = 2048 terms, still below 2e-5, and split BF16 stays
dominated by its 3 2^-16 per-product term.  Each result also reports, and gates
at the same bound, the max relative coefficient error max|x - x_ref| / max|x_ref|.

At full size the path generates D in chunks of consecutive orders (one chunk of
D staged at a time, at most 512 MB) and carries the recursion state of every
(degree, ring) across chunks in the workspace; those tests check that the
generator really ran several chunks (its launch count per run)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2311_14670_amd.synth import flm_gaussian, flmn_gaussian, map_gaussian, coeff_mask

pytestmark = pytest.mark.gpu

TOL = {"fp32": 2e-5, "split_bf16": 2e-4}
PRECS = ["fp32", "split_bf16"]


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def max_rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


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


def _check(name, prec, got, ref):
    e, m = rel_l2(got, ref), max_rel(got, ref)
    print(f"{name} {prec}: rel_l2={e:.3e} max_rel={m:.3e}", flush=True)
    assert e < TOL[prec]
    assert m < TOL[prec]
    assert e > 1e-12          # the reduced-precision products were really used


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L,spin,B", [(64, 0, 5), (48, 2, 3), (41, -1, 2), (130, 0, 9), (40, 13, 2)])
def test_mw_batched(binding, prec, L, spin, B):
    flm = flm_gaussian(L, spin, seed=20, batch=B, scale="inv1pl")
    plan = binding.Plan(L, spin=spin, max_batch=B, precision=prec)
    f = host(plan.inverse(dev(flm)))
    for b in (0, B - 1):
        _check(f"mw inverse L={L} s={spin} b={b}", prec, f[b], oracle.s2_inverse(flm[b], L, spin))
    g = map_gaussian((B, L, 2 * L - 1), seed=21)
    a = host(plan.forward(dev(g)))
    for b in (0, B - 1):
        _check(f"mw forward L={L} s={spin} b={b}", prec, a[b], oracle.s2_forward(g[b], L, spin))
    assert np.all(a[:, ~coeff_mask(L, spin)] == 0)
    adj = host(plan.inverse_adjoint(dev(g)))
    _check(f"mw adjoint L={L} s={spin}", prec, adj[0], oracle.s2_inverse_adjoint(g[0], L, spin))


@pytest.mark.parametrize("prec", PRECS)
def test_healpix_batched(binding, prec):
    nside, L, spin, B = 16, 32, 2, 3
    flm = flm_gaussian(L, spin, seed=22, batch=B)
    plan = binding.Plan(L, spin=spin, sampling="healpix", nside=nside, max_batch=B, precision=prec)
    f = host(plan.inverse(dev(flm)))
    _check("healpix inverse", prec, f[1], oracle.s2_inverse(flm[1], L, spin, oracle.HEALPIX, nside))
    g = map_gaussian((B, 12 * nside * nside), seed=23)
    a = host(plan.forward(dev(g)))
    _check("healpix forward", prec, a[2], oracle.s2_forward(g[2], L, spin, oracle.HEALPIX, nside))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("sampling", ["dh", "gl", "mwss"])
def test_dh_gl_batched(binding, prec, sampling):
    L, spin, B = 40, 2, 3
    samp = {"dh": oracle.DH, "gl": oracle.GL, "mwss": oracle.MWSS}[sampling]
    flm = flm_gaussian(L, spin, seed=26, batch=B)
    plan = binding.Plan(L, spin=spin, sampling=sampling, max_batch=B, precision=prec)
    f = host(plan.inverse(dev(flm)))
    _check(f"{sampling} inverse", prec, f[1], oracle.s2_inverse(flm[1], L, spin, samp))
    g = map_gaussian((B,) + plan.map_shape, seed=27)
    a = host(plan.forward(dev(g)))
    _check(f"{sampling} forward", prec, a[2], oracle.s2_forward(g[2], L, spin, samp))


def _so3_inverse_adjoint_oracle(g, L, N):
    """Adjoint of the inverse Wigner transform from the oracle's spin-SHT adjoint:
    slice n of the inverse is the spin -n inverse SHT of (-1)^n sqrt((2l+1)/(16 pi^3))
    flmn (Sec. 2.3) spread over gamma by e^{i n gamma_k}, so its adjoint is the
    unweighted gamma analysis sum_k g_k e^{-i n gamma_k} followed by the spin -n
    adjoint, times the same factor."""
    gam = 2 * np.pi * np.arange(2 * N - 1) / (2 * N - 1)
    ell = np.arange(L)[:, None]
    out = np.zeros((2 * N - 1, L, 2 * L - 1), dtype=np.complex128)
    for n in range(-(N - 1), N):
        gn = np.tensordot(np.exp(-1j * n * gam), g, axes=(0, 0))
        out[n + N - 1] = ((-1.0) ** n * np.sqrt((2 * ell + 1) / (16 * np.pi ** 3))
                          * oracle.s2_inverse_adjoint(gn, L, -n))
    return out


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("N", [8, 1])
def test_so3_batched(binding, prec, N):
    """N = 1 runs on a sphere plan (one slice: the gamma rule is the weight 2 pi)."""
    L, B = 40, 2
    flmn = flmn_gaussian(L, N, seed=24, batch=B)
    plan = binding.Plan(L, N=N, max_batch=B, precision=prec)
    f = host(plan.so3_inverse(dev(flmn)))
    _check("so3 inverse", prec, f[1], oracle.so3_inverse(flmn[1], L, N))
    back = host(plan.so3_forward(dev(f)))
    _check("so3 round trip", prec, back[1], flmn[1])
    g = map_gaussian((B, 2 * N - 1, L, 2 * L - 1), seed=25)
    _check("so3 forward", prec, host(plan.so3_forward(dev(g)))[0], oracle.so3_forward(g[0], L, N))
    # adjoint of the inverse (gradient path) against the oracle
    adj = host(plan.so3_inverse_adjoint(dev(g)))
    _check("so3 inverse adjoint", prec, adj[1], _so3_inverse_adjoint_oracle(g[1], L, N))


@pytest.mark.parametrize("prec", PRECS)
def test_batch_composition_invariance(binding, prec):
    """A map's result does not depend on the other maps of its batch."""
    L, B = 40, 6
    flm = flm_gaussian(L, 0, seed=25, batch=B)
    big = binding.Plan(L, max_batch=B, precision=prec)
    one = binding.Plan(L, max_batch=1, precision=prec)
    fb = host(big.inverse(dev(flm)))
    for b in (0, 3, 5):
        f1 = host(one.inverse(dev(flm[b])))
        assert np.array_equal(fb[b], f1)
    ab = host(big.forward(dev(fb)))
    a1 = host(one.forward(dev(fb[4])))
    assert np.array_equal(ab[4], a1)


# ----------------------------------------------------------------- order chunks
def _dgen_launches(plan, fn, x):
    plan.set_timing(True)
    plan.read_timing()
    y = fn(x)
    t = plan.read_timing()
    plan.set_timing(False)
    return y, t.get("dgen", (0.0, 0))[1]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L,spin", [(130, 0), (97, 2), (70, -3)])
def test_order_chunks_do_not_change_results(binding, monkeypatch, prec, L, spin):
    """The generator run in chunks of 7 orders (state carried across chunks in the
    workspace) gives bit-identical products to the one-chunk run."""
    B = 5
    flm = flm_gaussian(L, spin, seed=28, batch=B, scale="inv1pl")
    g = map_gaussian((B, L, 2 * L - 1), seed=29)
    one = binding.Plan(L, spin=spin, max_batch=B, precision=prec)
    monkeypatch.setenv("S2MI_MFMA_ORDER_CHUNK", "7")
    chunked = binding.Plan(L, spin=spin, max_batch=B, precision=prec)
    monkeypatch.delenv("S2MI_MFMA_ORDER_CHUNK")
    f1, n1 = _dgen_launches(one, one.inverse, dev(flm))
    f7, n7 = _dgen_launches(chunked, chunked.inverse, dev(flm))
    runs = 1 if spin == 0 else 2
    assert n7 > n1 and n7 >= runs * (L // 7)
    assert np.array_equal(host(f1), host(f7))
    assert np.array_equal(host(one.forward(dev(g))), host(chunked.forward(dev(g))))
    assert np.array_equal(host(one.inverse_adjoint(dev(g))), host(chunked.inverse_adjoint(dev(g))))
    _check(f"chunked inverse L={L} s={spin}", prec, host(f7)[B - 1], oracle.s2_inverse(flm[B - 1], L, spin))


def _rings(L):
    rings = {64 * k + (23 * k + 5) % 64 for k in range((L + 63) // 64)}
    rings |= {0, 1, 63, 64, L // 2, L - 2, L - 1}
    return np.array(sorted(r for r in rings if 0 <= r < L))


def _orders(L):
    ms = {0, 1, -1, 2, 7, 8, -8, L - 2, L - 1, -(L - 1), L // 2, -(L // 3)}
    for j in range(64, L, max(64, (L // 8) // 64 * 64)):
        ms |= {j - 1, j, -(j + 7)}
    return np.array(sorted(m for m in ms if -L < m < L))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("L,spin", [(640, 0), (640, 2), (1024, 0), (1024, 2)])
def test_full_size_chunked(binding, monkeypatch, prec, L, spin):
    """Full sizes with the generator staging D in four order chunks per run (the
    state carried across them), against the oracle on sampled rings and orders of
    the first and last map."""
    B = 4
    flm = flm_gaussian(L, spin, seed=30, batch=B, scale="inv1pl")
    monkeypatch.setenv("S2MI_MFMA_ORDER_CHUNK", str(L // 4))
    plan = binding.Plan(L, spin=spin, max_batch=B, precision=prec)
    monkeypatch.delenv("S2MI_MFMA_ORDER_CHUNK")
    f, nchunk = _dgen_launches(plan, plan.inverse, dev(flm))
    runs = 1 if spin == 0 else 2
    assert nchunk >= 4 * runs, nchunk
    rings = _rings(L)
    ms = _orders(L)
    for b in (0, B - 1):
        fr = host(f[b])[rings]
        _check(f"inverse L={L} s={spin} b={b}", prec, fr, oracle.s2_inverse(flm[b], L, spin, rings=rings).reshape(fr.shape))
    g = map_gaussian((B, L, 2 * L - 1), seed=31)
    a = host(plan.forward(dev(g)))
    for b in (0, B - 1):
        ref = oracle.s2_forward(g[b], L, spin, ms=ms)
        _check(f"forward L={L} s={spin} b={b}", prec, a[b][:, ms + L - 1], ref[:, ms + L - 1])


@pytest.mark.parametrize("prec", PRECS)
def test_c3_batch64_L2048(binding, prec):
    """The batched precision workload at its own size: 64 spin-0 MW maps at
    L = 2048 (Gaussian coefficients x 1/(1+l), seed 2) through the inverse and the
    forward, maps 0 and 63 against the oracle on sampled rings and orders, and the
    round trip of every map."""
    L, B = 2048, 64
    print("c3: drawing 64 maps of coefficients", flush=True)
    flm = flm_gaussian(L, 0, seed=2, batch=B, scale="inv1pl")
    x = dev(flm)
    plan = binding.Plan(L, max_batch=B, precision=prec)
    print(f"c3 {prec}: inverse", flush=True)
    f = plan.inverse(x)
    print(f"c3 {prec}: forward", flush=True)
    back = plan.forward(f)
    torch.cuda.synchronize()
    rings, ms = _rings(L), _orders(L)
    for b in (0, B - 1):
        fb = host(f[b])
        _check(f"c3 inverse b={b}", prec, fb[rings], oracle.s2_inverse(flm[b], L, 0, rings=rings).reshape(rings.size, -1))
        ref = oracle.s2_forward(fb, L, 0, ms=ms)
        _check(f"c3 forward b={b}", prec, host(back[b])[:, ms + L - 1], ref[:, ms + L - 1])
    # round trip of all 64 maps, reduced on the device
    d = (back - x).abs().amax(dim=(1, 2)) / x.abs().amax(dim=(1, 2))
    rt = float(d.max())
    print(f"c3 {prec}: worst round-trip max_rel over 64 maps {rt:.3e}", flush=True)
    assert rt < TOL[prec]
    del f, back, x
    torch.cuda.empty_cache()
