"""Matrix-core contraction path (precision FP32 and split BF16): the Wigner-d
recursion, quadrature weights and phi-DFTs stay FP64; the per-order products
run on MFMA with fp32 accumulation.  Results are compared with the FP64 oracle
at tolerances derived from the arithmetic:

  FP32        operands rounded to fp32 (2^-24 relative) and fp32 sums over
              K <= L terms (~sqrt(K) 2^-24 in rms): rel-L2 <= 2e-5 at L <= 256.
  split BF16  |x - hi - lo| <= 2^-16 |x| per operand and the dropped lo*lo
              term <= 2^-16 of the product: <= 3 2^-16 per product, rel-L2
              <= 2e-4.

Each result also reports the max relative coefficient error
max|x - x_ref| / max|x_ref|."""
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


@pytest.mark.parametrize("prec", PRECS)
def test_so3_batched(binding, prec):
    L, N, B = 40, 8, 2
    flmn = flmn_gaussian(L, N, seed=24, batch=B)
    plan = binding.Plan(L, N=N, max_batch=B, precision=prec)
    f = host(plan.so3_inverse(dev(flmn)))
    _check("so3 inverse", prec, f[1], oracle.so3_inverse(flmn[1], L, N))
    back = host(plan.so3_forward(dev(f)))
    _check("so3 round trip", prec, back[1], flmn[1])
    # adjoint of the inverse (gradient path) against the FP64 plan's
    g = map_gaussian((B, 2 * N - 1, L, 2 * L - 1), seed=25)
    adj = host(plan.so3_inverse_adjoint(dev(g)))
    ref = host(binding.Plan(L, N=N, max_batch=B).so3_inverse_adjoint(dev(g)))
    _check("so3 inverse adjoint", prec, adj[1], ref[1])


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
