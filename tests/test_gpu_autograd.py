"""Gradients of the inverse SHT through torch.autograd (Sec. 5).

loss = sum |inverse(flm) - target|^2 over all MW samples (south-pole ring
included).  Checked against central finite differences at L = 32 (the loss is
quadratic, so h = 1 gives the exact directional derivative up to rounding) and
against the oracle's gradient 2 A^H (A flm - target) at L = 512, batch 16.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2311_14670_amd.synth import flm_gaussian, map_gaussian, coeff_mask

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


@pytest.fixture(scope="module")
def ag():
    from paper_2311_14670_amd import autograd, binding
    binding.load_library()
    return autograd, binding


@pytest.mark.parametrize("spin", [0, 2])
def test_gradient_matches_finite_differences(ag, spin):
    autograd, binding = ag
    L, chunk = 32, 252
    flm = flm_gaussian(L, spin, seed=4)
    target = torch.from_numpy(map_gaussian((L, 2 * L - 1), seed=5)).cuda()
    plan = binding.Plan(L, spin=spin, max_batch=chunk)

    x = torch.from_numpy(flm).cuda().requires_grad_(True)
    loss = torch.view_as_real(autograd.inverse(x, plan) - target).pow(2).sum()
    loss.backward()
    grad = x.grad.cpu().numpy()

    # central differences over every real coordinate, batched through the plan
    base = torch.from_numpy(flm).cuda()
    n = L * (2 * L - 1)
    fd = np.zeros(2 * n)
    coords = np.arange(2 * n)
    for c0 in range(0, 2 * n, chunk // 2):
        cs = coords[c0:c0 + chunk // 2]
        pert = base.unsqueeze(0).repeat(2 * cs.size, 1, 1)
        flat = torch.view_as_real(pert).reshape(2 * cs.size, -1)
        idx = torch.from_numpy(cs).cuda()
        rows = torch.arange(cs.size, device="cuda")
        flat[rows, idx] += 1.0
        flat[rows + cs.size, idx] -= 1.0
        f = plan.inverse(pert)
        lv = torch.view_as_real(f - target).pow(2).sum(dim=(1, 2, 3)).cpu().numpy()
        fd[c0:c0 + cs.size] = (lv[:cs.size] - lv[cs.size:]) / 2.0
    fd_c = fd[0::2] + 1j * fd[1::2]
    fd_c = fd_c.reshape(L, 2 * L - 1)
    assert rel_l2(grad, fd_c) < 1e-9
    # coefficients the transform ignores have exactly zero gradient
    assert np.all(grad[~coeff_mask(L, spin)] == 0)


@pytest.mark.parametrize("spin", [0, 2])
def test_gradient_matches_oracle_at_L512(ag, spin):
    autograd, binding = ag
    L, B = 512, 16
    rng_seed = 4
    flm = flm_gaussian(L, spin, seed=rng_seed, batch=B)
    target = map_gaussian((B, L, 2 * L - 1), seed=rng_seed + 1)
    plan = binding.Plan(L, spin=spin, max_batch=B)
    x = torch.from_numpy(flm).cuda().requires_grad_(True)
    t = torch.from_numpy(target).cuda()
    loss = torch.view_as_real(autograd.inverse(x, plan) - t).pow(2).sum()
    loss.backward()
    grad = x.grad.cpu().numpy()
    for b in (0, B - 1):
        resid = oracle.s2_inverse(flm[b], L, spin) - target[b]
        ref = 2.0 * oracle.s2_inverse_adjoint(resid, L, spin)
        assert rel_l2(grad[b], ref) < 1e-11
    # every map of the batch gets the gradient it would get alone
    plan1 = binding.Plan(L, spin=spin)
    for b in (3, 9):
        xb = torch.from_numpy(flm[b]).cuda().requires_grad_(True)
        lb = torch.view_as_real(autograd.inverse(xb, plan1) - t[b]).pow(2).sum()
        lb.backward()
        assert rel_l2(grad[b], xb.grad.cpu().numpy()) < 1e-14


@pytest.mark.parametrize("sampling,L,nside,spin", [("mw", 24, 0, 0), ("mw", 20, 0, 2), ("mw", 17, 0, -3),
                                                   ("healpix", 16, 8, 0), ("healpix", 12, 8, 1), ("dh", 14, 0, 2),
                                                   ("gl", 15, 0, -1)])
def test_forward_adjoint_dot_product(ag, sampling, L, nside, spin):
    """<F f, G> = <f, F^H G> with F the oracle's forward transform."""
    autograd, binding = ag
    plan = binding.Plan(L, spin=spin, sampling=sampling, nside=nside)
    f = map_gaussian(plan.map_shape, seed=30)
    G = flm_gaussian(L, spin, seed=31)
    samp = {"mw": oracle.MW, "healpix": oracle.HEALPIX, "dh": oracle.DH, "gl": oracle.GL}[sampling]
    lhs = np.vdot(G, oracle.s2_forward(f, L, spin, samp, nside))           # <G, F f>
    FhG = plan.forward_adjoint(torch.from_numpy(G).cuda()).cpu().numpy()
    rhs = np.vdot(FhG, f)                                                   # <F^H G, f>
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("spin", [0, 2])
def test_forward_gradient_matches_finite_differences(ag, spin):
    """loss = sum |forward(f) - target|^2 over the coefficients, L = 16 MW."""
    autograd, binding = ag
    L = 16
    nmap = L * (2 * L - 1)
    chunk = 2 * 124
    f0 = map_gaussian((L, 2 * L - 1), seed=32)
    target = torch.from_numpy(flm_gaussian(L, spin, seed=33)).cuda()
    plan = binding.Plan(L, spin=spin, max_batch=chunk)
    x = torch.from_numpy(f0).cuda().requires_grad_(True)
    loss = torch.view_as_real(autograd.forward(x, plan) - target).pow(2).sum()
    loss.backward()
    grad = x.grad.cpu().numpy()
    base = torch.from_numpy(f0).cuda()
    fd = np.zeros(2 * nmap)
    for c0 in range(0, 2 * nmap, chunk // 2):
        cs = np.arange(c0, min(c0 + chunk // 2, 2 * nmap))
        pert = base.unsqueeze(0).repeat(2 * cs.size, 1, 1)
        flat = torch.view_as_real(pert).reshape(2 * cs.size, -1)
        idx = torch.from_numpy(cs).cuda()
        rows = torch.arange(cs.size, device="cuda")
        flat[rows, idx] += 1.0
        flat[rows + cs.size, idx] -= 1.0
        lv = torch.view_as_real(plan.forward(pert) - target).pow(2).sum(dim=(1, 2, 3)).cpu().numpy()
        fd[c0:c0 + cs.size] = (lv[:cs.size] - lv[cs.size:]) / 2.0
    fd_c = (fd[0::2] + 1j * fd[1::2]).reshape(L, 2 * L - 1)
    assert rel_l2(grad, fd_c) < 1e-9
