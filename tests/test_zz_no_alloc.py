"""s2_inverse_noalloc: the inverse SHT on the library's fixed per-device scratch
instead of a caller workspace.  Its output must equal s2_inverse's (the same
kernels run on the same inputs) on two calls in a row, the second with a
smaller input, and plans whose inverse does not fit the scratch are refused."""
import numpy as np
import pytest
import torch

import oracle
from paper_2311_14670_amd.synth import flm_gaussian

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def binding():
    from paper_2311_14670_amd import binding as b
    b.load_library()
    return b


def _both(binding, L, spin, batch, sampling="mw", nside=0, seed=0):
    flm = flm_gaussian(L, spin, seed=seed, batch=batch)
    plan = binding.Plan(L, spin=spin, sampling=sampling, nside=nside, max_batch=batch)
    x = torch.from_numpy(flm).to("cuda")
    ref = plan.inverse(x)
    got = plan.inverse_noalloc(x)
    torch.cuda.synchronize()
    return flm, ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_equals_workspace_inverse_two_calls(binding):
    print("noalloc: call 1, MW L=200 spin 2 batch 3", flush=True)
    flm, ref, got = _both(binding, 200, 2, 3, seed=40)
    assert np.array_equal(got, ref)
    e = np.linalg.norm(got[2] - oracle.s2_inverse(flm[2], 200, 2)) / np.linalg.norm(got[2])
    assert e < 1e-13, e
    print("noalloc: call 2, MW L=33 spin 0 batch 1 (smaller)", flush=True)
    flm, ref, got = _both(binding, 33, 0, 1, seed=41)
    assert np.array_equal(got, ref)
    e = np.linalg.norm(got[0] - oracle.s2_inverse(flm[0], 33, 0)) / np.linalg.norm(got[0])
    assert e < 1e-13, e


def test_noalloc_other_samplings_and_largest_mw(binding):
    for L, spin, samp, nside in [(64, 0, "healpix", 32), (48, -3, "dh", 0), (40, 1, "mwss", 0), (512, 2, "mw", 0)]:
        print(f"noalloc: {samp} L={L} spin {spin}", flush=True)
        _, ref, got = _both(binding, L, spin, 2, samp, nside, seed=42)
        assert np.array_equal(got, ref), (samp, L)


def test_noalloc_refuses_plans_beyond_the_scratch(binding):
    big = binding.Plan(1024)
    x = torch.zeros((1024, 2047), dtype=torch.complex128, device="cuda")
    with pytest.raises(binding.S2Error, match="bytes of scratch"):
        big.inverse_noalloc(x)
    mixed = binding.Plan(32, precision="fp32")
    with pytest.raises(binding.S2Error) as e:
        mixed.inverse_noalloc(torch.zeros((32, 63), dtype=torch.complex128, device="cuda"))
    assert e.value.code == -2
