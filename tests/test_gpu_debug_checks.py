"""The plan's debug check (environment S2MI_DEBUG_CHECKS=1): sum over |m| <= l of
(d^l_{m,n}(theta))^2 = 1 on sampled rings, for every degree and both runs n, -n,
with the values the transforms use.  Plans of every kind pass it; a tolerance set
from the host that nothing can meet makes plan creation fail with the check's error
code (the kernels run normally either way)."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def binding():
    from paper_2311_14670_amd import binding as b
    b.load_library()
    return b


@pytest.mark.parametrize("kw", [dict(L=256), dict(L=200, spin=3), dict(L=64, spin=-17), dict(L=40, spin=39),
                                dict(L=128, spin=2, sampling="healpix", nside=64), dict(L=130, sampling="dh"),
                                dict(L=97, spin=1, sampling="gl"), dict(L=120, spin=-2, sampling="mwss"),
                                dict(L=64, N=5), dict(L=2048), dict(L=1024, spin=2)],
                         ids=lambda kw: ",".join(f"{k}={v}" for k, v in kw.items()))
def test_plans_pass_the_unitarity_check(binding, monkeypatch, kw):
    monkeypatch.setenv("S2MI_DEBUG_CHECKS", "1")
    plan = binding.Plan(**kw)
    assert plan.info["L"] == kw["L"]


def test_unmeetable_tolerance_fails_the_plan(binding, monkeypatch):
    monkeypatch.setenv("S2MI_DEBUG_CHECKS", "1")
    monkeypatch.setenv("S2MI_DEBUG_CHECKS_TOL", "-1")
    with pytest.raises(binding.S2Error) as ei:
        binding.Plan(64, spin=2)
    assert ei.value.code == -5
    assert "debug check" in str(ei.value)
