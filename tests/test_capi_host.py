"""CPU-only checks of the native library: it loads, exports every symbol the
header declares, and validates arguments on the host before any device work."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "s2mi.h")


def _lib():
    from paper_2311_14670_amd import binding
    if not os.path.exists(binding.library_path()):
        from paper_2311_14670_amd import build
        build.build()
    return binding.load_library()


def header_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b((?:s2|so3)_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = _lib()
    syms = header_symbols()
    assert "s2_plan_create" in syms and "so3_forward" in syms and "s2_inverse_adjoint" in syms
    for s in syms:
        assert hasattr(lib, s), s


@pytest.mark.parametrize("kw,code", [
    (dict(L=1), -1), (dict(L=5000), -1), (dict(L=16, spin=16), -1), (dict(L=16, N=0), -1),
    (dict(L=16, N=9), -2), (dict(L=16, N=3, spin=2), -1), (dict(L=16, sampling=7), -1),
    (dict(L=16, sampling=1, nside=0), -1), (dict(L=16, sampling=1, nside=4, N=2), -2),
    (dict(L=16, sampling=2, N=2), -2), (dict(L=16, sampling=3, N=4), -2), (dict(L=16, sampling=4, N=2), -2),
    (dict(L=16, sampling=5), -1),
    (dict(L=16, max_batch=0), -1), (dict(L=16, precision=3), -1)])
def test_plan_create_validation(kw, code):
    from paper_2311_14670_amd import binding
    _lib()
    rc, h = binding.plan_create_raw(**kw)
    assert rc == code
    assert h.value is None
    assert binding.load_library().s2_last_error_message().decode() != ""


def test_transform_validation_without_plan():
    lib = _lib()
    vp = ctypes.c_void_p
    for fn in ["s2_inverse", "s2_forward", "s2_inverse_adjoint", "s2_forward_adjoint", "so3_inverse", "so3_forward",
               "so3_inverse_adjoint", "so3_forward_adjoint", "s2_inverse_real", "s2_forward_real",
               "s2_inverse_real_adjoint", "s2_forward_real_adjoint"]:
        rc = getattr(lib, fn)(None, vp(16), vp(16), 1, vp(256), None)
        assert rc == -1
    assert lib.s2_inverse_noalloc(None, vp(16), vp(16), 1, None) == -1
    assert lib.s2_plan_info(None, None) == -1
    assert lib.s2_plan_destroy(None) == 0
    assert lib.s2_error_string(-2).decode() == "unsupported"
    assert lib.s2_error_string(-5).decode() == "debug check failed"
