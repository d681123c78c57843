"""The C-ABI library loads and exports every symbol include/pse.h declares;
parameter validation (host logic, no GPU call) rejects what the error model
forbids."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pse.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pse_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_api():
    names = _declared()
    for must in ["pse_create", "pse_destroy", "pse_set_positions", "pse_sample", "pse_sample_with_noise",
                 "pse_real_matvec", "pse_real_sample", "pse_wave_sample", "pse_wave_apply", "pse_status_string"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1611_09322_amd as pse

    lib = pse.load()
    for name in _declared():
        assert hasattr(lib, name), name
    # and the binding mirrors the same names
    for name in _declared():
        assert hasattr(pse, name), name
    assert set(pse.EXPORTED) == set(_declared())


def _params(**kw):
    import paper_1611_09322_amd as pse

    base = dict(n=10, box=20.0, a=1.0, eta=1.0, kT=1.0, xi=0.5, rcut=8.0, grid=32, support=8, gauss_m=0.0,
                lanczos_tol=1e-4, lanczos_max_iter=32, precision=1, precond=0, flags=0, tol=0.0)
    base.update(kw)
    return pse.Params(*[base[f] for f, _ in pse.Params._fields_])


@pytest.mark.parametrize("bad,code", [
    (dict(rcut=10.0), -4),          # rcut must be < L/2 (minimum image)
    (dict(grid=40), -4),            # unsupported FFT size (5 x 2^3)
    (dict(support=7), -4),          # odd support
    (dict(grid=16, support=8, xi=2.0), -4),  # eta_SE = 4 xi^2 sigma^2 >= 1
    (dict(lanczos_max_iter=100), -4),
    (dict(tol=1e-6), -4),           # aliasing of the 32^3 grid (h = 0.63a) is above 1e-6
    (dict(tol=-1.0), -1),
    (dict(n=0), -1),
    (dict(box=-1.0), -1),
])
def test_parameter_validation_rejects(bad, code):
    import paper_1611_09322_amd as pse

    lib = pse.load()
    p = _params(**bad)
    ctx = ctypes.c_void_p()
    assert lib.pse_create(ctypes.byref(p), None, ctypes.byref(ctx)) == code
    assert not ctx.value


def test_null_arguments():
    import paper_1611_09322_amd as pse

    lib = pse.load()
    ctx = ctypes.c_void_p()
    assert lib.pse_create(None, None, ctypes.byref(ctx)) == -1
    assert lib.pse_set_positions(None, None) == -1
    assert lib.pse_sample(None, 0, 0, 1.0, None, None, None) == -1
    assert lib.pse_destroy(None) == 0
    assert lib.pse_status_string(-6).decode().startswith("Lanczos")
