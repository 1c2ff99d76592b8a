"""Host-side checks of the C ABI: the library loads, exports every symbol that
include/mg.h declares, and validates parameters without touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mg.h")
LIB = os.path.join(ROOT, "paper_2607_10983_amd", "libmg.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__ as g
        g.build()
    from paper_2607_10983_amd import _lib
    return _lib.load()


def test_header_declares_the_abi():
    syms = declared_symbols()
    for s in ["mg_create", "mg_destroy", "mg_vcycle", "mg_solve", "mg_solve_adjoint", "mg_coeff_grad",
              "mg_geometry", "mg_geometry_bwd", "mg_status_string", "mg_last_error"]:
        assert s in syms


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(mg_\w+)", out))
    missing = [s for s in declared_symbols() if s not in exported]
    assert not missing, missing
    for s in declared_symbols():
        assert hasattr(lib, s)


def test_binding_covers_the_abi():
    from paper_2607_10983_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared_symbols()


def _params(lib, n):
    from paper_2607_10983_amd._lib import MgParams
    p = MgParams()
    assert lib.mg_params_default(ctypes.byref(p), n) == 0
    return p


def test_default_params(lib):
    p = _params(lib, 256)
    assert (p.n, p.levels, p.cheb_degree) == (256, 7, 3)
    assert p.cheb_alpha == 8.0 and p.h == 1.0 / 256
    assert p.jacobi_omega == pytest.approx(2 / 3) and p.jacobi_sweeps == 2
    assert lib.mg_validate_params(ctypes.byref(p)) == 0


@pytest.mark.parametrize("field,value", [
    ("n", 48), ("n", 4), ("n", 4096), ("levels", 0), ("levels", 8), ("cheb_degree", 0),
    ("cheb_degree", 9), ("cheb_alpha", 1.0), ("h", 0.0), ("h", -1.0), ("precision", 3), ("smoother", 2),
])
def test_invalid_params_rejected_on_host(lib, field, value):
    p = _params(lib, 256)
    setattr(p, field, value)
    assert lib.mg_validate_params(ctypes.byref(p)) == 1
    # mg_create validates before touching any device
    h = ctypes.c_void_p()
    assert lib.mg_create(ctypes.byref(p), None, 1, None, ctypes.byref(h)) == 1
    assert not h.value


def test_levels_and_coarsest_size(lib):
    p = _params(lib, 1024)
    p.levels = 7          # coarsest 16^3 (seven-point)
    assert lib.mg_validate_params(ctypes.byref(p)) == 0
    p.levels = 6          # coarsest 32^3 is too large for the exact coarsest solve
    assert lib.mg_validate_params(ctypes.byref(p)) == 1
    p = _params(lib, 8)
    assert p.levels == 2
    assert lib.mg_validate_params(ctypes.byref(p)) == 0


def test_status_strings(lib):
    for s in range(7):
        assert lib.mg_status_string(s).decode().startswith("MG_")
    assert b"unknown" in lib.mg_status_string(99)
    assert lib.mg_last_error(None) == b""
    assert lib.mg_destroy(None) == 0
