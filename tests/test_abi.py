"""The C ABI library loads and exports every symbol the headers declare; host-side
argument checks reject bad input before any device work (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("rad.h", "rad_debug.h")]


def declared_functions():
    names = []
    for h in HEADERS:
        src = open(h).read()
        names += re.findall(r"^\s*(?:int|size_t|const char\s*\*)\s+(rad_\w+)\s*\(", src, re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def librad():
    from paper_1802_03972_amd import _lib
    from paper_1802_03972_amd.build import ensure_built
    ensure_built()    # a built library is used as is
    return _lib.lib()


def test_headers_declare_core_calls():
    names = declared_functions()
    for core in ("rad_create_grid", "rad_push_step", "rad_spectrum", "rad_destroy_grid"):
        assert core in names


def test_every_declared_symbol_is_exported(librad):
    from paper_1802_03972_amd import _lib
    names = declared_functions()
    for n in names:
        assert hasattr(librad, n), f"{n} declared in include/ but not exported"
        assert n in _lib.SIGNATURES, f"{n} has no ctypes signature in the binding"


def test_binding_declares_only_header_symbols():
    from paper_1802_03972_amd import _lib
    assert set(_lib.SIGNATURES) == set(declared_functions())


def test_invalid_grid_arguments_rejected_on_host(librad):
    from paper_1802_03972_amd import _lib
    dirs = np.array([[0.0, 0.0, 1.0]])
    def desc(**kw):
        base = dict(n_dir=1, dirs=dirs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), omega0=0.0,
                    domega=1e15, n_omega=8, shape=1, shape_len=1e-7, dt=1e-16, precision=0, device=0)
        base.update(kw)
        return _lib.GridDesc(**base)
    h = ctypes.c_void_p()
    bad = [dict(n_dir=0), dict(n_omega=0), dict(domega=-1.0), dict(shape=9), dict(shape_len=0.0),
           dict(dt=0.0), dict(precision=7), dict(omega0=float("nan"))]
    for kw in bad:
        rc = librad.rad_create_grid(ctypes.byref(h), ctypes.byref(desc(**kw)))
        assert rc == _lib.RAD_ERR_INVALID_ARG, kw
        assert h.value is None
        assert librad.rad_last_error()
    nonunit = np.array([[0.0, 0.0, 1.1]])
    rc = librad.rad_create_grid(ctypes.byref(h), ctypes.byref(
        desc(dirs=nonunit.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))))
    assert rc == _lib.RAD_ERR_INVALID_ARG and b"unit" in librad.rad_last_error()


def test_null_handles_rejected(librad):
    from paper_1802_03972_amd import _lib
    assert librad.rad_destroy_grid(None) == _lib.RAD_OK
    assert librad.rad_reset(None, None) == _lib.RAD_ERR_INVALID_ARG
    assert librad.rad_push_step(None, 0.0, 1, None, None) == _lib.RAD_ERR_INVALID_ARG
    assert librad.rad_spectrum(None, None, None) == _lib.RAD_ERR_INVALID_ARG
    assert librad.rad_state_size(None) == 0
