"""Host-side argument checks of the C ABI, exercised without a GPU: every descriptor and
argument error is reported with RAD_ERR_INVALID_ARG and a message before any HIP call, and
a valid request on a machine without a GPU fails loudly (no CPU fallback exists)."""
import ctypes

import numpy as np
import pytest

from paper_1802_03972_amd import _lib

DP = ctypes.POINTER(ctypes.c_double)


@pytest.fixture(scope="module")
def L():
    return _lib.lib()


def desc(dirs, **kw):
    d = dict(n_dir=len(dirs), dirs=dirs.ctypes.data_as(DP), omega0=0.0, domega=1e16, n_omega=8, shape=1,
             shape_len=1e-7, dt=5e-17, precision=0, device=0, omegas=None)
    d.update(kw)
    return _lib.GridDesc(*[d[k] for k, _ in _lib.GridDesc._fields_])


ONE = np.array([[0.0, 0.0, 1.0]])


@pytest.mark.parametrize("kw,msg", [
    (dict(n_dir=0), "n_dir"),
    (dict(n_omega=0), "n_omega"),
    (dict(shape=42), "unknown shape"),
    (dict(shape=1, shape_len=0.0), "shape_len"),
    (dict(dt=-1.0), "dt must be"),
    (dict(dt=float("nan")), "dt must be"),
    (dict(precision=7), "precision"),
    (dict(domega=-1.0), "domega"),
    (dict(omega0=float("inf")), "omega0"),
    (dict(n_dir=1 << 20, n_omega=1 << 10), "too large"),
])
def test_grid_descriptor_errors(L, kw, msg):
    dirs = ONE if "n_dir" not in kw or kw["n_dir"] <= 1 else np.tile(ONE, (kw["n_dir"], 1))
    h = ctypes.c_void_p()
    rc = L.rad_create_grid(ctypes.byref(h), ctypes.byref(desc(dirs, **kw)))
    assert rc == _lib.RAD_ERR_INVALID_ARG
    assert msg in L.rad_last_error().decode()
    assert not h.value                      # output untouched on error


def test_non_unit_direction_and_bad_frequency_list(L):
    h = ctypes.c_void_p()
    two = np.array([[0.0, 0.0, 2.0]])
    assert L.rad_create_grid(ctypes.byref(h), ctypes.byref(desc(two))) == _lib.RAD_ERR_INVALID_ARG
    assert "unit vector" in L.rad_last_error().decode()
    om = np.array([1e15, -1.0, 3e15])
    d = desc(ONE, n_omega=3, omegas=om.ctypes.data_as(DP))
    assert L.rad_create_grid(ctypes.byref(h), ctypes.byref(d)) == _lib.RAD_ERR_INVALID_ARG
    assert "omegas[1]" in L.rad_last_error().decode()


def test_null_handles_and_arguments(L):
    assert L.rad_create_grid(None, None) == _lib.RAD_ERR_INVALID_ARG
    assert L.rad_push_step(None, 0.0, 1, None, None) == _lib.RAD_ERR_INVALID_ARG
    assert L.rad_spectrum(None, None, None) == _lib.RAD_ERR_INVALID_ARG
    assert L.rad_destroy_grid(None) == _lib.RAD_OK
    cfg = _lib.ServerConfig(0, 1024, 8, 2, 16, 64, 20, 0)         # budget below 1 MiB
    h = ctypes.c_void_p()
    assert L.rad_server_create(ctypes.byref(h), ctypes.byref(cfg)) == _lib.RAD_ERR_INVALID_ARG
    assert L.rad_batcher_create(ctypes.byref(h), 0, 0) == _lib.RAD_ERR_INVALID_ARG
    d = desc(ONE)
    assert L.rad_tracked_create(ctypes.byref(h), ctypes.byref(d), 0) == _lib.RAD_ERR_INVALID_ARG
    d.precision = 1
    assert L.rad_tracked_create(ctypes.byref(h), ctypes.byref(d), 10) == _lib.RAD_ERR_INVALID_ARG


def test_valid_request_without_a_gpu_fails_loudly(L):
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = L.rad_create_grid(ctypes.byref(h), ctypes.byref(desc(ONE)))
    assert rc == _lib.RAD_ERR_DEVICE and not h.value
    assert L.rad_last_error().decode()


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus N > 1 (or a multi-rank launch) exits with status 2
    and says why, before touching the device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, WORLD_SIZE="1")
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, env=env, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""
    env["WORLD_SIZE"] = "4"
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py")], capture_output=True, text=True, env=env,
                       timeout=120)
    assert r.returncode == 2 and "WORLD_SIZE 4" in r.stderr
