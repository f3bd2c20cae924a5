"""ctypes declarations of librad.so (the C ABI in include/rad.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librad.so")

RAD_OK = 0
RAD_ERR_INVALID_ARG = -1
RAD_ERR_OOM = -2
RAD_ERR_DEVICE = -3
RAD_ERR_BAD_DATA = -4
RAD_ERR_QUEUE_FULL = -5

SHAPES = {"point": 0, "cic": 1, "tsc": 2, "qsc": 3, "gauss": 4, "cic3d": 5, "tsc3d": 6, "qsc3d": 7}
PHASE_F64 = 0
ALL_F32 = 1
F32 = 0
F64 = 1


class RadError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"rad error {code}: {msg}")
        self.code = code


class GridDesc(ctypes.Structure):
    _fields_ = [("n_dir", ctypes.c_int32), ("dirs", ctypes.POINTER(ctypes.c_double)),
                ("omega0", ctypes.c_double), ("domega", ctypes.c_double),
                ("n_omega", ctypes.c_int32), ("shape", ctypes.c_int32),
                ("shape_len", ctypes.c_double), ("dt", ctypes.c_double),
                ("precision", ctypes.c_int32), ("device", ctypes.c_int32),
                ("omegas", ctypes.POINTER(ctypes.c_double))]


class Particles(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32)] + [(k, ctypes.c_void_p) for k in
                                              ("x", "y", "z", "bx", "by", "bz", "dbx", "dby", "dbz", "w")]


class Tile(ctypes.Structure):
    _fields_ = [("w_per_lane", ctypes.c_int32), ("dir_per_wave", ctypes.c_int32),
                ("waves", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32)]


class ProfileStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("updates", ctypes.c_int64),
                ("accumulate_ms", ctypes.c_double), ("fold_ms", ctypes.c_double)]


class BatchItem(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_void_p), ("t0", ctypes.c_double), ("n_steps", ctypes.c_int32),
                ("n_particles", ctypes.c_int64), ("p", Particles)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("hbm_budget", ctypes.c_size_t), ("max_batch", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("max_admitted", ctypes.c_int32),
                ("max_pending", ctypes.c_int64), ("poll_us", ctypes.c_int32), ("use_graph", ctypes.c_int32)]


class ChunkStats(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_launch", ctypes.c_double),
                ("t_complete", ctypes.c_double), ("batch_size", ctypes.c_int32), ("status", ctypes.c_int32),
                ("batch_id", ctypes.c_int64)]


class ServerCounters(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("chunks_launched", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("completed", ctypes.c_int64), ("pending", ctypes.c_int64),
                ("admitted_waiting", ctypes.c_int64), ("inflight_batches", ctypes.c_int64),
                ("pool_used", ctypes.c_size_t), ("now", ctypes.c_double)]


# name -> (restype, argtypes); every symbol of include/rad.h and include/rad_debug.h
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "rad_create_grid": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(GridDesc)]),
    "rad_destroy_grid": (ctypes.c_int, [_vp]),
    "rad_reset": (ctypes.c_int, [_vp, _vp]),
    "rad_push_step": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_int64, ctypes.POINTER(Particles), _vp]),
    "rad_push_steps": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_int32, ctypes.c_int64,
                                      ctypes.POINTER(Particles), _vp]),
    "rad_push_step_noalloc": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_int64, ctypes.POINTER(Particles), _vp]),
    "rad_spectrum": (ctypes.c_int, [_vp, _dp, _vp]),
    "rad_spectrum_device": (ctypes.c_int, [_vp, _vp, _vp]),
    "rad_spectrum_complex": (ctypes.c_int, [_vp, _dp, _vp]),
    "rad_state_size": (ctypes.c_size_t, [_vp]),
    "rad_get_state": (ctypes.c_int, [_vp, _dp, _vp]),
    "rad_set_state": (ctypes.c_int, [_vp, _dp, _vp]),
    "rad_last_error": (ctypes.c_char_p, []),
    "rad_grid_variant": (ctypes.c_int, [_vp]),
    "rad_get_tile": (ctypes.c_int, [_vp, ctypes.POINTER(Tile)]),
    "rad_set_tile": (ctypes.c_int, [_vp, ctypes.POINTER(Tile)]),
    "rad_device_cus": (ctypes.c_int, [ctypes.c_int32]),
    "rad_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "rad_profile_read": (ctypes.c_int, [_vp, ctypes.POINTER(ProfileStats)]),
    "rad_batcher_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int32, ctypes.c_int32]),
    "rad_batcher_destroy": (ctypes.c_int, [_vp]),
    "rad_batcher_push": (ctypes.c_int, [_vp, ctypes.POINTER(BatchItem), ctypes.c_int32, _vp]),
    "rad_batcher_set_graph": (ctypes.c_int, [_vp, ctypes.c_int]),
    "rad_batcher_set_tile": (ctypes.c_int, [_vp, ctypes.POINTER(Tile)]),
    "rad_batcher_get_tile": (ctypes.c_int, [_vp, ctypes.POINTER(Tile)]),
    "rad_batcher_graph_stats": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                               ctypes.POINTER(ctypes.c_int64)]),
    "rad_batcher_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "rad_batcher_profile_read": (ctypes.c_int, [_vp, ctypes.POINTER(ProfileStats)]),
    "rad_server_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(ServerConfig)]),
    "rad_server_submit": (ctypes.c_int, [_vp, _vp, ctypes.c_double, ctypes.c_int64, ctypes.POINTER(Particles),
                                         ctypes.POINTER(ctypes.c_uint64)]),
    "rad_server_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(ChunkStats)]),
    "rad_server_wait": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(ChunkStats)]),
    "rad_server_drain": (ctypes.c_int, [_vp]),
    "rad_server_counters_read": (ctypes.c_int, [_vp, ctypes.POINTER(ServerCounters)]),
    "rad_server_set_tile": (ctypes.c_int, [_vp, ctypes.POINTER(Tile)]),
    "rad_server_get_tile": (ctypes.c_int, [_vp, ctypes.POINTER(Tile)]),
    "rad_server_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "rad_server_profile_read": (ctypes.c_int, [_vp, ctypes.POINTER(ProfileStats)]),
    "rad_server_destroy": (ctypes.c_int, [_vp]),
    "rad_tracked_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(GridDesc), ctypes.c_int64]),
    "rad_tracked_destroy": (ctypes.c_int, [_vp]),
    "rad_tracked_reset": (ctypes.c_int, [_vp, _vp]),
    "rad_tracked_push_step": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.POINTER(Particles), _vp]),
    "rad_tracked_push_steps": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_int32, ctypes.POINTER(Particles), _vp]),
    "rad_tracked_step_group": (ctypes.c_int, []),
    "rad_tracked_spectrum": (ctypes.c_int, [_vp, _dp, ctypes.c_int32, ctypes.c_double, _dp, _vp]),
    "rad_debug_trig_probe": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp]),
}

_lib = None


def lib():
    """Load librad.so from the package directory.  There is no fallback: the library
    must have been built (`python -c "import __graft_entry__ as g; g.build()"`)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != RAD_OK:
        msg = lib().rad_last_error()
        raise RadError(rc, msg.decode() if msg else "")
