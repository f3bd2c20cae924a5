"""MI355X-native in-situ radiation spectra of PIC macro-particles with form factors.

Python binding of librad.so (C ABI in include/rad.h); it only marshals arguments.  Every
step of the computation runs in the library's HIP kernels.  torch supplies device buffers
(`tensor.data_ptr()`) and streams (`torch.cuda.Stream.cuda_stream`).

    g = Grid(dirs, omega0, domega, n_omega, shape="cic", shape_len=1e-7, dt=5e-17)
    g.push_step(t, particles)          # dict of equal-length CUDA tensors x..dbz, w
    I = g.spectrum()                   # (n_dir, n_omega) float64, J s / sr

Equation references are to Pausch et al., arXiv:1802.03972: the sum is Eq. 13, the
amplitude and phase Eq. 1, the form factor Eqs. 11-12, the shapes Table 1.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (RadError, SHAPES, PHASE_F64, ALL_F32, F32, F64, RAD_ERR_BAD_DATA,
                   RAD_ERR_INVALID_ARG)

FIELDS = ("x", "y", "z", "bx", "by", "bz", "dbx", "dby", "dbz", "w")


def _stream_handle(stream, device: int):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _in_use_on(tensors, stream) -> None:
    """Tell torch's caching allocator that `tensors` are read by work queued on `stream`
    (when that is not the stream they were allocated on), so their memory is not handed out
    again before that work has run."""
    import torch
    if isinstance(stream, torch.cuda.Stream):
        for t in tensors:
            t.record_stream(stream)


def make_particles(fields: dict, expect_len: int | None = None, device: int | None = None):
    """Validate a dict of CUDA tensors and return (rad_particles, n, keepalive)."""
    import torch
    ts = [fields[k] for k in FIELDS]
    dt = ts[0].dtype
    if dt not in (torch.float32, torch.float64):
        raise TypeError(f"particle dtype must be float32 or float64, got {dt}")
    n = ts[0].numel()
    for k, t in zip(FIELDS, ts):
        if not t.is_cuda:
            raise TypeError(f"particle field {k} must be a CUDA tensor")
        if t.dtype != dt:
            raise TypeError(f"particle field {k} has dtype {t.dtype}, expected {dt}")
        if not t.is_contiguous():
            raise ValueError(f"particle field {k} must be contiguous")
        if t.numel() != n:
            raise ValueError(f"particle field {k} has {t.numel()} elements, expected {n}")
        if device is not None and t.device.index != device:
            raise ValueError(f"particle field {k} is on device {t.device.index}, grid is on {device}")
    if expect_len is not None and n != expect_len:
        raise ValueError(f"particle arrays hold {n} elements, expected {expect_len}")
    p = _lib.Particles(F32 if dt == torch.float32 else F64, *[t.data_ptr() for t in ts])
    return p, n, ts


class Grid:
    """One observation grid with its device-resident accumulated spectrum."""

    def __init__(self, dirs, omega0: float, domega: float, n_omega: int, shape="cic",
                 shape_len: float = 1e-7, dt: float = 5e-17, precision: int = PHASE_F64,
                 device: int = 0, tile="auto", omegas=None):
        """omegas: optional explicit frequency list (any spacing); then omega0/domega are
        ignored and n_omega is its length.
        tile: "auto" applies the autotuner's table entry for this grid shape if present
        (else the library's heuristic), None keeps the heuristic, or a dict of launch-shape
        fields (w_per_lane, dir_per_wave, waves, wg_per_cu)."""
        L = _lib.lib()
        self._dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
        self.n_dir = int(self._dirs.shape[0])
        self._omegas = None if omegas is None else np.ascontiguousarray(omegas, np.float64).reshape(-1)
        if self._omegas is not None:
            n_omega = self._omegas.size
        self.n_omega = int(n_omega)
        self.device = int(device)
        self.dt = float(dt)
        self.precision = int(precision)
        self.omega0, self.domega = float(omega0), float(domega)
        sid = SHAPES[shape] if isinstance(shape, str) else int(shape)
        desc = _lib.GridDesc(self.n_dir, self._dirs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             self.omega0, self.domega, self.n_omega, sid, float(shape_len),
                             self.dt, int(precision), self.device,
                             None if self._omegas is None else
                             self._omegas.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        h = ctypes.c_void_p()
        _lib.check(L.rad_create_grid(ctypes.byref(h), ctypes.byref(desc)))
        self._h = h
        v = L.rad_grid_variant(h)
        _lib.check(min(v, 0))
        self.variant = int(v)       # kernel variant bits chosen by the library
        if tile == "auto":
            from .autotune import lookup
            t = lookup(self.n_dir, self.n_omega, int(precision), variant=self.variant)
            if t is not None:
                self.set_tile(**t)
        elif isinstance(tile, dict):
            self.set_tile(**tile)

    # ------------------------------------------------------------------ lifetime
    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(_lib.lib().rad_destroy_grid(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    # ------------------------------------------------------------------ accumulate
    def push_step(self, t: float, particles: dict, stream=None) -> None:
        p, n, keep = make_particles(particles, device=self.device)
        _lib.check(_lib.lib().rad_push_step(self._h, float(t), n, ctypes.byref(p),
                                            _stream_handle(stream, self.device)))
        _in_use_on(keep, stream)

    def push_step_noalloc(self, t: float, particles: dict, stream=None) -> None:
        """rad_push_step_noalloc: the same push without any device allocation (partial sums
        in the library's fixed per-GPU scratch; calls on one GPU must not overlap)."""
        p, n, keep = make_particles(particles, device=self.device)
        _lib.check(_lib.lib().rad_push_step_noalloc(self._h, float(t), n, ctypes.byref(p),
                                                    _stream_handle(stream, self.device)))
        _in_use_on(keep, stream)

    def push_steps(self, t0: float, n_steps: int, particles: dict, stream=None) -> None:
        p, n, keep = make_particles(particles, device=self.device)
        if n_steps <= 0 or n % n_steps:
            raise ValueError("particle arrays must hold n_steps * n_particles elements")
        _lib.check(_lib.lib().rad_push_steps(self._h, float(t0), int(n_steps), n // n_steps,
                                             ctypes.byref(p), _stream_handle(stream, self.device)))
        _in_use_on(keep, stream)

    def reset(self, stream=None) -> None:
        _lib.check(_lib.lib().rad_reset(self._h, _stream_handle(stream, self.device)))

    # ------------------------------------------------------------------ read-out
    def spectrum(self, stream=None) -> np.ndarray:
        out = np.empty((self.n_dir, self.n_omega), np.float64)
        _lib.check(_lib.lib().rad_spectrum(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           _stream_handle(stream, self.device)))
        return out

    def spectrum_device(self, out, stream=None):
        """Write the spectrum into a CUDA float64 tensor of n_dir * n_omega elements."""
        import torch
        if out.dtype != torch.float64 or not out.is_cuda or out.numel() != self.n_dir * self.n_omega \
                or not out.is_contiguous():
            raise ValueError("out must be a contiguous CUDA float64 tensor of n_dir*n_omega elements")
        _lib.check(_lib.lib().rad_spectrum_device(self._h, ctypes.c_void_p(out.data_ptr()),
                                                  _stream_handle(stream, self.device)))
        return out

    def spectrum_complex(self, stream=None) -> np.ndarray:
        out = np.empty((self.n_dir, self.n_omega, 3, 2), np.float64)
        _lib.check(_lib.lib().rad_spectrum_complex(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                   _stream_handle(stream, self.device)))
        return out[..., 0] + 1j * out[..., 1]

    # ------------------------------------------------------------------ state
    def state_size(self) -> int:
        return int(_lib.lib().rad_state_size(self._h))

    def get_state(self, stream=None) -> np.ndarray:
        out = np.empty(self.state_size(), np.float64)
        _lib.check(_lib.lib().rad_get_state(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            _stream_handle(stream, self.device)))
        return out

    def set_state(self, state: np.ndarray, stream=None) -> None:
        st = np.ascontiguousarray(state, np.float64)
        if st.size != self.state_size():
            raise ValueError(f"state has {st.size} doubles, grid needs {self.state_size()}")
        _lib.check(_lib.lib().rad_set_state(self._h, st.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            _stream_handle(stream, self.device)))

    # ------------------------------------------------------------------ kernel timing
    def profile(self, enable=True) -> None:
        """True (or 1): time every accumulate launch; an integer k > 1: every k-th one;
        False / 0: stop timing."""
        k = int(enable) if not isinstance(enable, bool) else (1 if enable else 0)
        _lib.check(_lib.lib().rad_profile_enable(self._h, max(0, k)))

    def profile_read(self) -> dict:
        st = _lib.ProfileStats()
        _lib.check(_lib.lib().rad_profile_read(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _lib.ProfileStats._fields_}

    # ------------------------------------------------------------------ launch shape
    def get_tile(self) -> dict:
        t = _lib.Tile()
        _lib.check(_lib.lib().rad_get_tile(self._h, ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in _lib.Tile._fields_}

    def set_tile(self, **kw) -> None:
        cur = self.get_tile()
        cur.update(kw)
        t = _lib.Tile(*[int(cur[k]) for k, _ in _lib.Tile._fields_])
        _lib.check(_lib.lib().rad_set_tile(self._h, ctypes.byref(t)))


class Batcher:
    """Accumulates many (grid, steps, particles) items with one persistent launch."""

    def __init__(self, device: int = 0, max_items: int = 256, graph: bool = False, tile="auto"):
        """tile: "auto" applies the autotuner's batched-kernel entry for the first pushed
        grid's shape (if any), None keeps the library default, or a dict of the four fields."""
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().rad_batcher_create(ctypes.byref(h), int(device), int(max_items)))
        self._h = h
        self.device = int(device)
        self.max_items = int(max_items)
        self._auto = tile == "auto"
        if isinstance(tile, dict):
            self.set_tile(**tile)
        if graph:
            _lib.check(_lib.lib().rad_batcher_set_graph(h, 1))

    def set_tile(self, **kw) -> None:
        """Launch shape of the batched kernel (all four fields), or no arguments to restore
        the default.  An explicit choice replaces a pending tile="auto" lookup."""
        self._auto = False
        if not kw:
            _lib.check(_lib.lib().rad_batcher_set_tile(self._h, None))
            return
        t = _lib.Tile(*[int(kw[k]) for k, _ in _lib.Tile._fields_])
        _lib.check(_lib.lib().rad_batcher_set_tile(self._h, ctypes.byref(t)))

    def get_tile(self):
        """The batcher's launch shape, or None while the library default applies."""
        t = _lib.Tile()
        if _lib.lib().rad_batcher_get_tile(self._h, ctypes.byref(t)) != 0:
            return None
        return {k: getattr(t, k) for k, _ in _lib.Tile._fields_}

    def graph_stats(self) -> dict:
        g, l, f = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _lib.check(_lib.lib().rad_batcher_graph_stats(self._h, ctypes.byref(g), ctypes.byref(l), ctypes.byref(f)))
        return {"graphs": g.value, "launches": l.value, "failures": f.value}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(_lib.lib().rad_batcher_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def push(self, items, stream=None) -> None:
        """items: iterable of (grid, t0, n_steps, particles) with particles a dict of CUDA
        tensors holding n_steps * n_particles elements each (step-major)."""
        items = list(items)
        if self._auto and items:
            from .autotune import lookup_batch
            g0 = items[0][0]
            t = lookup_batch(g0.n_dir, g0.n_omega, g0.precision) if g0.variant == 0 else None
            if t is not None:
                self.set_tile(**t)
            self._auto = False
        arr = (_lib.BatchItem * max(1, len(items)))()
        keep = []
        for k, (grid, t0, n_steps, parts) in enumerate(items):
            p, n, ts = make_particles(parts, device=self.device)
            keep.append(ts)
            if n_steps <= 0 or n % n_steps:
                raise ValueError("particle arrays must hold n_steps * n_particles elements")
            arr[k] = _lib.BatchItem(grid.handle.value, float(t0), int(n_steps), n // n_steps, p)
        _lib.check(_lib.lib().rad_batcher_push(self._h, arr, len(items), _stream_handle(stream, self.device)))
        for ts in keep:
            _in_use_on(ts, stream)

    def profile(self, enable: bool = True) -> None:
        _lib.check(_lib.lib().rad_batcher_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        st = _lib.ProfileStats()
        _lib.check(_lib.lib().rad_batcher_profile_read(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _lib.ProfileStats._fields_}


class Server:
    """Continuous-batching serving loop (scheduler thread in librad.so).

    submit() takes one chunk (one time step of one bunch) as HOST arrays: a dict of numpy
    arrays or CPU tensors (pinned memory lets the copies run asynchronously).  The arrays
    are kept alive here until the chunk completes."""

    def __init__(self, device: int = 0, hbm_budget: int = 1 << 30, max_batch: int = 64,
                 max_inflight: int = 2, max_admitted: int = 256, max_pending: int = 1 << 20,
                 poll_us: int = 20, use_graph: bool = True, tile="auto"):
        """tile: "auto" applies the autotuner's batched-kernel entry for the first submitted
        grid's shape (if any), None keeps the library default, or a dict of the four fields."""
        cfg = _lib.ServerConfig(int(device), int(hbm_budget), int(max_batch), int(max_inflight),
                                int(max_admitted), int(max_pending), int(poll_us), 1 if use_graph else 0)
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().rad_server_create(ctypes.byref(h), ctypes.byref(cfg)))
        self._h = h
        self._keep = {}
        self._auto = tile == "auto"
        if isinstance(tile, dict):
            self.set_tile(**tile)

    def set_tile(self, **kw) -> None:
        """Launch shape of the batched launches (all four fields), or none for the default.
        An explicit choice replaces a pending tile="auto" lookup."""
        self._auto = False
        if not kw:
            _lib.check(_lib.lib().rad_server_set_tile(self._h, None))
            return
        t = _lib.Tile(*[int(kw[k]) for k, _ in _lib.Tile._fields_])
        _lib.check(_lib.lib().rad_server_set_tile(self._h, ctypes.byref(t)))

    def get_tile(self):
        t = _lib.Tile()
        if _lib.lib().rad_server_get_tile(self._h, ctypes.byref(t)) != 0:
            return None
        return {k: getattr(t, k) for k, _ in _lib.Tile._fields_}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(_lib.lib().rad_server_destroy(self._h))
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, grid: "Grid", t: float, host_fields: dict) -> int:
        if self._auto:
            from .autotune import lookup_batch
            tt = lookup_batch(grid.n_dir, grid.n_omega, grid.precision) if grid.variant == 0 else None
            if tt is not None:
                self.set_tile(**tt)
            self._auto = False
        arrs = []
        for k in FIELDS:
            a = host_fields[k]
            if hasattr(a, "is_cuda"):
                if a.is_cuda or not a.is_contiguous():
                    raise ValueError(f"field {k} must be a contiguous CPU tensor")
                ptr, n, dt = a.data_ptr(), a.numel(), str(a.dtype).replace("torch.", "")
            else:
                a = np.ascontiguousarray(a)
                ptr, n, dt = a.ctypes.data, a.size, str(a.dtype)
            arrs.append((a, ptr, n, dt))
        n, dt = arrs[0][2], arrs[0][3]
        if any(x[2] != n or x[3] != dt for x in arrs) or dt not in ("float32", "float64"):
            raise ValueError("all fields must share one length and dtype (float32 or float64)")
        p = _lib.Particles(F32 if dt == "float32" else F64, *[x[1] for x in arrs])
        tk = ctypes.c_uint64()
        _lib.check(_lib.lib().rad_server_submit(self._h, grid.handle, float(t), int(n), ctypes.byref(p),
                                                ctypes.byref(tk)))
        self._keep[tk.value] = arrs
        return tk.value

    @staticmethod
    def _stats(st) -> dict:
        return {k: getattr(st, k) for k, _ in _lib.ChunkStats._fields_}

    def poll(self, ticket: int):
        st = _lib.ChunkStats()
        rc = _lib.lib().rad_server_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(st))
        if rc < 0:
            _lib.check(rc)
        if rc == 0:
            return None
        self._keep.pop(ticket, None)
        return self._stats(st)

    def wait(self, ticket: int) -> dict:
        st = _lib.ChunkStats()
        rc = _lib.lib().rad_server_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(st))
        if rc < 0:
            _lib.check(rc)
        self._keep.pop(ticket, None)
        return self._stats(st)

    def drain(self) -> None:
        _lib.check(_lib.lib().rad_server_drain(self._h))

    def profile(self, enable: bool = True) -> None:
        _lib.check(_lib.lib().rad_server_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self) -> dict:
        st = _lib.ProfileStats()
        _lib.check(_lib.lib().rad_server_profile_read(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _lib.ProfileStats._fields_}

    def counters(self) -> dict:
        c = _lib.ServerCounters()
        _lib.check(_lib.lib().rad_server_counters_read(self._h, ctypes.byref(c)))
        return {k: getattr(c, k) for k, _ in _lib.ServerCounters._fields_}


class Tracked:
    """Post-processing variant for a small set of tracked particles: per-particle time
    integrals on the device, form factor (weights and shape) applied at read-out."""

    def __init__(self, dirs, omega0: float, domega: float, n_omega: int, n_particles: int,
                 dt: float = 5e-17, device: int = 0, omegas=None):
        self._dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
        self._omegas = None if omegas is None else np.ascontiguousarray(omegas, np.float64).reshape(-1)
        if self._omegas is not None:
            n_omega = self._omegas.size
        self.n_dir, self.n_omega, self.n_particles = int(self._dirs.shape[0]), int(n_omega), int(n_particles)
        self.device = int(device)
        desc = _lib.GridDesc(self.n_dir, self._dirs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             float(omega0), float(domega), self.n_omega, 0, 0.0, float(dt), PHASE_F64,
                             self.device, None if self._omegas is None else
                             self._omegas.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().rad_tracked_create(ctypes.byref(h), ctypes.byref(desc), self.n_particles))
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.check(_lib.lib().rad_tracked_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self, stream=None) -> None:
        _lib.check(_lib.lib().rad_tracked_reset(self._h, _stream_handle(stream, self.device)))

    def push_step(self, t: float, particles: dict, stream=None) -> None:
        p, n, keep = make_particles(particles, expect_len=self.n_particles, device=self.device)
        _lib.check(_lib.lib().rad_tracked_push_step(self._h, float(t), ctypes.byref(p),
                                                    _stream_handle(stream, self.device)))
        _in_use_on(keep, stream)

    @staticmethod
    def step_group() -> int:
        """Steps one launch sums in registers per read-modify-write of the integrals."""
        return int(_lib.lib().rad_tracked_step_group())

    def push_steps(self, t0: float, n_steps: int, particles: dict, stream=None) -> None:
        """n_steps steps at t0 + j dt; arrays of n_steps * n_particles elements, step-major."""
        p, n, keep = make_particles(particles, expect_len=int(n_steps) * self.n_particles, device=self.device)
        _lib.check(_lib.lib().rad_tracked_push_steps(self._h, float(t0), int(n_steps), ctypes.byref(p),
                                                     _stream_handle(stream, self.device)))
        _in_use_on(keep, stream)

    def spectrum(self, weights, shape="cic", shape_len: float = 1e-7, stream=None) -> np.ndarray:
        w = np.ascontiguousarray(weights, np.float64).reshape(-1)
        if w.size != self.n_particles:
            raise ValueError(f"need {self.n_particles} weights")
        out = np.empty((self.n_dir, self.n_omega), np.float64)
        sid = SHAPES[shape] if isinstance(shape, str) else int(shape)
        _lib.check(_lib.lib().rad_tracked_spectrum(self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), sid,
                                                   float(shape_len), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                   _stream_handle(stream, self.device)))
        return out


def device_cus(device: int = 0) -> int:
    rc = _lib.lib().rad_device_cus(int(device))
    if rc < 0:
        _lib.check(rc)
    return rc


def trig_probe(revs, stream=None):
    """Hardware and library sin/cos of 2 pi r on the device (diagnostic)."""
    import torch
    x = torch.as_tensor(np.asarray(revs, np.float32), device="cuda").contiguous()
    out = torch.empty(4 * x.numel(), dtype=torch.float32, device="cuda")
    _lib.check(_lib.lib().rad_debug_trig_probe(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                               x.numel(), _stream_handle(stream, x.device.index)))
    torch.cuda.synchronize()
    return out.view(-1, 4).cpu().numpy()
