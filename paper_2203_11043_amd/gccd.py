"""ctypes binding of libgccd.so (include/gccd.h), same names as the C ABI.

Argument marshalling only: every step of the hot path runs in the HIP
library.  PyTorch supplies device memory (tensors) and the HIP stream.  If the
library is missing this module raises at import; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, fields

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# GCCD_LIB selects another build of the same library (the tests point it at the
# host-sanitized variant)
LIB_PATH = os.environ.get("GCCD_LIB") or os.path.join(_HERE, "libgccd.so")
ABI_VERSION = 4
CLOSURE_WEIGHTS = 290784      # GCCD_CLOSURE_WEIGHTS
GCCD_NOALLOC_MAX_CARRIERS = 32768   # largest load of gccd_field_noalloc

GCCD_OK = 0
GCCD_E_INVALID = -1
GCCD_E_STATE = -2
GCCD_E_DEVICE = -3
GCCD_E_NOMEM = -4
GCCD_E_NONFINITE = -5

# arithmetic of the Eq. (6) kernel (gccd_set_precision)
GCCD_PRECISION_DEFAULT = 0
GCCD_PRECISION_BLOCK = 1
GCCD_PRECISION_EVENT = 2
GCCD_PRECISION_ABSOLUTE = 3
GCCD_PRECISION_COMPENSATED = 4
GCCD_PRECISION_FP64 = 5
PRECISION_MODES = {"default": 0, "block": 1, "event": 2, "absolute": 3, "compensated": 4,
                   "fp64": 5}
SCHEDULES = {"grid": 0, "queue": 1, "graph": 2}   # GCCD_SCHEDULE_*

# every symbol the header declares
EXPORTS = ("gccd_init", "gccd_load", "gccd_load_events", "gccd_run", "gccd_image",
           "gccd_image_events", "gccd_field", "gccd_positions", "gccd_stats",
           "gccd_set_launch", "gccd_autotune", "gccd_set_precision", "gccd_set_closure",
           "gccd_closure_parts", "gccd_set_timing", "gccd_set_schedule", "gccd_field_noalloc",
           "gccd_set_tile",
           "gccd_strerror", "gccd_last_error", "gccd_destroy")


class CParams(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32),
        ("reserved0", ctypes.c_uint32),
        ("thickness_um", ctypes.c_double),
        ("a1_Vcm_per_um", ctypes.c_double),
        ("a2_Vcm", ctypes.c_double),
        ("well_z_um", ctypes.c_double),
        ("temperature_K", ctypes.c_double),
        ("eps_r", ctypes.c_double),
        ("softening_um", ctypes.c_double),
        ("coulomb", ctypes.c_int32),
        ("diffusion", ctypes.c_int32),
        ("mobility_model", ctypes.c_int32),
        ("collected_are_sources", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("event", ctypes.c_uint32),
        ("reserved1", ctypes.c_uint32),
    ]


class CStats(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64),
        ("n_carriers", ctypes.c_int64),
        ("n_active", ctypes.c_int64),
        ("carrier_steps", ctypes.c_uint64),
        ("pair_interactions", ctypes.c_uint64),
        ("field_ms", ctypes.c_double),
        ("field_launches", ctypes.c_int64),
        ("targets_per_thread", ctypes.c_int32),
        ("source_chunks", ctypes.c_int32),
        ("n_events", ctypes.c_int64),
        ("max_source_chunks", ctypes.c_int64),
        ("closure_steps", ctypes.c_int64),
        ("near_chunks", ctypes.c_int64),
        ("graph_replays", ctypes.c_int64),
        ("schedule", ctypes.c_int32),
        ("graph_usable", ctypes.c_int32),
        ("tile_sources", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.gccd_init.argtypes = [ctypes.POINTER(CParams), P, ctypes.POINTER(P)]
    L.gccd_load.argtypes = [P, i64, P, P, P]
    L.gccd_load_events.argtypes = [P, i32, P, P, P, P]
    L.gccd_image_events.argtypes = [P, d, d, d, i32, i32, P, P]
    L.gccd_run.argtypes = [P, d, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.gccd_image.argtypes = [P, d, d, d, i32, i32, P, P]
    L.gccd_field.argtypes = [P, P, P, P]
    L.gccd_positions.argtypes = [P, P, P, P, P]
    L.gccd_stats.argtypes = [P, ctypes.POINTER(CStats)]
    L.gccd_set_launch.argtypes = [P, i32, i32]
    L.gccd_set_tile.argtypes = [P, i32]
    L.gccd_set_precision.argtypes = [P, i32]
    L.gccd_autotune.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                ctypes.POINTER(d)]
    L.gccd_set_closure.argtypes = [P, P, i64, i64]
    L.gccd_closure_parts.argtypes = [P, P, P, P, P, P, P, P, P]
    L.gccd_set_timing.argtypes = [P, i32]
    L.gccd_set_schedule.argtypes = [P, i32]
    L.gccd_field_noalloc.argtypes = [ctypes.POINTER(CParams), i64, P, P, P, P, P, P, P]
    L.gccd_strerror.argtypes = [ctypes.c_int]
    L.gccd_strerror.restype = ctypes.c_char_p
    L.gccd_last_error.argtypes = [P]
    L.gccd_last_error.restype = ctypes.c_char_p
    L.gccd_destroy.argtypes = [P]
    L.gccd_destroy.restype = None
    for name in EXPORTS:
        if name not in ("gccd_strerror", "gccd_last_error", "gccd_destroy"):
            getattr(L, name).restype = ctypes.c_int
    return L


lib = _load()


class GccdError(RuntimeError):
    def __init__(self, status: int, detail: str = ""):
        self.status = status
        msg = lib.gccd_strerror(status).decode()
        super().__init__(f"{msg} ({status})" + (f": {detail}" if detail else ""))


@dataclass
class Params:
    """Mirror of gccd_params with the defaults of the 675 um, 140 K device."""
    thickness_um: float = 675.0
    a1_Vcm_per_um: float = 2000.0 / 675.0
    a2_Vcm: float = 2200.0
    well_z_um: float = 0.0
    temperature_K: float = 140.0
    eps_r: float = 11.7
    softening_um: float = 1e-3
    coulomb: int = 1
    diffusion: int = 1
    mobility_model: int = 0
    collected_are_sources: int = 1
    seed: int = 1
    event: int = 0

    @classmethod
    def from_device(cls, dev: dict) -> "Params":
        """From the device dictionary of paper_2203_11043_amd.workloads."""
        m = dict(thickness_um=dev["thickness_um"], a1_Vcm_per_um=dev["a1"],
                 a2_Vcm=dev["a2"], well_z_um=dev["z_well_um"],
                 temperature_K=dev["temperature_K"], eps_r=dev["eps_r"],
                 softening_um=dev["softening_um"])
        for k in ("coulomb", "diffusion", "mobility_model", "collected_are_sources",
                  "seed", "event"):
            m[k] = dev[k]
        return cls(**m)

    def c(self) -> CParams:
        p = CParams()
        p.abi_version = ABI_VERSION
        for f in fields(self):
            setattr(p, f.name, getattr(self, f.name))
        return p


def _check(ctx, status: int):
    if status != GCCD_OK:
        detail = lib.gccd_last_error(ctx).decode() if ctx else ""
        raise GccdError(status, detail)


def _f64_dev(t: torch.Tensor, n: int) -> int:
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == n):
        raise ValueError("expected a contiguous float64 device tensor of n elements")
    return t.data_ptr()


def gccd_init(params: Params | CParams, stream=None) -> int:
    """Returns an opaque context handle (int)."""
    cp = params.c() if isinstance(params, Params) else params
    if stream is None and torch.cuda.is_available():
        stream = torch.cuda.current_stream()
    handle = stream.cuda_stream if stream is not None else None
    out = ctypes.c_void_p()
    _check(None, lib.gccd_init(ctypes.byref(cp), handle, ctypes.byref(out)))
    return out.value


def gccd_load(ctx: int, x: torch.Tensor, y: torch.Tensor, z: torch.Tensor) -> None:
    n = x.numel()
    _check(ctx, lib.gccd_load(ctx, n, _f64_dev(x, n), _f64_dev(y, n), _f64_dev(z, n)))


def gccd_load_events(ctx: int, offsets, x: torch.Tensor, y: torch.Tensor,
                     z: torch.Tensor) -> None:
    """offsets: n_events + 1 carrier offsets (host sequence); event e holds
    carriers [offsets[e], offsets[e+1]) of the device arrays x, y, z."""
    off = (ctypes.c_int64 * len(offsets))(*[int(v) for v in offsets])
    n = int(offsets[-1])
    _check(ctx, lib.gccd_load_events(ctx, len(offsets) - 1, off, _f64_dev(x, n),
                                     _f64_dev(y, n), _f64_dev(z, n)))


def gccd_run(ctx: int, dt_ps: float, max_steps: int):
    """Returns (steps_done, n_active)."""
    done, na = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(ctx, lib.gccd_run(ctx, float(dt_ps), int(max_steps), ctypes.byref(done),
                             ctypes.byref(na)))
    return done.value, na.value


def gccd_image(ctx: int, x0_um: float, y0_um: float, pitch_um: float, nx: int, ny: int,
               counts: torch.Tensor | None = None, n_outside: torch.Tensor | None = None):
    """Returns (counts[ny, nx] uint32 device tensor, n_outside uint64 device tensor)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    if counts is None:
        counts = torch.empty((ny, nx), dtype=torch.uint32, device=dev)
    if n_outside is None:
        n_outside = torch.empty(1, dtype=torch.uint64, device=dev)
    if counts.numel() != nx * ny or counts.dtype != torch.uint32 or not counts.is_contiguous():
        raise ValueError("counts must be a contiguous uint32 tensor of ny*nx elements")
    _check(ctx, lib.gccd_image(ctx, float(x0_um), float(y0_um), float(pitch_um), int(nx),
                               int(ny), counts.data_ptr(), n_outside.data_ptr()))
    return counts, n_outside


def gccd_image_events(ctx: int, n_events: int, x0_um: float, y0_um: float, pitch_um: float,
                      nx: int, ny: int):
    """Returns (counts[n_events, ny, nx] uint32, n_outside[n_events] uint64) device tensors."""
    dev = torch.device("cuda", torch.cuda.current_device())
    counts = torch.empty((n_events, ny, nx), dtype=torch.uint32, device=dev)
    n_outside = torch.empty(n_events, dtype=torch.uint64, device=dev)
    _check(ctx, lib.gccd_image_events(ctx, float(x0_um), float(y0_um), float(pitch_um), int(nx),
                                      int(ny), counts.data_ptr(), n_outside.data_ptr()))
    return counts, n_outside


def gccd_field(ctx: int, n: int, out=None):
    """Eq. (6) at every carrier; returns a (3, n) float64 device tensor (V/cm)."""
    if out is None:
        out = torch.empty((3, n), dtype=torch.float64,
                          device=torch.device("cuda", torch.cuda.current_device()))
    _check(ctx, lib.gccd_field(ctx, out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr()))
    return out


def gccd_field_noalloc(params, x: torch.Tensor, y: torch.Tensor, z: torch.Tensor, out=None,
                       stream=None):
    """Eq. (6) at n holes of one event without any device allocation by the
    library; returns a (3, n) float64 device tensor (V/cm).  `out` (3, n)
    float64 on the device may be given so that the call allocates nothing."""
    n = int(x.numel())
    cp = params.c() if isinstance(params, Params) else params
    if out is None:
        out = torch.empty((3, n), dtype=torch.float64, device=x.device)
    if stream is None:
        stream = torch.cuda.current_stream()
    st = stream.cuda_stream
    _check(None, lib.gccd_field_noalloc(ctypes.byref(cp), n, _f64_dev(x, n), _f64_dev(y, n),
                                        _f64_dev(z, n), out[0].data_ptr(), out[1].data_ptr(),
                                        out[2].data_ptr(), st))
    return out


def gccd_set_closure(ctx: int, weights, min_carriers: int = 0) -> None:
    """weights: GCCD_CLOSURE_WEIGHTS floats (any array-like) or None to disable."""
    if weights is None:
        _check(ctx, lib.gccd_set_closure(ctx, None, 0, 0))
        return
    import numpy as np
    w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).ravel())
    _check(ctx, lib.gccd_set_closure(ctx, w.ctypes.data_as(ctypes.c_void_p), int(w.size),
                                     int(min_carriers)))


def gccd_closure_parts(ctx: int, n: int):
    """Returns (near (3, n) float64, far (3, n) float64, rho (32, 32, 32) float32,
    grid (4,) float64: node-0 position and spacing) as device tensors."""
    dev = torch.device("cuda", torch.cuda.current_device())
    near = torch.empty((3, n), dtype=torch.float64, device=dev)
    far = torch.empty((3, n), dtype=torch.float64, device=dev)
    rho = torch.empty((32, 32, 32), dtype=torch.float32, device=dev)
    grid = torch.empty(4, dtype=torch.float64, device=dev)
    _check(ctx, lib.gccd_closure_parts(ctx, near[0].data_ptr(), near[1].data_ptr(),
                                       near[2].data_ptr(), far[0].data_ptr(), far[1].data_ptr(),
                                       far[2].data_ptr(), rho.data_ptr(), grid.data_ptr()))
    return near, far, rho, grid


def gccd_positions(ctx: int, n: int):
    """Returns (pos (3, n) float64, collect_step (n,) int32) device tensors."""
    dev = torch.device("cuda", torch.cuda.current_device())
    pos = torch.empty((3, n), dtype=torch.float64, device=dev)
    cs = torch.empty(n, dtype=torch.int32, device=dev)
    _check(ctx, lib.gccd_positions(ctx, pos[0].data_ptr(), pos[1].data_ptr(),
                                   pos[2].data_ptr(), cs.data_ptr()))
    return pos, cs


def gccd_stats(ctx: int) -> dict:
    s = CStats()
    _check(ctx, lib.gccd_stats(ctx, ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in CStats._fields_}


def gccd_set_launch(ctx: int, targets_per_thread: int = 0, source_chunks: int = 0) -> None:
    _check(ctx, lib.gccd_set_launch(ctx, int(targets_per_thread), int(source_chunks)))


def gccd_set_tile(ctx: int, sources: int = 0) -> None:
    """Sources per staged tile of the Eq. (6) work split: 64, 128, 256 or 0
    (automatic)."""
    _check(ctx, lib.gccd_set_tile(ctx, int(sources)))


def gccd_autotune(ctx: int):
    """Returns (targets_per_thread, source_chunks, ms_per_launch) of the
    fastest measured launch shape, which the context keeps."""
    t, s, ms = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_double(0.0)
    _check(ctx, lib.gccd_autotune(ctx, ctypes.byref(t), ctypes.byref(s), ctypes.byref(ms)))
    return t.value, s.value, ms.value


def gccd_set_schedule(ctx: int, mode) -> None:
    """mode: a GCCD_SCHEDULE_* value or its name ("grid", "queue", "graph")."""
    m = SCHEDULES[mode] if isinstance(mode, str) else int(mode)
    _check(ctx, lib.gccd_set_schedule(ctx, m))


def gccd_set_precision(ctx: int, mode) -> None:
    """mode: a GCCD_PRECISION_* value or its name ("default", "fp64", ...)."""
    m = PRECISION_MODES[mode] if isinstance(mode, str) else int(mode)
    _check(ctx, lib.gccd_set_precision(ctx, m))


def gccd_set_timing(ctx: int, on: bool) -> None:
    _check(ctx, lib.gccd_set_timing(ctx, 1 if on else 0))


def gccd_destroy(ctx: int) -> None:
    if ctx:
        lib.gccd_destroy(ctx)


class Simulation:
    """Owns one context; thin convenience over the functions above."""

    def __init__(self, params: Params, x, y, z, stream=None):
        self.ctx = gccd_init(params, stream)
        dev = torch.device("cuda", torch.cuda.current_device())
        self.n = int(len(x))
        t = [torch.as_tensor(v, dtype=torch.float64).to(dev).contiguous() for v in (x, y, z)]
        gccd_load(self.ctx, *t)

    def run(self, dt_ps: float, max_steps: int):
        return gccd_run(self.ctx, dt_ps, max_steps)

    def field(self):
        return gccd_field(self.ctx, self.n)

    def positions(self):
        return gccd_positions(self.ctx, self.n)

    def image(self, x0_um, y0_um, pitch_um, nx, ny):
        return gccd_image(self.ctx, x0_um, y0_um, pitch_um, nx, ny)

    def stats(self):
        return gccd_stats(self.ctx)

    def close(self):
        gccd_destroy(self.ctx)
        self.ctx = None

    def __del__(self):
        if getattr(self, "ctx", None):
            self.close()
