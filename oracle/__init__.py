"""FP64 CPU oracle for the G-CoReCCD time step -- TEST INFRASTRUCTURE ONLY.

Avalos & Sofo Haro, "G-CoReCCD: a GPU-based simulator of the charge transport
in fully-depleted CCDs" (arXiv 2203.11043).  This package wraps the plain C
reference in ``gccd_oracle.c`` with ctypes.  Only ``tests/``, the smoke check
in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it;
the GPU library never does, and the two share no code.

Functions follow the paper:
  * ``mobility``            -- Eq. (2), hole mobility mu(E, T)
  * ``coulomb_constant``    -- K of Eq. (6), q / (4 pi eps0 eps_r)
  * ``field``               -- Eq. (6), softened all-pairs Coulomb field
  * ``philox4x32_10``/``normals`` -- random diffusion vectors (Sec. III.B)
  * ``prepare``/``run``     -- the per-step sequence of Sec. III.B, Fig. 2
  * ``image``               -- 2D histogram of collected charge (Sec. V.A)
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB lets the mutation test point the pins at a deliberately broken build
LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "_build", "liboracle.so")
SOURCES = [os.path.join(_HERE, "gccd_oracle.c")]


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc: -O2, OpenMP, no FMA contraction, no fast-math."""
    import subprocess

    os.makedirs(os.path.dirname(LIB_PATH), exist_ok=True)
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC",
           "-shared", "-Wall", "-o", tmp] + SOURCES + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [
        ("thickness_um", ctypes.c_double),
        ("a1", ctypes.c_double),
        ("a2", ctypes.c_double),
        ("z_well_um", ctypes.c_double),
        ("temperature_K", ctypes.c_double),
        ("eps_r", ctypes.c_double),
        ("softening_um", ctypes.c_double),
        ("coulomb", ctypes.c_int32),
        ("diffusion", ctypes.c_int32),
        ("mobility_model", ctypes.c_int32),
        ("collected_are_sources", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("event", ctypes.c_uint32),
        ("pad_", ctypes.c_uint32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        d, i64, u32, u64, i32 = (ctypes.c_double, ctypes.c_int64, ctypes.c_uint32,
                                 ctypes.c_uint64, ctypes.c_int32)
        P = ctypes.c_void_p
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_normals.argtypes = [u64, u32, u32, u32, P]
        L.orc_mobility.argtypes = [d, d, i32]
        L.orc_mobility.restype = d
        L.orc_coulomb_constant.argtypes = [d]
        L.orc_coulomb_constant.restype = d
        L.orc_thermal_voltage.argtypes = [d]
        L.orc_thermal_voltage.restype = d
        L.orc_field.argtypes = [i64, P, P, P, i64, P, P, P, d, d, P, P, P, P]
        L.orc_field_window.argtypes = [i64, P, P, P, i64, P, P, P, d, d, d, d, P, P, P]
        L.orc_prepare.argtypes = [P, i64, P, P, P, P]
        L.orc_prepare.restype = i64
        L.orc_run.argtypes = [P, d, i64, P, P, P, P, i64, i64, P, P]
        L.orc_run.restype = ctypes.c_int
        L.orc_image.argtypes = [i64, P, P, P, d, d, d, i32, i32, P, P]
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Device:
    """Physical and numerical settings of one simulated CCD (see Sec. III.B)."""
    thickness_um: float = 675.0
    a1: float = 2000.0 / 675.0
    a2: float = 2200.0
    z_well_um: float = 0.0
    temperature_K: float = 140.0
    eps_r: float = 11.7
    softening_um: float = 1e-3
    coulomb: int = 1
    diffusion: int = 1
    mobility_model: int = 0
    collected_are_sources: int = 1
    seed: int = 1
    event: int = 0

    def c(self) -> Params:
        return Params(self.thickness_um, self.a1, self.a2, self.z_well_um,
                      self.temperature_K, self.eps_r, self.softening_um,
                      int(self.coulomb), int(self.diffusion), int(self.mobility_model),
                      int(self.collected_are_sources), int(self.seed), int(self.event), 0)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def normals(seed: int, j: int, s: int, event: int = 0) -> np.ndarray:
    out = np.zeros(3, dtype=np.float64)
    lib().orc_normals(seed, j, s, event, _ptr(out))
    return out


def mobility(E: float, T: float, model: int = 0) -> float:
    return float(lib().orc_mobility(E, T, model))


def coulomb_constant(eps_r: float) -> float:
    return float(lib().orc_coulomb_constant(eps_r))


def thermal_voltage(T: float) -> float:
    return float(lib().orc_thermal_voltage(T))


def field(targets, sources=None, softening_um: float = 1e-3, eps_r: float = 11.7,
          with_magnitude: bool = False):
    """Eq. (6) at target points (3 x nt array) from source charges (3 x ns).

    Returns (E[3, nt]) or (E, A) where A[j] = K sum_i |r_ij|/(r_ij^2+eps^2)^{3/2}.
    """
    t = [_f64(v) for v in targets]
    s = t if sources is None else [_f64(v) for v in sources]
    nt, ns = t[0].size, s[0].size
    E = np.zeros((3, nt), dtype=np.float64)
    A = np.zeros(nt, dtype=np.float64) if with_magnitude else None
    K = coulomb_constant(eps_r)
    lib().orc_field(nt, _ptr(t[0]), _ptr(t[1]), _ptr(t[2]), ns, _ptr(s[0]), _ptr(s[1]),
                    _ptr(s[2]), softening_um, K,
                    _ptr(E[0]), _ptr(E[1]), _ptr(E[2]),
                    _ptr(A) if A is not None else None)
    return (E, A) if with_magnitude else E


def field_window(targets, sources, r_lo: float, r_hi: float, softening_um: float = 1e-3,
                 eps_r: float = 11.7):
    """Eq. (6) at the targets from the sources at distance r_lo <= r < r_hi."""
    t = [_f64(v) for v in targets]
    s = [_f64(v) for v in sources]
    E = np.zeros((3, t[0].size), dtype=np.float64)
    lib().orc_field_window(t[0].size, _ptr(t[0]), _ptr(t[1]), _ptr(t[2]), s[0].size,
                           _ptr(s[0]), _ptr(s[1]), _ptr(s[2]), softening_um,
                           coulomb_constant(eps_r), float(r_lo), float(r_hi),
                           _ptr(E[0]), _ptr(E[1]), _ptr(E[2]))
    return E


class State:
    """Carrier state: FP64 positions (um) and the step at which each was
    collected (-1 while it is still travelling)."""

    def __init__(self, dev: Device, x, y, z):
        self.dev = dev
        self.x, self.y, self.z = _f64(x).copy(), _f64(y).copy(), _f64(z).copy()
        self.n = self.x.size
        self.cstep = np.zeros(self.n, dtype=np.int32)
        self.step = 0
        self._p = dev.c()
        self.n_active = int(lib().orc_prepare(ctypes.byref(self._p), self.n, _ptr(self.x),
                                              _ptr(self.y), _ptr(self.z), _ptr(self.cstep)))

    def run(self, dt_ps: float, max_steps: int):
        done = ctypes.c_int64(0)
        na = ctypes.c_int64(0)
        rc = lib().orc_run(ctypes.byref(self._p), dt_ps * 1e-12, self.n, _ptr(self.x),
                           _ptr(self.y), _ptr(self.z), _ptr(self.cstep), self.step,
                           int(max_steps), ctypes.byref(done), ctypes.byref(na))
        if rc != 0:
            raise RuntimeError(f"oracle run failed with code {rc}")
        self.step += done.value
        self.n_active = na.value
        return done.value, na.value

    def image(self, x0: float, y0: float, pitch: float, nx: int, ny: int):
        return image(self.x, self.y, self.cstep, x0, y0, pitch, nx, ny)


def image(x, y, cstep, x0: float, y0: float, pitch: float, nx: int, ny: int):
    x, y = _f64(x), _f64(y)
    c = np.ascontiguousarray(cstep, dtype=np.int32)
    counts = np.zeros((ny, nx), dtype=np.uint32)
    out = ctypes.c_uint64(0)
    lib().orc_image(x.size, _ptr(x), _ptr(y), _ptr(c), x0, y0, pitch, nx, ny,
                    _ptr(counts), ctypes.byref(out))
    return counts, int(out.value)
