"""Seeded synthetic inputs for the charge-transport hot path.

This module only draws initial carrier positions and names the device
settings of each workload; it holds none of the method's arithmetic, so both
the GPU path and the CPU oracle can take their inputs from it.

The paper's own workloads (an X-ray charge cloud, Sec. V.A, and a GEANT4 muon
track, Sec. V.B) are not available, so these generators stand in for them with
the shapes the paper describes: a 3D Gaussian cloud of holes and a straight
track through the full 675 um thickness.

Units: um for lengths, ps for the time step, V/cm for fields.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

# Device and run settings shared by every workload (Sec. III.B user inputs).
DEVICE = dict(
    thickness_um=675.0,
    a1=2000.0 / 675.0,       # Eq. (1): 200 V/cm at z = 675 um, 2200 V/cm at z = 0
    a2=2200.0,
    z_well_um=0.0,
    temperature_K=140.0,
    eps_r=11.7,
    softening_um=1e-3,
    coulomb=1,
    diffusion=1,
    mobility_model=0,
    collected_are_sources=1,
    seed=1,
    event=0,
)
DT_PS = 10.0
PITCH_UM = 15.0


@dataclass
class Workload:
    name: str
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    nx: int = 64
    ny: int = 64
    pitch_um: float = PITCH_UM
    dt_ps: float = DT_PS
    device: dict = field(default_factory=lambda: dict(DEVICE))

    @property
    def n(self) -> int:
        return int(self.x.size)


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, stream])))


def gaussian_cloud(n: int, sigma_um: float, center, seed: int, stream: int = 0):
    """n points from an isotropic 3D Gaussian of width sigma around center."""
    g = _rng(seed, stream)
    pts = g.normal(0.0, sigma_um, size=(3, n))
    return (pts[0] + center[0], pts[1] + center[1], pts[2] + center[2])


def cloud_sigma(n: int) -> float:
    """Cloud width that keeps the central hole density the same for every n:
    0.5 um at 1000 holes, growing as n^(1/3)."""
    return 0.5 * (n / 1000.0) ** (1.0 / 3.0)


def x_ray_cloud(seed: int = 1) -> Workload:
    """1000 holes, sigma 0.5 um, centred at 300 um depth under the corner of
    four pixels of a 64x64 grid of 15 um pixels."""
    x, y, z = gaussian_cloud(1000, 0.5, (480.0, 480.0, 300.0), seed)
    return Workload("cloud_n1000_d300", x, y, z)


def single_cloud(n: int, seed: int = 1, depth_um: float | None = None) -> Workload:
    """One Gaussian cloud of n holes; depth uniform in [50, 650] um unless
    given.  Same device and 64x64 grid as the 1000-hole cloud."""
    g = _rng(seed, 1)
    d = float(g.uniform(50.0, 650.0)) if depth_um is None else float(depth_um)
    x, y, z = gaussian_cloud(n, cloud_sigma(n), (480.0, 480.0, d), seed, stream=2)
    return Workload(f"cloud_n{n}_d{d:.1f}", x, y, z)


def muon_track(seed: int = 1, zenith_deg: float = 30.0, holes_per_um: float = 80.0,
               radial_sigma_um: float = 0.3) -> Workload:
    """Straight track through the full thickness: entry point on the back
    surface uniform over the central 64x64 pixels of a 256x256 grid, azimuth
    uniform, holes uniform along the path with a Gaussian radial spread."""
    g = _rng(seed, 3)
    thick = DEVICE["thickness_um"]
    th = math.radians(zenith_deg)
    phi = float(g.uniform(0.0, 2.0 * math.pi))
    length = thick / math.cos(th)
    n = int(round(holes_per_um * length))
    x0 = float(g.uniform(96 * PITCH_UM, 160 * PITCH_UM))
    y0 = float(g.uniform(96 * PITCH_UM, 160 * PITCH_UM))
    d = np.array([math.sin(th) * math.cos(phi), math.sin(th) * math.sin(phi), -math.cos(th)])
    u = np.array([-math.sin(phi), math.cos(phi), 0.0])
    w = np.cross(d, u)
    t = g.uniform(0.0, length, size=n)
    off = g.normal(0.0, radial_sigma_um, size=(2, n))
    pts = (np.array([x0, y0, thick])[:, None] + d[:, None] * t[None, :]
           + u[:, None] * off[0][None, :] + w[:, None] * off[1][None, :])
    return Workload(f"track_n{n}_zen{zenith_deg:g}", pts[0].copy(), pts[1].copy(),
                    pts[2].copy(), nx=256, ny=256)


def batch_of_clouds(n_events: int = 4096, seed: int = 1, n_min: int = 200,
                    n_max: int = 20000):
    """Independent clouds with hole counts log-uniform in [n_min, n_max] and
    depths uniform over the thickness; widths as in single_cloud."""
    g = _rng(seed, 4)
    counts = np.exp(g.uniform(math.log(n_min), math.log(n_max), size=n_events))
    counts = np.rint(counts).astype(np.int64)
    depths = g.uniform(0.0, DEVICE["thickness_um"], size=n_events)
    events = []
    for e in range(n_events):
        x, y, z = gaussian_cloud(int(counts[e]), cloud_sigma(int(counts[e])),
                                 (480.0, 480.0, float(depths[e])), seed, stream=1000 + e)
        events.append((x, y, z))
    return events
