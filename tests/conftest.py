import math
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds")


@pytest.fixture(scope="session")
def orc():
    import oracle
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()
    return oracle


@pytest.fixture(scope="session")
def step_bound(orc):
    """Displacement (um) per V/cm of field error in one step, from Eqs. (1)-(4).

    Drift: v = mu(|E|) E has a Jacobian no larger than mu(0) (the velocity
    rises monotonically with |E|), so drift moves by at most mu(0) dt per
    V/cm.  Diffusion: sigma ~ sqrt(mu), so a field error dE changes the
    displacement sigma g by sigma |g| |mu'| dE / (2 mu); |g| is at most 6.7
    for normals drawn from 32-bit uniforms (sqrt(-2 ln 2^-32)), and the
    largest |mu'|/mu is taken on a fine grid of |E| with a margin of 2."""
    import numpy as np

    def bound(d, dt_ps):
        T, dt = d["temperature_K"], dt_ps * 1e-12
        mu0 = orc.mobility(0.0, T, d["mobility_model"])
        E = np.linspace(1.0, 2e5, 20001)
        mu = np.array([orc.mobility(e, T, d["mobility_model"]) for e in E])
        slope = 2.0 * float(np.max(np.abs(np.diff(mu) / np.diff(E)) / mu[1:]))
        sigma0 = math.sqrt(2.0 * orc.thermal_voltage(T) * mu0 * dt) * 1e4
        return mu0 * dt * 1e4 + sigma0 * 6.7 * slope / 2.0
    return bound
